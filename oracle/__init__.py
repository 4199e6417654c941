"""CPU reference oracle for batched Smith-Waterman / Gotoh alignment.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product path
(``paper_2303_01845_amd``) never does.  It shares no code with the HIP library:
its own C source (``sw_oracle.c``), its own substitution table parsed from
``blosum62.txt``, its own ASCII encoder.

The recurrence, the gap model and the tie rule are stated in the header of
``sw_oracle.c`` (the paper, section "Load balancing techniques": the aligner
fills the entire dynamic-programming matrix; "Performance results", program
parameter table: affine gap open / extension penalties, integer scores).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sw_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
MATRIX_TXT = os.path.join(HERE, "blosum62.txt")


class Result(ctypes.Structure):
    _fields_ = [("score", ctypes.c_int32), ("q_start", ctypes.c_int32),
                ("q_end", ctypes.c_int32), ("r_start", ctypes.c_int32),
                ("r_end", ctypes.c_int32)]


def compile_oracle(src: str, out: str) -> str:
    """Plain ``gcc -O2`` build (no SIMD pragmas, no tuning)."""
    tmp = out + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-pthread",
                           "-o", tmp, src])
    os.replace(tmp, out)
    return out


def build(force: bool = True) -> str:
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        compile_oracle(SRC, LIB)
    return LIB


class OracleLib:
    """ctypes view of one compiled oracle library (the default build, or a
    deliberately altered copy used to show that the pins catch mistakes)."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        L.oracle_matrix_size.restype = ctypes.c_size_t
        L.oracle_matrix_parse.argtypes = [ctypes.c_char_p, ctypes.c_void_p]
        L.oracle_encode.argtypes = [ctypes.c_void_p, ctypes.c_char_p, ctypes.c_int64,
                                    ctypes.c_void_p]
        L.oracle_encode.restype = ctypes.c_int64
        L.oracle_align.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                   ctypes.c_int32, ctypes.POINTER(Result)]
        L.oracle_fill_H.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                                    ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_void_p]
        L.oracle_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                   ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                   ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                   ctypes.c_int]
        self.L = L
        self.path = path
        self._buf = ctypes.create_string_buffer(L.oracle_matrix_size())
        with open(MATRIX_TXT, "rb") as f:
            rc = L.oracle_matrix_parse(f.read(), self._buf)
        if rc != 0:
            raise ValueError("cannot parse substitution matrix (rc=%d)" % rc)
        raw = self._buf.raw
        self.letters = raw[:24].decode("ascii")
        self.scores = np.frombuffer(raw[25:25 + 576], dtype=np.int8).reshape(24, 24).copy()

    @property
    def mx(self):
        return ctypes.addressof(self._buf)

    def encode(self, ascii) -> np.ndarray:
        if isinstance(ascii, str):
            ascii = ascii.encode("ascii")
        ascii = bytes(ascii)
        out = np.empty(len(ascii), dtype=np.int8)
        bad = self.L.oracle_encode(self.mx, ascii, len(ascii), out.ctypes.data)
        if bad:
            raise ValueError("%d residues are not symbols of the matrix" % bad)
        return out

    def _codes(self, x) -> np.ndarray:
        if isinstance(x, (bytes, bytearray, str)):
            return self.encode(x)
        return np.ascontiguousarray(x, dtype=np.int8)

    def align(self, q, r, go: int = 11, ge: int = 1):
        """(score, q_start, q_end, r_start, r_end) for one pair."""
        qc, rc = self._codes(q), self._codes(r)
        res = Result()
        code = self.L.oracle_align(qc.ctypes.data, len(qc), rc.ctypes.data, len(rc), self.mx,
                                   go, ge, ctypes.byref(res))
        if code != 0:
            raise ValueError("oracle_align failed (rc=%d)" % code)
        return (res.score, res.q_start, res.q_end, res.r_start, res.r_end)

    def fill_H(self, q, r, go: int = 11, ge: int = 1) -> np.ndarray:
        qc, rc = self._codes(q), self._codes(r)
        H = np.zeros((len(qc), len(rc)), dtype=np.int32)
        if self.L.oracle_fill_H(qc.ctypes.data, len(qc), rc.ctypes.data, len(rc), self.mx,
                                go, ge, H.ctypes.data) != 0:
            raise ValueError("bad gap parameters")
        return H

    def batch(self, codes, offsets, pairs, go: int = 11, ge: int = 1,
              threads: int | None = None) -> np.ndarray:
        """Align every (query, reference) index pair; int32 [n_pairs, 5] in the
        field order score, q_start, q_end, r_start, r_end."""
        codes = np.ascontiguousarray(codes, dtype=np.int8)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        out = np.zeros((len(pairs), 5), dtype=np.int32)
        if threads is None:
            threads = len(os.sched_getaffinity(0))
        rc = self.L.oracle_batch(codes.ctypes.data, offsets.ctypes.data, len(offsets) - 1,
                                 pairs.ctypes.data, len(pairs), self.mx, go, ge,
                                 out.ctypes.data, int(threads))
        if rc != 0:
            raise ValueError("oracle_batch failed (rc=%d)" % rc)
        return out


_lock = threading.Lock()
_default = None


def default() -> OracleLib:
    global _default
    with _lock:
        if _default is None:
            build(force=False)
            _default = OracleLib(LIB)
    return _default


def matrix() -> np.ndarray:
    return default().scores


def encode(ascii) -> np.ndarray:
    return default().encode(ascii)


def align(q, r, go: int = 11, ge: int = 1):
    return default().align(q, r, go, ge)


def fill_H(q, r, go: int = 11, ge: int = 1) -> np.ndarray:
    return default().fill_H(q, r, go, ge)


def batch(codes, offsets, pairs, go: int = 11, ge: int = 1, threads: int | None = None):
    return default().batch(codes, offsets, pairs, go, ge, threads)


def batch_ascii(ascii: np.ndarray, offsets, pairs, go: int = 11, ge: int = 1,
                threads: int | None = None) -> np.ndarray:
    """Encode a concatenated ASCII buffer with the oracle's own encoder, then
    align.  Residues that are not matrix symbols raise."""
    codes = default().encode(np.ascontiguousarray(ascii, dtype=np.uint8).tobytes())
    return default().batch(codes, offsets, pairs, go, ge, threads)
