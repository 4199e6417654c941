"""CPU reference oracle for batched Smith-Waterman / Gotoh alignment.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package; the product path
(``paper_2303_01845_amd``) never does.  It shares no code with the HIP library:
its own C source (``sw_oracle.c``), its own substitution table parsed from
``blosum62.txt``, its own ASCII encoder.

The recurrence, the gap model and the tie rule are stated in the header of
``sw_oracle.c``; candidate discovery (distinct shared k-mers, the overlap
product of the k-mer matrix with itself) in the header of
``discover_oracle.c``; identity and coverage of aligned pairs (the
similarity-graph filter) in the header of ``identity_oracle.c`` (the paper, section "Load balancing techniques": the aligner
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
DISCOVER_SRC = os.path.join(HERE, "discover_oracle.c")
DISCOVER_LIB = os.path.join(HERE, "liboracle_discover.so")
IDENTITY_SRC = os.path.join(HERE, "identity_oracle.c")
IDENTITY_LIB = os.path.join(HERE, "liboracle_identity.so")
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
    for src, lib in ((SRC, LIB), (DISCOVER_SRC, DISCOVER_LIB), (IDENTITY_SRC, IDENTITY_LIB)):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(src):
            compile_oracle(src, lib)
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


class DiscoverLib:
    """ctypes view of one compiled candidate-discovery oracle (the default
    build, or a deliberately altered copy used to show that its pins catch
    mistakes)."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        L.oracle_discover.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                      ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]
        L.oracle_distinct_kmers.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                            ctypes.c_int32, ctypes.c_void_p]
        self.L = L

    def discover_codes(self, q_codes, q_offs, r_codes, r_offs, k: int = 6, min_shared: int = 2,
                       mode: int = 0):
        """(query, reference, shared) int32 arrays of every pair with at least
        ``min_shared`` distinct common k-mers, in (query, reference) order.
        mode 0: all pairs; 1: query < reference; 2: the index-parity rule."""
        qc = np.ascontiguousarray(q_codes, dtype=np.int8)
        rc_ = np.ascontiguousarray(r_codes, dtype=np.int8)
        qo = np.ascontiguousarray(q_offs, dtype=np.int64)
        ro = np.ascontiguousarray(r_offs, dtype=np.int64)
        found = ctypes.c_int64(0)
        args = (qc.ctypes.data, qo.ctypes.data, len(qo) - 1, rc_.ctypes.data, ro.ctypes.data,
                len(ro) - 1, k, min_shared, mode)
        rc = self.L.oracle_discover(*args, 0, None, None, None, ctypes.byref(found))
        if rc != 0:
            raise ValueError("oracle_discover failed (rc=%d)" % rc)
        n = found.value
        out = np.zeros((3, max(n, 1)), dtype=np.int32)
        rc = self.L.oracle_discover(*args, n, out[0].ctypes.data, out[1].ctypes.data,
                                    out[2].ctypes.data, ctypes.byref(found))
        if rc != 0 or found.value != n:
            raise ValueError("oracle_discover failed (rc=%d)" % rc)
        return out[0, :n].copy(), out[1, :n].copy(), out[2, :n].copy()

    def distinct_kmers_codes(self, codes, offs, k: int = 6) -> np.ndarray:
        c = np.ascontiguousarray(codes, dtype=np.int8)
        o = np.ascontiguousarray(offs, dtype=np.int64)
        out = np.zeros(max(len(o) - 1, 1), dtype=np.int64)
        rc = self.L.oracle_distinct_kmers(c.ctypes.data, o.ctypes.data, len(o) - 1, k,
                                          out.ctypes.data)
        if rc != 0:
            raise ValueError("oracle_distinct_kmers failed (rc=%d)" % rc)
        return out[:len(o) - 1]


_discover = None


def discover_lib() -> DiscoverLib:
    global _discover
    with _lock:
        if _discover is None:
            build(force=False)
            _discover = DiscoverLib(DISCOVER_LIB)
    return _discover


def _ascii_codes(ascii) -> np.ndarray:
    if isinstance(ascii, (bytes, bytearray, str)):
        return default().encode(ascii)
    return default().encode(np.ascontiguousarray(ascii, dtype=np.uint8).tobytes())


def discover(q_ascii, q_offs, r_ascii, r_offs, k: int = 6, min_shared: int = 2, mode: int = 0):
    """Candidate pairs of two ASCII sequence sets (see ``DiscoverLib.discover_codes``)."""
    return discover_lib().discover_codes(_ascii_codes(q_ascii), q_offs, _ascii_codes(r_ascii),
                                         r_offs, k, min_shared, mode)


def distinct_kmers(ascii, offs, k: int = 6) -> np.ndarray:
    """Number of distinct k-mers of every sequence."""
    return discover_lib().distinct_kmers_codes(_ascii_codes(ascii), offs, k)


class IdentityLib:
    """ctypes view of one compiled identity oracle (the default build, or a
    deliberately altered copy used to show that its pins catch mistakes)."""

    def __init__(self, path: str):
        L = ctypes.CDLL(path)
        L.oracle_identity_box.argtypes = [ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32,
                                          ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32,
                                          ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                          ctypes.POINTER(ctypes.c_int64)]
        L.oracle_identity_batch.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p]
        self.L = L

    def box(self, q, r, scores, go: int = 11, ge: int = 1):
        """(score, matches, columns) of the best global alignment of two code
        arrays (higher score, then more matches, then fewer columns)."""
        qc = np.ascontiguousarray(q, dtype=np.int8)
        rc_ = np.ascontiguousarray(r, dtype=np.int8)
        sc = np.ascontiguousarray(scores, dtype=np.int8).reshape(-1)
        s, m, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        if self.L.oracle_identity_box(qc.ctypes.data, len(qc), rc_.ctypes.data, len(rc_), sc.ctypes.data, go, ge,
                                      ctypes.byref(s), ctypes.byref(m), ctypes.byref(c)) != 0:
            raise ValueError("oracle_identity_box failed")
        return s.value, m.value, c.value

    def batch(self, codes, offsets, pairs, aligned, scores, go: int = 11, ge: int = 1,
              ani_permille: int = 300, cov_permille: int = 700) -> np.ndarray:
        """int64 [n_pairs, 4]: box score, matches, columns, keep."""
        codes = np.ascontiguousarray(codes, dtype=np.int8)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        pairs = np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)
        aligned = np.ascontiguousarray(aligned, dtype=np.int32).reshape(-1, 5)
        sc = np.ascontiguousarray(scores, dtype=np.int8).reshape(-1)
        out = np.zeros((len(pairs), 4), dtype=np.int64)
        if self.L.oracle_identity_batch(codes.ctypes.data, offsets.ctypes.data, len(offsets) - 1,
                                        pairs.ctypes.data, len(pairs), aligned.ctypes.data, sc.ctypes.data,
                                        go, ge, ani_permille, cov_permille, out.ctypes.data) != 0:
            raise ValueError("oracle_identity_batch failed")
        return out


_identity = None


def identity_lib() -> IdentityLib:
    global _identity
    with _lock:
        if _identity is None:
            build(force=False)
            _identity = IdentityLib(IDENTITY_LIB)
    return _identity


def identity_ascii(ascii, offsets, pairs, aligned, go: int = 11, ge: int = 1, ani_permille: int = 300,
                   cov_permille: int = 700) -> np.ndarray:
    """Identity filter records (see ``IdentityLib.batch``) of aligned pairs of
    an ASCII sequence buffer, encoded with the oracle's own encoder."""
    codes = _ascii_codes(ascii)
    return identity_lib().batch(codes, offsets, pairs, aligned, default().scores, go, ge, ani_permille,
                                cov_permille)
