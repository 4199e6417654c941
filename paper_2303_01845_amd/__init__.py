"""Python binding of the batched Smith-Waterman library (include/sw.h).

Argument marshalling only: every step of the alignment path runs in the HIP
kernels of ``libsw_hip.so``.  PyTorch supplies device memory and streams.  If
the library is not built, every entry point raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsw_hip.so")

SW_OK = 0
SW_EINVAL = -1
SW_ERANGE = -2
SW_ECODE = -3
SW_ENOMEM = -4
SW_EDEVICE = -5
SW_ETIMEOUT = -6
SW_EAGAIN = -7
SW_ECANCELED = -8
MAX_SEQ_LEN = 65535

PERSISTENT = 0
PLAIN = 1
VALIDATE = 2
NO_GRAPH = 4
TIMED = 8
COVERAGE_FIRST = 16

# every function the C header declares
EXPORTS = ("sw_packed_bytes", "sw_pack", "sw_batch_align", "sw_align_sets", "sw_align_sets_ws",
           "sw_align_sets_static",
           "sw_workspace_size", "sw_check", "sw_timing_read",
           "sw_timing_read_passes", "sw_set_tuning",
           "sw_get_tuning", "sw_autotune", "sw_matrix", "sw_strerror", "sw_last_device_error", "sw_server_create",
           "sw_server_submit", "sw_server_poll", "sw_server_wait", "sw_server_stats",
           "sw_server_request_bytes", "sw_server_destroy", "sw_discover", "sw_identity", "sw_search")

DISCOVER_ALL = 0
DISCOVER_UPPER = 1
DISCOVER_PARITY = 2


class SwError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        L = _lib
        msg = L.sw_strerror(status).decode() if L is not None else str(status)
        if status == SW_EDEVICE and L is not None:
            msg += " (" + L.sw_last_device_error().decode() + ")"
        super().__init__("%s: %s [%d]" % (where, msg, status))


class Scoring(ctypes.Structure):
    _fields_ = [("matrix_id", ctypes.c_int32), ("gap_open", ctypes.c_int32),
                ("gap_extend", ctypes.c_int32)]


NUM_BUCKETS = 17


class Tuning(ctypes.Structure):
    _fields_ = [("rows_per_lane", ctypes.c_int32), ("inter_max_len", ctypes.c_int32),
                ("blocks_per_cu", ctypes.c_int32), ("group16_max_len", ctypes.c_int32),
                ("group8_max_len", ctypes.c_int32), ("bucket_lanes", ctypes.c_int8 * NUM_BUCKETS)]


class SearchStats(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int64), ("edges", ctypes.c_int64), ("blocks", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]





_lib = None


def lib():
    """The loaded C library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libsw_hip.so is not built (run __graft_entry__.build() or "
                              "python paper_2303_01845_amd/build.py)")
        L = ctypes.CDLL(LIB_PATH)
        L.sw_packed_bytes.argtypes = [ctypes.c_int64]
        L.sw_packed_bytes.restype = ctypes.c_size_t
        L.sw_pack.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t,
                              ctypes.c_void_p]
        L.sw_batch_align.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(Scoring),
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]
        L.sw_align_sets.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                    ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(Scoring),
                                    ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]
        L.sw_align_sets_ws.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(Scoring),
                                       ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p,
                                       ctypes.c_uint32]
        L.sw_align_sets_static.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                           ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(Scoring),
                                           ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint32]
        L.sw_workspace_size.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
        L.sw_check.argtypes = [ctypes.c_void_p]
        L.sw_timing_read.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                     ctypes.POINTER(ctypes.c_int64)]
        L.sw_timing_read_passes.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_double),
                                            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]
        L.sw_server_create.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.POINTER(Scoring), ctypes.c_size_t, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.sw_server_submit.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                       ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_uint64)]
        L.sw_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
        L.sw_server_wait.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64]
        L.sw_server_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64),
                                      ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)]
        L.sw_server_request_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int64]
        L.sw_server_request_bytes.restype = ctypes.c_size_t
        L.sw_server_destroy.argtypes = [ctypes.c_void_p]
        L.sw_set_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.sw_get_tuning.argtypes = [ctypes.POINTER(Tuning)]
        L.sw_autotune.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                  ctypes.c_int64, ctypes.POINTER(Scoring), ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_int32, ctypes.c_char_p, ctypes.POINTER(Tuning),
                                  ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_int32)]
        L.sw_search.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64, ctypes.c_void_p,
                                ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                ctypes.POINTER(Scoring), ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                ctypes.POINTER(SearchStats), ctypes.c_void_p]

        L.sw_matrix.argtypes = [ctypes.c_int32, ctypes.c_void_p, ctypes.c_char_p]
        L.sw_identity.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(Scoring),
                                  ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_uint32]
        L.sw_discover.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                  ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int64, ctypes.POINTER(ctypes.c_int64),
                                  ctypes.c_size_t, ctypes.c_void_p]
        L.sw_strerror.argtypes = [ctypes.c_int]
        L.sw_strerror.restype = ctypes.c_char_p
        L.sw_last_device_error.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != SW_OK:
        raise SwError(status, where)


def _stream_ptr(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def packed_bytes(n_residues: int) -> int:
    return int(lib().sw_packed_bytes(int(n_residues)))


def pack(ascii, stream=None):
    """ASCII residues (uint8 tensor on the GPU, or bytes/numpy, copied there)
    -> packed device buffer (uint8 tensor)."""
    import torch
    if not isinstance(ascii, torch.Tensor):
        ascii = torch.from_numpy(np.frombuffer(bytes(ascii), dtype=np.uint8).copy()
                                 if not isinstance(ascii, np.ndarray) else ascii.astype(np.uint8))
    if not ascii.is_cuda:
        ascii = ascii.to("cuda", non_blocking=False)
    ascii = ascii.contiguous()
    n = ascii.numel()
    cap = packed_bytes(n)
    out = torch.empty(cap, dtype=torch.uint8, device=ascii.device)
    _check(lib().sw_pack(ctypes.c_void_p(ascii.data_ptr() if n else 0), n,
                         ctypes.c_void_p(out.data_ptr()), cap, _stream_ptr(stream)), "sw_pack")
    return out


def align(packed, offsets, pairs, gap_open: int = 11, gap_extend: int = 1, flags: int = PERSISTENT,
          out=None, stream=None):
    """Align every (query, reference) pair.  ``packed`` from ``pack``;
    ``offsets`` int64 [n_seqs+1] and ``pairs`` int32 [n_pairs, 2] on the GPU.
    Returns int32 [n_pairs, 5] on the GPU: score, q_start, q_end, r_start, r_end."""
    import torch
    n_pairs = int(pairs.shape[0]) if pairs.dim() == 2 else int(pairs.numel() // 2)
    if out is None:
        out = torch.empty((n_pairs, 5), dtype=torch.int32, device=pairs.device)
    assert offsets.dtype == torch.int64 and pairs.dtype == torch.int32 and out.dtype == torch.int32
    assert offsets.is_contiguous() and pairs.is_contiguous() and out.is_contiguous()
    sc = Scoring(0, int(gap_open), int(gap_extend))
    _check(lib().sw_batch_align(ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                                int(offsets.numel()) - 1, ctypes.c_void_p(pairs.data_ptr()), n_pairs,
                                ctypes.byref(sc), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream),
                                int(flags)), "sw_batch_align")
    return out


def align_sets(q_packed, q_offsets, r_packed, r_offsets, pairs, gap_open: int = 11,
               gap_extend: int = 1, flags: int = PERSISTENT, out=None, stream=None):
    """Like align with queries and references in two packed buffers."""
    import torch
    n_pairs = int(pairs.shape[0]) if pairs.dim() == 2 else int(pairs.numel() // 2)
    if out is None:
        out = torch.empty((n_pairs, 5), dtype=torch.int32, device=pairs.device)
    assert q_offsets.dtype == torch.int64 and r_offsets.dtype == torch.int64
    assert pairs.dtype == torch.int32 and out.dtype == torch.int32 and pairs.is_contiguous()
    sc = Scoring(0, int(gap_open), int(gap_extend))
    _check(lib().sw_align_sets(ctypes.c_void_p(q_packed.data_ptr()), ctypes.c_void_p(q_offsets.data_ptr()),
                               int(q_offsets.numel()) - 1, ctypes.c_void_p(r_packed.data_ptr()),
                               ctypes.c_void_p(r_offsets.data_ptr()), int(r_offsets.numel()) - 1,
                               ctypes.c_void_p(pairs.data_ptr()), n_pairs, ctypes.byref(sc),
                               ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream), int(flags)),
           "sw_align_sets")
    return out


def workspace_size(n_pairs: int, max_len: int = MAX_SEQ_LEN) -> int:
    """Bytes of a caller-owned workspace for sw_align_sets_ws (full grid,
    every pair up to ``max_len`` reference residues on the whole-wave scan)."""
    b = ctypes.c_size_t()
    _check(lib().sw_workspace_size(int(n_pairs), int(max_len), ctypes.byref(b)), "sw_workspace_size")
    return int(b.value)


def align_sets_ws(q_packed, q_offsets, r_packed, r_offsets, pairs, workspace, gap_open: int = 11,
                  gap_extend: int = 1, flags: int = PERSISTENT, out=None, stream=None):
    """align_sets with a caller-owned device workspace (a uint8 tensor,
    256-byte aligned; see workspace_size)."""
    import torch
    n_pairs = int(pairs.shape[0]) if pairs.dim() == 2 else int(pairs.numel() // 2)
    if out is None:
        out = torch.empty((n_pairs, 5), dtype=torch.int32, device=pairs.device)
    assert q_offsets.dtype == torch.int64 and r_offsets.dtype == torch.int64
    assert pairs.dtype == torch.int32 and out.dtype == torch.int32 and pairs.is_contiguous()
    sc = Scoring(0, int(gap_open), int(gap_extend))
    _check(lib().sw_align_sets_ws(ctypes.c_void_p(q_packed.data_ptr()), ctypes.c_void_p(q_offsets.data_ptr()),
                                  int(q_offsets.numel()) - 1, ctypes.c_void_p(r_packed.data_ptr()),
                                  ctypes.c_void_p(r_offsets.data_ptr()), int(r_offsets.numel()) - 1,
                                  ctypes.c_void_p(pairs.data_ptr()), n_pairs, ctypes.byref(sc),
                                  ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(workspace.data_ptr()),
                                  int(workspace.numel() * workspace.element_size()), _stream_ptr(stream),
                                  int(flags)), "sw_align_sets_ws")
    return out


def align_sets_static(q_packed, q_offsets, r_packed, r_offsets, pairs, gap_open: int = 11,
                      gap_extend: int = 1, flags: int = PERSISTENT, out=None, stream=None):
    """align_sets through the entry point that allocates nothing (its
    workspace is the library's fixed per-device array).  ``out`` must be
    given by callers that cannot allocate."""
    import torch
    n_pairs = int(pairs.shape[0]) if pairs.dim() == 2 else int(pairs.numel() // 2)
    if out is None:
        out = torch.empty((n_pairs, 5), dtype=torch.int32, device=pairs.device)
    assert q_offsets.dtype == torch.int64 and r_offsets.dtype == torch.int64
    assert pairs.dtype == torch.int32 and out.dtype == torch.int32 and pairs.is_contiguous()
    sc = Scoring(0, int(gap_open), int(gap_extend))
    _check(lib().sw_align_sets_static(ctypes.c_void_p(q_packed.data_ptr()), ctypes.c_void_p(q_offsets.data_ptr()),
                                      int(q_offsets.numel()) - 1, ctypes.c_void_p(r_packed.data_ptr()),
                                      ctypes.c_void_p(r_offsets.data_ptr()), int(r_offsets.numel()) - 1,
                                      ctypes.c_void_p(pairs.data_ptr()), n_pairs, ctypes.byref(sc),
                                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream), int(flags)),
           "sw_align_sets_static")
    return out


def check(stream=None):
    """Synchronise and raise for device-detected errors (SW_ERANGE / SW_ECODE)."""
    _check(lib().sw_check(_stream_ptr(stream)), "sw_check")


def timing_read(stream=None):
    """(kernel milliseconds, calls) summed over the SW_TIMED calls on `stream`
    since the previous read; synchronises the stream."""
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().sw_timing_read(_stream_ptr(stream), ctypes.byref(ms), ctypes.byref(n)), "sw_timing_read")
    return ms.value, n.value


def timing_read_passes(stream=None):
    """(forward ms, start-pass ms, calls) over the SW_TIMED calls on `stream`
    since the previous read (SW_PLAIN calls count as forward); synchronises."""
    f, s, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(lib().sw_timing_read_passes(_stream_ptr(stream), ctypes.byref(f), ctypes.byref(s), ctypes.byref(n)),
           "sw_timing_read_passes")
    return f.value, s.value, n.value


def _tuning_dict(t) -> dict:
    return {"rows_per_lane": t.rows_per_lane, "inter_max_len": t.inter_max_len,
            "blocks_per_cu": t.blocks_per_cu, "group16_max_len": t.group16_max_len,
            "group8_max_len": t.group8_max_len, "bucket_lanes": list(t.bucket_lanes)}


def set_tuning(rows_per_lane: int = 0, inter_max_len: int = 0, blocks_per_cu: int = 0,
               group16_max_len: int = 0, group8_max_len: int = 0, bucket_lanes=None):
    """0 keeps a field; blocks_per_cu -1 returns to the occupancy-derived grid;
    bucket_lanes (17 lane counts, 0 = the threshold rule) is applied as given
    (all zeros when omitted)."""
    lanes = (ctypes.c_int8 * NUM_BUCKETS)(*(bucket_lanes or [0] * NUM_BUCKETS))
    _check(lib().sw_set_tuning(ctypes.byref(Tuning(rows_per_lane, inter_max_len, blocks_per_cu,
                                                   group16_max_len, group8_max_len, lanes))), "sw_set_tuning")


def get_tuning() -> dict:
    t = Tuning()
    _check(lib().sw_get_tuning(ctypes.byref(t)), "sw_get_tuning")
    return _tuning_dict(t)


def autotune(packed, offsets, pairs, gap_open: int = 11, gap_extend: int = 1, reps: int = 3,
             out=None, stream=None, cache_path=None):
    """Per length bucket, pick and keep the fastest lane count for this
    workload (results must be identical across candidates), with an optional
    JSON cache of earlier choices.  Returns (tuning dict, ms per call of the
    whole workload, bucket candidates timed)."""
    import torch
    n_pairs = int(pairs.shape[0])
    if out is None:
        out = torch.empty((n_pairs, 5), dtype=torch.int32, device=pairs.device)
    t = Tuning()
    ms = ctypes.c_float()
    trials = ctypes.c_int32()
    sc = Scoring(0, int(gap_open), int(gap_extend))
    path = None if cache_path is None else str(cache_path).encode()
    _check(lib().sw_autotune(ctypes.c_void_p(packed.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                             int(offsets.numel()) - 1, ctypes.c_void_p(pairs.data_ptr()), n_pairs,
                             ctypes.byref(sc), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream), int(reps),
                             path, ctypes.byref(t), ctypes.byref(ms), ctypes.byref(trials)), "sw_autotune")
    return _tuning_dict(t), float(ms.value), int(trials.value)


def search(q_packed, q_offsets, r_packed, r_offsets, k: int = 6, min_shared: int = 2, mode: int = 0,
           gap_open: int = 11, gap_extend: int = 1, ani_permille: int = 300, cov_permille: int = 700,
           block_queries: int = 0, edge_cap=None, stream=None):
    """The whole search on the device (sw_search): discovery, alignment and
    the identity / coverage filter, block by block.  Returns (edges int32
    [n, 2], alignment results int32 [n, 5], identity records int32 [n, 4],
    stats dict); the edges come in no particular order."""
    import torch
    dev = q_packed.device
    n_q = int(q_offsets.numel()) - 1
    cap = int(edge_cap) if edge_cap is not None else max(1024, 32 * n_q)
    sc = Scoring(0, int(gap_open), int(gap_extend))
    while True:
        e = torch.empty((cap, 2), dtype=torch.int32, device=dev)
        r = torch.empty((cap, 5), dtype=torch.int32, device=dev)
        i = torch.empty((cap, 4), dtype=torch.int32, device=dev)
        st = SearchStats()
        rc = lib().sw_search(ctypes.c_void_p(q_packed.data_ptr()), ctypes.c_void_p(q_offsets.data_ptr()), n_q,
                             ctypes.c_void_p(r_packed.data_ptr()), ctypes.c_void_p(r_offsets.data_ptr()),
                             int(r_offsets.numel()) - 1, int(k), int(min_shared), int(mode), ctypes.byref(sc),
                             int(ani_permille), int(cov_permille), int(block_queries), ctypes.c_void_p(e.data_ptr()),
                             ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(i.data_ptr()), cap, ctypes.byref(st),
                             _stream_ptr(stream))
        if rc == SW_ENOMEM and edge_cap is None and st.edges > cap:
            cap = int(st.edges)
            continue
        _check(rc, "sw_search")
        n = int(st.edges)
        return e[:n], r[:n], i[:n], {"candidates": int(st.candidates), "edges": n, "blocks": int(st.blocks)}


def matrix():
    """(int8 [24, 24] scores, alphabet string) as compiled into the library."""
    scores = np.zeros(24 * 24, dtype=np.int8)
    letters = ctypes.create_string_buffer(25)
    _check(lib().sw_matrix(0, scores.ctypes.data, letters), "sw_matrix")
    return scores.reshape(24, 24), letters.value.decode()


def discover(q_packed, q_offsets, r_packed, r_offsets, k: int = 6, min_shared: int = 2,
             mode: int = DISCOVER_ALL, capacity: int | None = None, table_budget: int = 0, stream=None):
    """Candidate pairs with at least ``min_shared`` distinct common k-mers
    (sw_discover).  Returns (pairs int32 [n, 2], shared int32 [n]) on the GPU,
    in unspecified order.  Without ``capacity`` the library is asked for the
    count first; with it, a too-small capacity raises SW_ENOMEM.
    ``table_budget`` bounds the pair-counter table in bytes (0: no bound)."""
    import torch
    assert q_offsets.dtype == torch.int64 and r_offsets.dtype == torch.int64
    L = lib()
    st = _stream_ptr(stream)
    dev = q_offsets.device
    args = (ctypes.c_void_p(q_packed.data_ptr()), ctypes.c_void_p(q_offsets.data_ptr()),
            int(q_offsets.numel()) - 1, ctypes.c_void_p(r_packed.data_ptr()),
            ctypes.c_void_p(r_offsets.data_ptr()), int(r_offsets.numel()) - 1, int(k), int(min_shared), int(mode))
    found = ctypes.c_int64()
    if capacity is None:
        status = L.sw_discover(*args, None, None, 0, ctypes.byref(found), int(table_budget), st)
        if status not in (SW_OK, SW_ENOMEM):
            _check(status, "sw_discover")
        capacity = found.value
    pairs = torch.empty((max(capacity, 1), 2), dtype=torch.int32, device=dev)
    shared = torch.empty(max(capacity, 1), dtype=torch.int32, device=dev)
    _check(L.sw_discover(*args, ctypes.c_void_p(pairs.data_ptr()), ctypes.c_void_p(shared.data_ptr()),
                         int(capacity), ctypes.byref(found), int(table_budget), st), "sw_discover")
    n = found.value
    return pairs[:n], shared[:n]


def identity(q_packed, q_offsets, r_packed, r_offsets, pairs, aligned, gap_open: int = 11,
             gap_extend: int = 1, ani_permille: int = 300, cov_permille: int = 700, flags: int = 0,
             out=None, stream=None):
    """Identity and coverage records of aligned pairs (sw_identity): int32
    [n_pairs, 4] on the GPU -- box score, matches, columns, keep."""
    import torch
    n_pairs = int(pairs.shape[0]) if pairs.dim() == 2 else int(pairs.numel() // 2)
    if out is None:
        out = torch.empty((n_pairs, 4), dtype=torch.int32, device=pairs.device)
    assert q_offsets.dtype == torch.int64 and r_offsets.dtype == torch.int64
    assert pairs.dtype == torch.int32 and aligned.dtype == torch.int32 and out.dtype == torch.int32
    assert pairs.is_contiguous() and aligned.is_contiguous() and out.is_contiguous()
    sc = Scoring(0, int(gap_open), int(gap_extend))
    _check(lib().sw_identity(ctypes.c_void_p(q_packed.data_ptr()), ctypes.c_void_p(q_offsets.data_ptr()),
                             int(q_offsets.numel()) - 1, ctypes.c_void_p(r_packed.data_ptr()),
                             ctypes.c_void_p(r_offsets.data_ptr()), int(r_offsets.numel()) - 1,
                             ctypes.c_void_p(pairs.data_ptr()), n_pairs, ctypes.byref(sc),
                             ctypes.c_void_p(aligned.data_ptr()), int(ani_permille), int(cov_permille),
                             ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream), int(flags)), "sw_identity")
    return out


class Batch:
    """Sequences resident on the GPU (packed) plus their offsets."""

    def __init__(self, ascii: np.ndarray, offsets: np.ndarray, stream=None):
        import torch
        self.offsets = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.int64)).cuda()
        a = torch.from_numpy(np.ascontiguousarray(ascii, dtype=np.uint8)).cuda()
        self.packed = pack(a, stream)
        self.n_residues = int(a.numel())

    def align(self, pairs, gap_open: int = 11, gap_extend: int = 1, flags: int = PERSISTENT,
              out=None, stream=None):
        import torch
        if not isinstance(pairs, torch.Tensor):
            pairs = torch.from_numpy(np.ascontiguousarray(pairs, dtype=np.int32).reshape(-1, 2)).cuda()
        return align(self.packed, self.offsets, pairs, gap_open, gap_extend, flags, out, stream)
