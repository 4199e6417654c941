"""Serving loop over the C server (sw_server_* in include/sw.h).

``Server`` wraps one server object: a reference set resident in HBM, a fixed
number of slots (HIP streams) and an HBM budget for requests in flight; the
admission decision (free slot and free budget) is taken by the library.
``run_open_loop`` drives it with requests arriving at given times: arrived
requests wait in a FIFO queue and are submitted as soon as the server admits
them (continuous batching: a request that arrives while others run joins the
GPU as soon as a slot and memory free up), completions are polled, and the
latency of each request is its completion time minus its arrival time.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from . import SW_EAGAIN, SW_OK, Scoring, SwError, lib


class Server:
    def __init__(self, refs_packed, ref_offsets, gap_open: int = 11, gap_extend: int = 1,
                 hbm_budget: int = 16 << 30, max_slots: int = 4):
        L = lib()
        self._refs = (refs_packed, ref_offsets)  # keep the device buffers alive
        h = ctypes.c_void_p()
        sc = Scoring(0, gap_open, gap_extend)
        rc = L.sw_server_create(ctypes.c_void_p(refs_packed.data_ptr()), ctypes.c_void_p(ref_offsets.data_ptr()),
                                int(ref_offsets.numel()) - 1, ctypes.byref(sc), int(hbm_budget), int(max_slots),
                                ctypes.byref(h))
        if rc != SW_OK:
            raise SwError(rc, "sw_server_create")
        self.h = h
        self._pending = {}

    @staticmethod
    def request_bytes(n_res: int, n_q: int, n_cand: int) -> int:
        return int(lib().sw_server_request_bytes(n_res, n_q, n_cand))

    def submit(self, q_ascii: np.ndarray, q_offsets: np.ndarray, cand: np.ndarray):
        """Ticket, or None when the request is not admissible now."""
        q_ascii = np.ascontiguousarray(q_ascii, dtype=np.uint8)
        q_offsets = np.ascontiguousarray(q_offsets, dtype=np.int64)
        cand = np.ascontiguousarray(cand, dtype=np.int32).reshape(-1, 2)
        out = np.empty((len(cand), 5), dtype=np.int32)
        t = ctypes.c_uint64()
        rc = lib().sw_server_submit(self.h, q_ascii.ctypes.data, q_offsets.ctypes.data, len(q_offsets) - 1,
                                    cand.ctypes.data, len(cand), out.ctypes.data, ctypes.byref(t))
        if rc == SW_EAGAIN:
            return None
        if rc != SW_OK:
            raise SwError(rc, "sw_server_submit")
        self._pending[t.value] = (out, q_ascii, q_offsets, cand)
        return t.value

    def poll(self, ticket):
        """Result array once complete, else None."""
        rc = lib().sw_server_poll(self.h, ctypes.c_uint64(ticket))
        if rc == SW_EAGAIN:
            return None
        if rc != SW_OK:
            raise SwError(rc, "sw_server_poll")
        return self._pending.pop(ticket)[0]

    def wait(self, ticket, timeout_us: int = -1):
        rc = lib().sw_server_wait(self.h, ctypes.c_uint64(ticket), int(timeout_us))
        if rc != SW_OK:
            raise SwError(rc, "sw_server_wait")
        return self._pending.pop(ticket)[0]

    def stats(self) -> dict:
        a, b, c = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        lib().sw_server_stats(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c))
        return {"inflight": a.value, "bytes_in_use": b.value, "budget": c.value}

    def close(self):
        if self.h:
            lib().sw_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_open_loop(server, requests, arrivals, clock=time.perf_counter, idle=lambda: time.sleep(20e-6),
                  progress=None):
    """Serve `requests` (each (q_ascii, q_offsets, cand)) arriving at the
    relative times `arrivals` (seconds, non-decreasing).  Returns per-request
    dicts: arrival, submit, done, latency, result."""
    n = len(requests)
    rec = [dict(arrival=float(a), submit=None, done=None, latency=None, result=None) for a in arrivals]
    queue = []          # arrived, not yet admitted (FIFO)
    inflight = {}       # ticket -> request index
    nxt = 0
    finished = 0
    t0 = clock()
    while finished < n:
        now = clock() - t0
        while nxt < n and arrivals[nxt] <= now:
            queue.append(nxt)
            nxt += 1
        # admit in arrival order while the server accepts
        while queue:
            k = queue[0]
            t = server.submit(*requests[k])
            if t is None:
                break
            queue.pop(0)
            inflight[t] = k
            rec[k]["submit"] = clock() - t0
        progressed = False
        for t in list(inflight):
            res = server.poll(t)
            if res is not None:
                k = inflight.pop(t)
                rec[k]["done"] = clock() - t0
                rec[k]["latency"] = rec[k]["done"] - rec[k]["arrival"]
                rec[k]["result"] = res
                finished += 1
                progressed = True
                if progress and finished % 100 == 0:
                    progress(finished, n)
        if not progressed:
            idle()
    return rec


def summarize(rec, cells_per_request):
    lat = np.array([r["latency"] for r in rec])
    span = max(r["done"] for r in rec) - min(r["arrival"] for r in rec)
    return {"requests": len(rec), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "span_s": float(span), "gcups": float(np.sum(cells_per_request) / span / 1e9)}
