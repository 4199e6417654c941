"""Host-side checks of the HIP library (no GPU needed): it loads, exports every
symbol the C header declares, carries the right substitution table, and
rejects bad arguments before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2303_01845_amd as sw

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in os.listdir(os.path.join(ROOT, "include")):
        if h.endswith(".h"):
            text = open(os.path.join(ROOT, "include", h)).read()
            names |= set(re.findall(r"SW_API\s+[\w\s\*]+?\b(sw_\w+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = sw.lib()
    decl = declared_functions()
    assert len(decl) >= 9
    assert decl == set(sw.EXPORTS)
    for name in decl:
        assert hasattr(L, name), name


def test_library_matrix_matches_oracle_table():
    scores, letters = sw.matrix()
    O = oracle.default()
    assert letters == O.letters
    assert (scores == O.scores).all()


def test_strerror_covers_every_status():
    L = sw.lib()
    seen = set()
    for code in range(0, -9, -1):
        s = L.sw_strerror(code).decode()
        assert s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 9
    assert L.sw_strerror(-99).decode() == "unknown status"


def test_packed_bytes_grows_with_length():
    assert sw.packed_bytes(0) > 256
    sizes = [sw.packed_bytes(n) for n in (0, 1, 255, 256, 10 ** 6, 3 * 10 ** 10)]
    assert sizes == sorted(sizes)
    assert sw.packed_bytes(10 ** 6) < 10 ** 6  # 5 bits per residue plus overhead
    assert sw.lib().sw_packed_bytes(-1) == 0


def _align_raw(go, ge, n_pairs=1, flags=0, null=False, matrix_id=0):
    L = sw.lib()
    sc = sw.Scoring(matrix_id, go, ge)
    p = ctypes.c_void_p(0 if null else 0x1000)
    return L.sw_batch_align(p, p, 10, p, n_pairs, ctypes.byref(sc), p, None, flags)


def test_align_argument_checks_precede_device_use():
    assert _align_raw(11, 1, n_pairs=0) == sw.SW_OK            # nothing to do
    assert _align_raw(0, 0) == sw.SW_EINVAL                     # gap_open must be >= 1
    assert _align_raw(2, 3) == sw.SW_EINVAL                     # extend above open
    assert _align_raw(11, -1) == sw.SW_EINVAL
    assert _align_raw((1 << 20) + 1, 1) == sw.SW_EINVAL
    assert _align_raw(11, 1, matrix_id=1) == sw.SW_EINVAL
    assert _align_raw(11, 1, flags=64) == sw.SW_EINVAL
    assert _align_raw(11, 1, null=True) == sw.SW_EINVAL
    assert _align_raw(11, 1, n_pairs=-5) == sw.SW_EINVAL
    L = sw.lib()
    assert L.sw_batch_align(None, None, 0, None, 0, None, None, None, 0) == sw.SW_EINVAL


def test_pack_argument_checks_precede_device_use():
    L = sw.lib()
    assert L.sw_pack(None, 10, ctypes.c_void_p(0x1000), 1 << 20, None) == sw.SW_EINVAL
    assert L.sw_pack(ctypes.c_void_p(0x1000), -1, ctypes.c_void_p(0x1000), 1 << 20, None) == sw.SW_EINVAL
    assert L.sw_pack(ctypes.c_void_p(0x1000), 10, None, 1 << 20, None) == sw.SW_EINVAL
    assert L.sw_pack(ctypes.c_void_p(0x1000), 1000, ctypes.c_void_p(0x1000), 100, None) == sw.SW_ENOMEM


def test_tuning_argument_checks():
    L = sw.lib()
    assert L.sw_set_tuning(None) == sw.SW_EINVAL
    for bad in [(32, 0, 0, 0), (24, 0, 0, 0), (0, 32, 0, 0), (0, 4096, 0, 0), (0, 0, 9, 0), (8, 1024, 0, 0),
                (0, 0, 0, 3000), (0, 0, 0, 8192), (0, 0, 0, 32), (0, 0, -2, 0), (0, 0, 0, 0, 32),
                (0, 0, 0, 0, 3000), (0, 0, 0, 0, 8192)]:
        assert L.sw_set_tuning(ctypes.byref(sw.Tuning(*bad))) == sw.SW_EINVAL
    for b, lanes in [(0, 2), (5, 32), (11, 1), (13, 8), (13, 16), (16, -1), (3, 4)]:
        table = [0] * sw.NUM_BUCKETS
        table[b] = lanes
        t = sw.Tuning(0, 0, 0, 0, 0, (ctypes.c_int8 * sw.NUM_BUCKETS)(*table))
        assert L.sw_set_tuning(ctypes.byref(t)) == sw.SW_EINVAL, (b, lanes)
    assert L.sw_get_tuning(None) == sw.SW_EINVAL
    assert L.sw_matrix(1, None, None) == sw.SW_EINVAL


def test_no_cpu_fallback_when_library_missing(tmp_path, monkeypatch):
    monkeypatch.setattr(sw, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(sw, "_lib", None)
    with pytest.raises(ImportError):
        sw.lib()


def _discover_raw(n_q=10, n_r=10, k=6, t=2, mode=0, cap=0, out=False, null=False, found=True):
    L = sw.lib()
    p = ctypes.c_void_p(0 if null else 0x1000)
    o = ctypes.c_void_p(0x2000 if out else 0)
    n = ctypes.c_int64(-1)
    rc = L.sw_discover(p, p, n_q, p, p, n_r, k, t, mode, o, None, cap,
                       ctypes.byref(n) if found else None, 0, None)
    return rc, n.value


def test_discover_argument_checks_precede_device_use():
    assert _discover_raw(found=False)[0] == sw.SW_EINVAL
    for kw in ({"k": 0}, {"k": 7}, {"t": 0}, {"mode": 3}, {"mode": -1}, {"cap": -1},
               {"mode": 1, "n_r": 9}, {"mode": 2, "n_q": 3}, {"cap": 5}, {"n_q": -1}):
        assert _discover_raw(**kw) == (sw.SW_EINVAL, 0), kw
    assert _discover_raw(n_q=1 << 31) == (sw.SW_ERANGE, 0)
    assert _discover_raw(n_q=0) == (sw.SW_OK, 0)                  # nothing to do
    assert _discover_raw(n_r=0, cap=4, out=True) == (sw.SW_OK, 0)
    assert _discover_raw(null=True) == (sw.SW_EINVAL, 0)


def _identity_raw(go=11, ge=1, n_pairs=3, ani=300, cov=700, flags=0, null=False):
    L = sw.lib()
    sc = sw.Scoring(0, go, ge)
    p = ctypes.c_void_p(0 if null else 0x1000)
    return L.sw_identity(p, p, 10, p, p, 10, p, n_pairs, ctypes.byref(sc), p, ani, cov, p, None, flags)


def test_identity_argument_checks_precede_device_use():
    assert _identity_raw(n_pairs=0) == sw.SW_OK
    assert _identity_raw(go=0, ge=0) == sw.SW_EINVAL
    assert _identity_raw(go=2, ge=3) == sw.SW_EINVAL
    assert _identity_raw(ani=-1) == sw.SW_EINVAL
    assert _identity_raw(cov=1001) == sw.SW_EINVAL
    assert _identity_raw(flags=sw.PLAIN) == sw.SW_EINVAL
    assert _identity_raw(flags=sw.TIMED) == sw.SW_EINVAL
    assert _identity_raw(n_pairs=-1) == sw.SW_EINVAL
    assert _identity_raw(null=True) == sw.SW_EINVAL
    assert _identity_raw(n_pairs=1 << 31) == sw.SW_ERANGE


def _ws_raw(ws=0x100000, ws_bytes=1 << 30, go=11, ge=1, n_pairs=3, flags=0, null=False):
    L = sw.lib()
    sc = sw.Scoring(0, go, ge)
    p = ctypes.c_void_p(0 if null else 0x1000)
    return L.sw_align_sets_ws(p, p, 10, p, p, 10, p, n_pairs, ctypes.byref(sc), p, ctypes.c_void_p(ws), ws_bytes,
                              None, flags)


def test_caller_workspace_argument_checks_precede_device_use():
    assert _ws_raw(ws=0) == sw.SW_EINVAL                     # the workspace is required
    assert _ws_raw(ws=0x100010) == sw.SW_EINVAL              # not 256-byte aligned
    assert _ws_raw(go=0, ge=0) == sw.SW_EINVAL
    assert _ws_raw(flags=64) == sw.SW_EINVAL
    assert _ws_raw(null=True) == sw.SW_EINVAL
    assert _ws_raw(n_pairs=-1) == sw.SW_EINVAL
    assert _ws_raw(n_pairs=0) == sw.SW_OK                    # nothing to do
    L = sw.lib()
    b = ctypes.c_size_t(7)
    assert L.sw_workspace_size(10, 100, None) == sw.SW_EINVAL
    assert L.sw_workspace_size(-1, 100, ctypes.byref(b)) == sw.SW_EINVAL
    assert L.sw_workspace_size(10, -1, ctypes.byref(b)) == sw.SW_EINVAL
    assert L.sw_workspace_size(10, sw.MAX_SEQ_LEN + 1, ctypes.byref(b)) == sw.SW_ERANGE
    assert b.value == 0
