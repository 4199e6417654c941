"""GPU test of the whole search on the device (sw_search): discovery by
shared k-mers, alignment and the identity / coverage filter, block by block.
On family sets small enough for the oracle, the edges (pairs kept, with their
alignment and identity records) equal the oracle's own three stages, for
several block sizes and for a self search with the triangle filter; on the
full 50k x 50k block set they equal the library's separate stage calls, and a
sample of them the oracle."""
import sys

import numpy as np
import pytest

import oracle
from workloads import proteins as P

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def sw():
    import torch
    assert torch.cuda.is_available(), "no GPU"
    import paper_2303_01845_amd as lib
    lib.lib()
    lib.set_tuning(16, 1024, -1, 2048, 2048)
    return lib


def split_family_set(config, n_fam, n_members):
    asc, offs, _ = P.families(config, n_fam, n_members)
    L = np.diff(offs)

    def take(ix):
        o = np.zeros(len(ix) + 1, dtype=np.int64)
        np.cumsum(L[ix], out=o[1:])
        return asc[P.gather_segments(offs[ix], L[ix])], o

    qa, qo = take(np.arange(0, n_members, 2))
    ra, ro = take(np.arange(1, n_members, 2))
    return qa, qo, ra, ro


def oracle_edges(qa, qo, ra, ro, mode=0, ani=300, cov=700):
    """{(q, r): (alignment record, identity record)} of the pairs the
    oracle's discovery, alignment and identity filter keep."""
    q, r, _ = oracle.discover(qa, qo, ra, ro, 6, 2, mode)
    nq = len(qo) - 1
    asc = np.concatenate([qa, ra])
    offs = np.concatenate([qo, ro[1:] + qo[-1]])
    pairs = np.stack([q, r + nq], 1).astype(np.int32)
    aln = oracle.batch_ascii(asc, offs, pairs, 11, 1)
    idr = oracle.identity_ascii(asc, offs, pairs, aln, 11, 1, ani, cov)
    keep = np.flatnonzero(idr[:, 3] == 1)
    return len(q), {(int(q[k]), int(r[k])): (tuple(aln[k]), tuple(idr[k])) for k in keep}


def gpu_edges(e, rr, ii):
    e, rr, ii = e.cpu().numpy(), rr.cpu().numpy(), ii.cpu().numpy()
    out = {(int(a), int(b)): (tuple(x), tuple(y)) for (a, b), x, y in zip(e, rr, ii)}
    assert len(out) == len(e), "an edge is reported twice"
    return out


def test_search_matches_oracle_stages(sw):
    qa, qo, ra, ro = split_family_set(9, 150, 3000)
    n_cand, exp = oracle_edges(qa, qo, ra, ro)
    say("family set: %d x %d, %d candidates, %d edges by the oracle" % (len(qo) - 1, len(ro) - 1, n_cand, len(exp)))
    qb, rb = sw.Batch(qa, qo), sw.Batch(ra, ro)
    for block in (0, 100, 333, 1500):
        e, rr, ii, st = sw.search(qb.packed, qb.offsets, rb.packed, rb.offsets, block_queries=block)
        got = gpu_edges(e, rr, ii)
        say("block_queries %d: %s" % (block, st))
        assert st["candidates"] == n_cand
        assert got == exp, "block_queries %d: %d edges vs %d" % (block, len(got), len(exp))


def test_search_capacity_and_self_search(sw):
    import ctypes
    import torch
    qa, qo, ra, ro = split_family_set(10, 120, 2400)
    _, exp = oracle_edges(qa, qo, ra, ro)
    qb, rb = sw.Batch(qa, qo), sw.Batch(ra, ro)
    cap = max(1, len(exp) // 3)
    e = torch.empty((cap, 2), dtype=torch.int32, device="cuda")
    r = torch.empty((cap, 5), dtype=torch.int32, device="cuda")
    i = torch.empty((cap, 4), dtype=torch.int32, device="cuda")
    st = sw.SearchStats()
    sc = sw.Scoring(0, 11, 1)
    rc = sw.lib().sw_search(ctypes.c_void_p(qb.packed.data_ptr()), ctypes.c_void_p(qb.offsets.data_ptr()),
                            len(qo) - 1, ctypes.c_void_p(rb.packed.data_ptr()), ctypes.c_void_p(rb.offsets.data_ptr()),
                            len(ro) - 1, 6, 2, 0, ctypes.byref(sc), 300, 700, 200, ctypes.c_void_p(e.data_ptr()),
                            ctypes.c_void_p(r.data_ptr()), ctypes.c_void_p(i.data_ptr()), cap, ctypes.byref(st), None)
    assert rc == sw.SW_ENOMEM and st.edges == len(exp)
    part = gpu_edges(e, r, i)
    assert len(part) == cap and all(exp[k] == v for k, v in part.items())
    # self search of one set with the triangle filter (q < r only)
    n_cand, exp_self = oracle_edges(qa, qo, qa, qo, mode=1)
    e, rr, ii, st = sw.search(qb.packed, qb.offsets, qb.packed, qb.offsets, mode=1, block_queries=300)
    got = gpu_edges(e, rr, ii)
    say("self search: %s, oracle %d candidates, %d edges" % (st, n_cand, len(exp_self)))
    assert st["candidates"] == n_cand and got == exp_self
    assert all(a < b for a, b in got)


def test_search_block_set_full_size(sw):
    import torch
    ps = P.config_block()
    nq = 50_000
    say("block set: %d pairs by the generator" % ps.n_pairs)
    b = sw.Batch(ps.ascii, ps.offsets)
    qoff, roff = b.offsets[:nq + 1], b.offsets[nq:]
    nr = ps.n_seqs - nq
    e, rr, ii, st = sw.search(b.packed, qoff, b.packed, roff, block_queries=12_500)
    say("search: %s" % st)
    assert st["blocks"] == 4 and st["candidates"] == ps.n_pairs
    got = gpu_edges(e, rr, ii)
    # the separate stage calls on the same sets
    pairs, _ = sw.discover(b.packed, qoff, b.packed, roff)
    aln = sw.align_sets(b.packed, qoff, b.packed, roff, pairs, flags=sw.VALIDATE)
    idr = sw.identity(b.packed, qoff, b.packed, roff, pairs, aln, 11, 1, 300, 700, flags=sw.VALIDATE)
    p, a, i = pairs.cpu().numpy(), aln.cpu().numpy(), idr.cpu().numpy()
    keep = np.flatnonzero(i[:, 3] == 1)
    stages = {(int(p[k, 0]), int(p[k, 1])): (tuple(a[k]), tuple(i[k])) for k in keep}
    assert got == stages, "%d edges vs %d by the stage calls" % (len(got), len(stages))
    say("full block set: %d edges equal to the stage calls" % len(got))
    # a sample of the edges against the oracle's alignment and identity
    keys = sorted(got)
    rng = np.random.default_rng(23)
    pick = [keys[k] for k in rng.choice(len(keys), 300, replace=False)]
    pr = np.array([[q, r + nq] for q, r in pick], dtype=np.int32)
    sub = P.PairSet(ps.ascii, ps.offsets, pr).subset(np.arange(len(pr)))
    exp_aln = oracle.batch_ascii(sub.ascii, sub.offsets, sub.pairs, 11, 1)
    exp_id = oracle.identity_ascii(sub.ascii, sub.offsets, sub.pairs, exp_aln, 11, 1, 300, 700)
    for k, key in enumerate(pick):
        assert got[key] == (tuple(exp_aln[k]), tuple(exp_id[k])), key
