"""GPU parity at full workload sizes, in the configuration the benchmark
times (persistent form, HIP graph, default tuning).

* The 1M log-normal set and the 50k x 50k block set: every pair against the
  CPU oracle, bit for bit on all five outputs (the oracle runs on all host
  threads, about a minute per set, checked in four slices so that no test
  runs long without reporting), and the plain form equal to the persistent
  one on every pair.
* The heavy-tailed batching mix: its first seeded chunk (65,536 pairs, about
  3,300 of them 5,000-35,000 residues long) aligned in one call; every short
  pair against the oracle, plus 500 long pairs: the 20 costliest and 480
  drawn at random, in five slices of 100.  The whole 10M-pair mix is 153 such
  chunks drawn the same way, so this is one chunk-sized shard of it.
"""
import os
import sys
import time

import numpy as np
import pytest

import oracle
from workloads import proteins as P

pytestmark = pytest.mark.gpu

THREADS = max(1, min(16, len(os.sched_getaffinity(0))))
SLICES = 4


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


def align(sw, ps, flags):
    import torch
    b = sw.Batch(ps.ascii, ps.offsets)
    out = b.align(ps.pairs, 11, 1, flags | sw.VALIDATE)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def check_properties(ps, got):
    """Bounds every result must satisfy, whatever the pair."""
    L = ps.lengths().astype(np.int64)
    m = L[ps.pairs[:, 0]]
    n = L[ps.pairs[:, 1]]
    s, qs, qe, rs, re = (got[:, k].astype(np.int64) for k in range(5))
    assert (s >= 0).all() and (s <= 11 * np.minimum(m, n)).all()
    zero = s == 0
    assert (got[zero, 1:] == -1).all()
    pos = ~zero
    assert (qs[pos] >= 0).all() and (qs[pos] <= qe[pos]).all() and (qe[pos] < m[pos]).all()
    assert (rs[pos] >= 0).all() and (rs[pos] <= re[pos]).all() and (re[pos] < n[pos]).all()


def oracle_rows(ps, idx):
    """The oracle's results for pairs idx of ps (all host threads)."""
    sub = ps if idx is None else ps.subset(idx)
    t = time.perf_counter()
    exp = oracle.batch_ascii(sub.ascii, sub.offsets, sub.pairs, 11, 1, threads=THREADS)
    say("oracle: %d pairs, %.3g cells in %.1f s on %d threads" % (sub.n_pairs, sub.cells(),
                                                                   time.perf_counter() - t, THREADS))
    return exp


def assert_rows(got, exp, idx, label):
    bad = np.flatnonzero((got != exp).any(axis=1))
    if len(bad):
        k = int(bad[0])
        pid = k if idx is None else int(idx[k])
        raise AssertionError("%s: %d of %d pairs differ from the oracle; first pair %d: gpu %s oracle %s" % (
            label, len(bad), len(got), pid, got[k].tolist(), exp[k].tolist()))


def aligned_set(sw, ps, label):
    """Persistent results of every pair, checked for bounds and against the
    plain form."""
    say("%s: %d pairs, %.4g cells, longest %d" % (label, ps.n_pairs, ps.cells(), ps.lengths().max()))
    got = align(sw, ps, sw.PERSISTENT)
    say("%s: aligned (persistent + graph)" % label)
    check_properties(ps, got)
    plain = align(sw, ps, sw.PLAIN)
    diff = np.flatnonzero((got != plain).any(axis=1))
    assert len(diff) == 0, "%s: persistent and plain differ on %d pairs (first %d)" % (label, len(diff), diff[0])
    say("%s: plain form equal on every pair" % label)
    return ps, got


def check_slice(state, k, label):
    ps, got = state
    idx = np.array_split(np.arange(ps.n_pairs), SLICES)[k]
    assert_rows(got[idx], oracle_rows(ps, idx), idx, "%s slice %d" % (label, k))
    say("%s: slice %d (%d pairs) bit-exact against the oracle" % (label, k, len(idx)))


@pytest.fixture(scope="module")
def lognormal(sw):
    say("generating the 1M log-normal workload")
    return aligned_set(sw, P.config_1m(1_000_000), "1M log-normal")


@pytest.fixture(scope="module")
def block(sw):
    say("generating the block all-vs-all workload (k-mer candidates)")
    return aligned_set(sw, P.config_block(), "block 50k x 50k")


@pytest.mark.parametrize("k", range(SLICES))
def test_lognormal_1m_every_pair(lognormal, k):
    check_slice(lognormal, k, "1M log-normal")


@pytest.mark.parametrize("k", range(SLICES))
def test_block_all_vs_all_every_pair(block, k):
    check_slice(block, k, "block 50k x 50k")


@pytest.fixture(scope="module")
def heavy(sw):
    say("generating chunk 0 of the heavy-tailed batching mix")
    ps = P.config_batching(P.CHUNK)
    L = ps.lengths().astype(np.int64)
    m, n = L[ps.pairs[:, 0]], L[ps.pairs[:, 1]]
    long_ = np.maximum(m, n) > 4096
    say("heavy tail shard: %d pairs (%d long), %.4g cells, longest %d" % (
        ps.n_pairs, int(long_.sum()), ps.cells(), L.max()))
    got = align(sw, ps, sw.PERSISTENT)
    say("heavy tail shard: aligned")
    check_properties(ps, got)
    long_idx = np.flatnonzero(long_)
    cost = (m * n)[long_idx]
    top = long_idx[np.argsort(cost)[-20:]]
    rest = np.setdiff1d(long_idx, top)
    rng = np.random.default_rng(13)
    pick = np.concatenate([top, rng.choice(rest, 480, replace=False)])
    assert len(np.unique(pick)) == 500
    say("heavy tail shard: 500 long pairs (20 costliest up to %d x %d), %.4g cells" % (
        int(m[top[-1]]), int(n[top[-1]]), float((m * n)[pick].sum())))
    return ps, got, np.flatnonzero(~long_), pick


def test_heavy_tail_short_pairs(heavy):
    ps, got, short_idx, _ = heavy
    assert_rows(got[short_idx], oracle_rows(ps, short_idx), short_idx, "heavy tail short pairs")
    say("heavy tail shard: all %d short pairs bit-exact" % len(short_idx))


@pytest.mark.parametrize("k", range(5))
def test_heavy_tail_long_pairs(heavy, k):
    """Slice k of the 500 long pairs (slice 0 holds the 20 costliest)."""
    ps, got, _, pick = heavy
    idx = np.sort(pick[100 * k:100 * (k + 1)])
    assert_rows(got[idx], oracle_rows(ps, idx), idx, "heavy tail long pairs, slice %d" % k)
    say("heavy tail shard: long pairs %d..%d bit-exact" % (100 * k, 100 * k + 99))
