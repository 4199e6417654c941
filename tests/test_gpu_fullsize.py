"""GPU parity at full workload sizes, in the configuration the benchmark
times (persistent form, HIP graph, default tuning): every pair checked
against properties that hold at any size, the persistent and plain forms
compared on all pairs, and a stratified sample (random pairs plus the
costliest ones) against the CPU oracle bit for bit."""
import os
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


def align_both(sw, ps):
    import torch
    b = sw.Batch(ps.ascii, ps.offsets)
    out = b.align(ps.pairs, 11, 1, sw.PERSISTENT)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    out = b.align(ps.pairs, 11, 1, sw.PLAIN, out=out)
    torch.cuda.synchronize()
    plain = out.cpu().numpy()
    return got, plain


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


def sample_indices(ps, n_random, n_top, seed):
    cost = ps.lengths().astype(np.int64)
    cost = cost[ps.pairs[:, 0]] * cost[ps.pairs[:, 1]]
    rng = np.random.default_rng(seed)
    pick = rng.choice(ps.n_pairs, min(n_random, ps.n_pairs), replace=False)
    top = np.argsort(cost)[-n_top:]
    return np.unique(np.concatenate([pick, top, [0, ps.n_pairs - 1]]))


def run(sw, ps, label, n_random, n_top, seed):
    say("%s: %d pairs, %.3g cells, longest %d" % (label, ps.n_pairs, ps.cells(), ps.lengths().max()))
    got, plain = align_both(sw, ps)
    say("%s: aligned" % label)
    check_properties(ps, got)
    diff = np.flatnonzero((got != plain).any(axis=1))
    assert len(diff) == 0, "%s: persistent and plain differ on %d pairs (first %d)" % (label, len(diff), diff[0])
    idx = sample_indices(ps, n_random, n_top, seed)
    sub = ps.subset(idx)
    exp = oracle.batch_ascii(sub.ascii, sub.offsets, sub.pairs, 11, 1, threads=min(16, os.cpu_count() or 1))
    bad = np.flatnonzero((got[idx] != exp).any(axis=1))
    say("%s: %d sampled pairs checked" % (label, len(idx)))
    assert len(bad) == 0, "%s: pair %d differs: gpu %s oracle %s" % (
        label, idx[bad[0]], got[idx[bad[0]]].tolist(), exp[bad[0]].tolist())


def test_lognormal_1m_full_size(sw):
    say("generating the 1M log-normal workload")
    run(sw, P.config_1m(1_000_000), "1M log-normal", 1500, 200, 11)


def test_block_all_vs_all_full_size(sw):
    say("generating the block all-vs-all workload (k-mer candidates)")
    run(sw, P.config_block(), "block 50k x 50k", 1500, 200, 12)


def test_heavy_tail_sampled(sw):
    # the heavy-tail length mix (5% of pairs 5,000-35,000 residues) at 20,000
    # pairs; the full 10M-pair set holds ~26 G residues on the host
    say("generating the heavy-tail workload")
    run(sw, P.config_batching(20_000), "heavy tail 20k", 400, 12, 13)
