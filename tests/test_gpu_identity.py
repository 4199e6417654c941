"""GPU identity / coverage pass (sw_identity) against the oracle.  The oracle
gets the oracle's own alignment results as its boxes; the GPU pass gets the
GPU aligner's (which equal them, and are checked to), so no expected value
comes from the HIP path."""
import numpy as np
import pytest

import oracle
from workloads import proteins as P

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def sw():
    import torch
    assert torch.cuda.is_available()
    import paper_2303_01845_amd as m
    return m


def run_both(sw, ps, go=11, ge=1, ani=300, cov=700, flags=None):
    import torch
    b = sw.Batch(ps.ascii, ps.offsets)
    pairs = torch.from_numpy(np.ascontiguousarray(ps.pairs, dtype=np.int32)).cuda()
    aligned = b.align(pairs, go, ge, sw.VALIDATE)
    got = sw.identity(b.packed, b.offsets, b.packed, b.offsets, pairs, aligned, go, ge, ani, cov,
                      flags=sw.VALIDATE if flags is None else flags).cpu().numpy()
    exp_aln = oracle.batch_ascii(ps.ascii, ps.offsets, ps.pairs, go, ge)
    assert (aligned.cpu().numpy() == exp_aln).all()
    exp = oracle.identity_ascii(ps.ascii, ps.offsets, ps.pairs, exp_aln, go, ge, ani, cov)
    return got, exp, exp_aln


def from_seqs(seqs_q, seqs_r):
    n = len(seqs_q)
    seqs = list(seqs_q) + list(seqs_r)
    asc = np.frombuffer("".join(seqs).encode(), dtype=np.uint8).copy()
    offs = np.zeros(len(seqs) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in seqs])
    pairs = np.stack([np.arange(n), np.arange(n) + n], 1).astype(np.int32)
    return P.PairSet(asc, offs, pairs, "custom")


def test_small_config_thresholds_and_gaps(sw):
    ps = P.config_small(400)
    for go, ge in ((11, 1), (2, 1), (5, 5), (1, 0)):
        for ani, cov in ((300, 700), (0, 0), (1000, 1000), (450, 300)):
            say("small go=%d ge=%d ani=%d cov=%d" % (go, ge, ani, cov))
            got, exp, aln = run_both(sw, ps, go, ge, ani, cov)
            assert np.array_equal(got, exp.astype(np.int32)), (go, ge, ani, cov)
            assert (got[aln[:, 0] > 0, 0] == aln[aln[:, 0] > 0, 0]).all()


def test_tie_heavy_and_multi_strip(sw):
    rng = np.random.default_rng(31)
    qs, rs = [], []
    for t in range(120):
        alpha = ["AC", "ACD", "W", "ARNDCQEGHILKMFPSTWYV"][t % 4]
        L = int(rng.integers(1, 260))
        q = "".join(rng.choice(list(alpha), L))
        # a mutated copy: substitutions and a few indels keep the box large
        r = list(q)
        for _ in range(int(rng.integers(0, 6))):
            p = int(rng.integers(0, len(r) + 1))
            if rng.random() < 0.5 and len(r) > 1:
                del r[min(p, len(r) - 1)]
            else:
                r.insert(p, str(rng.choice(list(alpha))))
        for _ in range(int(rng.integers(0, 10))):
            r[int(rng.integers(0, len(r)))] = str(rng.choice(list(alpha)))
        qs.append(q)
        rs.append("".join(r))
    ps = from_seqs(qs, rs)
    for go, ge in ((11, 1), (3, 1), (4, 4)):
        got, exp, _ = run_both(sw, ps, go, ge)
        assert np.array_equal(got, exp.astype(np.int32)), (go, ge)


def test_last_strip_rows_per_lane(sw):
    """Boxes just past one or two 256-row strips, whose last strip runs on 1,
    2 or 4 rows per lane after full strips on 4, with 32-bit keys (boxes up to
    511), exact 64-bit keys (larger ones) and the cut form (gap penalties too
    large for the exact forms): the oracle's records."""
    rng = np.random.default_rng(12)
    alpha = list("ARNDCQEGHILKMFPSTWYV")
    qs, rs = [], []
    for M in (257, 258, 300, 320, 321, 350, 384, 385, 449, 511, 512, 513, 577, 640, 641, 700, 769):
        for rate in (0.05, 0.3):
            q = "".join(rng.choice(alpha, M))
            r = list(q)
            for i in np.flatnonzero(rng.random(M) < rate):
                r[i] = str(rng.choice(alpha))
            qs.append(q)
            rs.append("".join(r))
    ps = from_seqs(qs, rs)
    for go, ge in ((11, 1), (10 ** 5, 10 ** 5)):
        got, exp, aln = run_both(sw, ps, go, ge)
        rows = aln[:, 2] - aln[:, 1] + 1
        say("last-strip boxes go=%d ge=%d: rows %d..%d" % (go, ge, rows.min(), rows.max()))
        assert np.array_equal(got, exp.astype(np.int32)), (go, ge)


def test_long_boxes(sw):
    rng = np.random.default_rng(8)
    L = "ARNDCQEGHILKMFPSTWYV"
    big = "".join(rng.choice(list(L), 12000))
    mid = "".join(rng.choice(list(L), 3000))
    mid2 = mid[:1000] + "".join(rng.choice(list(L), 7)) + mid[1000:2500] + mid[2510:]
    say("long: 12000 self, 3000 homolog")
    ps = from_seqs([big, mid, mid[500:2900]], [big, mid2, mid2])
    got, exp, aln = run_both(sw, ps)
    assert np.array_equal(got, exp.astype(np.int32))
    assert got[0].tolist()[1:] == [12000, 12000, 1]


def test_errors(sw):
    import torch
    ps = P.config_small(50)
    b = sw.Batch(ps.ascii, ps.offsets)
    pairs = torch.from_numpy(np.ascontiguousarray(ps.pairs, dtype=np.int32)).cuda()
    aligned = b.align(pairs, 11, 1, sw.VALIDATE)
    # a box whose score does not match
    bad = aligned.clone()
    k = int(torch.nonzero(bad[:, 0] > 0)[0])
    bad[k, 0] += 1
    with pytest.raises(sw.SwError) as e:
        sw.identity(b.packed, b.offsets, b.packed, b.offsets, pairs, bad, flags=sw.VALIDATE)
    assert e.value.status == sw.SW_ERANGE
    # coordinates past the sequence end
    bad = aligned.clone()
    bad[k, 2] = 70000
    with pytest.raises(sw.SwError) as e:
        sw.identity(b.packed, b.offsets, b.packed, b.offsets, pairs, bad, flags=sw.VALIDATE)
    assert e.value.status == sw.SW_ERANGE
    # a pair index out of range
    bp = pairs.clone()
    bp[k, 1] = ps.n_seqs + 5
    with pytest.raises(sw.SwError) as e:
        sw.identity(b.packed, b.offsets, b.packed, b.offsets, bp, aligned, flags=sw.VALIDATE)
    assert e.value.status == sw.SW_ERANGE
    # the library stays usable; score-0 pairs get zeros
    got = sw.identity(b.packed, b.offsets, b.packed, b.offsets, pairs, aligned, flags=sw.VALIDATE).cpu().numpy()
    a = aligned.cpu().numpy()
    assert (got[a[:, 0] == 0] == 0).all()
    assert (got[a[:, 0] > 0, 0] == a[a[:, 0] > 0, 0]).all()


def test_block_workload_full_size_sampled(sw):
    """All 921k candidate pairs of the 50k x 50k block set: every record's
    score equals the aligned score (checked on the device), matches <=
    columns; a stratified sample against the oracle."""
    import torch
    ps = P.config_block()
    b = sw.Batch(ps.ascii, ps.offsets)
    pairs = torch.from_numpy(np.ascontiguousarray(ps.pairs, dtype=np.int32)).cuda()
    aligned = b.align(pairs, 11, 1, sw.VALIDATE)
    got = sw.identity(b.packed, b.offsets, b.packed, b.offsets, pairs, aligned, flags=sw.VALIDATE).cpu().numpy()
    a = aligned.cpu().numpy()
    say("block: %d pairs, %d kept" % (len(got), int(got[:, 3].sum())))
    # coverage first: the same keep flags; swept pairs unchanged, the others -1
    cf = sw.identity(b.packed, b.offsets, b.packed, b.offsets, pairs, aligned,
                     flags=sw.VALIDATE | sw.COVERAGE_FIRST).cpu().numpy()
    assert np.array_equal(cf[:, 3], got[:, 3]) and np.array_equal(cf[:, 0], got[:, 0])
    swept = cf[:, 1] >= 0
    assert np.array_equal(cf[swept], got[swept])
    assert (cf[~swept, 1:3] == -1).all() and (got[~swept & (a[:, 0] > 0), 3] == 0).all()
    say("block: coverage-first sweeps %d of %d pairs" % (int(swept.sum()), len(cf)))
    pos = a[:, 0] > 0
    assert (got[pos, 0] == a[pos, 0]).all() and (got[~pos] == 0).all()
    assert (got[:, 1] <= got[:, 2]).all()
    box = (a[:, 2] - a[:, 1] + 1).astype(np.int64) * (a[:, 4] - a[:, 3] + 1)
    order = np.argsort(box)
    rng = np.random.default_rng(3)
    sample = np.unique(np.concatenate([order[-40:], rng.choice(len(a), 1500, replace=False)]))
    sub = ps.subset(sample)
    exp_aln = oracle.batch_ascii(sub.ascii, sub.offsets, sub.pairs, 11, 1)
    assert (a[sample] == exp_aln).all()
    exp = oracle.identity_ascii(sub.ascii, sub.offsets, sub.pairs, exp_aln, 11, 1, 300, 700)
    assert np.array_equal(got[sample], exp.astype(np.int32))
