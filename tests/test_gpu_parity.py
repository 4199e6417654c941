"""GPU parity: the HIP path (through the C ABI) against the CPU oracle, bit for
bit on all five int32 outputs, on seeded synthetic inputs."""
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


def gpu_align(sw, ps, go=11, ge=1, flags=0):
    import torch
    b = sw.Batch(ps.ascii, ps.offsets)
    out = b.align(ps.pairs, go, ge, flags)
    torch.cuda.synchronize()
    return out.cpu().numpy()


def expect(ps, go=11, ge=1):
    return oracle.batch_ascii(ps.ascii, ps.offsets, ps.pairs, go, ge)


def assert_same(got, exp, ps, label):
    bad = np.flatnonzero((got != exp).any(axis=1))
    if len(bad):
        k = int(bad[0])
        q, r = ps.pairs[k]
        L = ps.lengths()
        raise AssertionError("%s: %d of %d pairs differ; first pair %d (m=%d n=%d): gpu %s oracle %s"
                             % (label, len(bad), len(got), k, L[q], L[r], got[k].tolist(),
                                exp[k].tolist()))


def pairset_from_strings(pairs_str):
    seqs = []
    for q, r in pairs_str:
        seqs += [q, r]
    L = np.array([len(s) for s in seqs], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(L)])
    asc = np.frombuffer(("".join(seqs)).encode(), dtype=np.uint8).copy()
    prs = np.arange(2 * len(pairs_str), dtype=np.int32).reshape(-1, 2)
    return P.PairSet(asc, offs, prs, "strings")


def test_small_config_all_forms(sw):
    ps = P.config_small()
    exp = expect(ps)
    for flags, label in [(0, "persistent+graph"), (sw.NO_GRAPH, "persistent"), (sw.PLAIN, "plain")]:
        say("small config, %s" % label)
        assert_same(gpu_align(sw, ps, flags=flags), exp, ps, label)


def test_golden_fixture_cases(sw):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "oracle_cases.tsv")
    rows = [l.rstrip("\n").split("\t") for l in open(path) if l.strip() and not l.startswith("#")]
    by_gap = {}
    for q, r, go, ge, *e in rows:
        by_gap.setdefault((int(go), int(ge)), []).append((q, r, [int(x) for x in e]))
    for (go, ge), cases in by_gap.items():
        say("golden cases gap %d/%d" % (go, ge))
        ps = pairset_from_strings([(q, r) for q, r, _ in cases])
        got = gpu_align(sw, ps, go, ge)
        assert_same(got, np.array([e for _, _, e in cases], dtype=np.int32), ps, "golden")


def adversarial_set(seed, n, max_len):
    rng = np.random.default_rng(seed)
    letters = np.frombuffer(b"ARNDCQEGHILKMFPSTWYVBZX*", dtype=np.uint8)
    out = []
    for t in range(n):
        kind = t % 6
        m, nn = (int(x) for x in rng.integers(1, max_len + 1, 2))
        if kind == 0:
            a = letters[rng.integers(0, 24)]
            q, r = bytes([a]) * m, bytes([a]) * nn
        elif kind == 1:
            ab = rng.choice(letters[:20], 2, replace=False)
            q, r = rng.choice(ab, m).tobytes(), rng.choice(ab, nn).tobytes()
        elif kind == 2:
            u = rng.choice(letters[:20], int(rng.integers(1, 6))).tobytes()
            q, r = (u * (max_len // len(u) + 2))[:m], (u * (max_len // len(u) + 2))[1:nn + 1]
        elif kind == 3:
            q = rng.choice(letters, int(rng.integers(1, 4))).tobytes()
            r = rng.choice(letters, int(rng.integers(1, 4))).tobytes()
        elif kind == 4:
            q = rng.choice(letters[:20], m).tobytes()
            r = q[: nn // 2] + rng.choice(letters[:20], int(rng.integers(1, 9))).tobytes() + q[nn // 2:]
        else:
            q, r = rng.choice(letters, m).tobytes(), rng.choice(letters, nn).tobytes()
        out.append((q.decode(), r.decode()))
    return pairset_from_strings(out)


@pytest.mark.parametrize("gaps", [(11, 1), (2, 1), (1, 0), (3, 3), (11, 2), (10 ** 6, 10 ** 6)])
def test_adversarial_short(sw, gaps):
    ps = adversarial_set(100 + gaps[0], 700, 300)
    say("adversarial short gap %s" % (gaps,))
    assert_same(gpu_align(sw, ps, *gaps), expect(ps, *gaps), ps, "adversarial %s" % (gaps,))


def test_adversarial_long_wide(sw):
    # every pair longer than the short-pair limit: the wide variant (32-bit
    # boundary cells, folded 12-bit column tags)
    ps = adversarial_set(7, 36, 3000)
    keep = [k for k in range(ps.n_pairs) if max(ps.lengths()[ps.pairs[k]]) > 1024]
    ps = ps.subset(keep)
    say("adversarial long: %d pairs" % ps.n_pairs)
    for gaps in [(11, 1), (2, 1)]:
        assert_same(gpu_align(sw, ps, *gaps), expect(ps, *gaps), ps, "long %s" % (gaps,))


def test_lognormal_prefix_full_parity(sw):
    ps = P.config_1m(65536)
    say("lognormal prefix: %d pairs %.2f Gcells" % (ps.n_pairs, ps.cells() / 1e9))
    exp = expect(ps)
    assert_same(gpu_align(sw, ps), exp, ps, "lognormal persistent")
    assert_same(gpu_align(sw, ps, flags=sw.PLAIN), exp, ps, "lognormal plain")


def test_heavy_tail_mix(sw):
    ps = P.config_batching(1500)
    say("heavy tail: %d pairs %.2f Gcells, longest %d" % (ps.n_pairs, ps.cells() / 1e9,
                                                          ps.lengths().max()))
    assert_same(gpu_align(sw, ps), expect(ps), ps, "heavy tail")


def test_tuning_does_not_change_results(sw):
    ps = P.concat([P.config_small(), adversarial_set(3, 300, 1500)])
    ref = None
    try:
        for R, im, bpc, g16, g8 in [(16, 1024, 0, 2048, 1024), (8, 512, 0, 1024, 64), (16, 64, 0, 64, 64),
                                    (8, 256, 2, 4096, 512), (16, 512, 1, 512, 4096), (8, 64, 3, 2048, 128),
                                    (16, 768, 0, 4096, 2048), (16, 64, -1, 4096, 256)]:
            sw.set_tuning(R, im, bpc, g16, g8)
            say("tuning R=%d inter_max=%d bpc=%d group16_max=%d group8_max=%d" % (R, im, bpc, g16, g8))
            got = gpu_align(sw, ps)
            if ref is None:
                ref = got
                assert_same(got, expect(ps), ps, "tuning reference")
            assert (got == ref).all(), (R, im, bpc)
    finally:
        sw.set_tuning(16, 1024, -1, 2048, 2048)


def test_permuted_pairs(sw):
    ps = P.config_small()
    rng = np.random.default_rng(9)
    perm = rng.permutation(ps.n_pairs)
    ps2 = P.PairSet(ps.ascii, ps.offsets, ps.pairs[perm].copy(), "perm")
    a = gpu_align(sw, ps)
    b = gpu_align(sw, ps2)
    assert (a[perm] == b).all()


def test_empty_invalid_and_bad_residues(sw):
    import torch
    seqs = ["", "ACDEFGHIK", "WWWW", "MKV"]
    L = np.array([len(s) for s in seqs], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(L)])
    asc = np.frombuffer("".join(seqs).encode(), dtype=np.uint8).copy()
    pairs = np.array([[0, 1], [1, 0], [2, 2], [1, 4], [-1, 2], [3, 1]], dtype=np.int32)
    b = sw.Batch(asc, offs)
    with pytest.raises(sw.SwError) as e:
        b.align(pairs, flags=sw.VALIDATE)
    assert e.value.status == sw.SW_ERANGE
    out = b.align(pairs).cpu().numpy()
    with pytest.raises(sw.SwError) as e:      # raised again by the non-validating call
        sw.check()
    assert e.value.status == sw.SW_ERANGE
    sw.check()                                 # and cleared by the check
    assert out[0].tolist() == [0, -1, -1, -1, -1]
    assert out[1].tolist() == [0, -1, -1, -1, -1]
    assert out[2].tolist() == [44, 0, 3, 0, 3]
    assert out[3].tolist() == [-1] * 5 and out[4].tolist() == [-1] * 5
    assert tuple(out[5]) == oracle.align(b"MKV", b"ACDEFGHIK")


def test_invalid_residue_reported(sw):
    with pytest.raises(sw.SwError) as e:
        sw.Batch(np.frombuffer(b"ACDJKL", dtype=np.uint8), np.array([0, 3, 6])).align(
            np.array([[0, 1]], dtype=np.int32), flags=sw.VALIDATE)
    assert e.value.status == sw.SW_ECODE


def test_maximum_length_pairs(sw):
    rng = np.random.default_rng(11)
    a = P.background(rng, 65535)
    b = np.concatenate([a[30000:30400], P.background(rng, 100)])
    c = P.background(rng, 20)
    seqs = [a, b, c]
    L = np.array([len(s) for s in seqs], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(L)])
    ps = P.PairSet(np.concatenate(seqs), offs, np.array([[0, 1], [1, 0], [0, 2], [2, 0]], np.int32), "max")
    say("maximum length pairs")
    assert_same(gpu_align(sw, ps), expect(ps), ps, "max length")


def _self_score_sequence(rng, M, target, length_hint=14000):
    """A sequence whose BLOSUM62 self-score (the sum of its diagonal entries)
    is exactly `target`: a background prefix, then residues of diagonal score
    4 and one of 4..7 to make up the rest."""
    a = P.background(rng, length_hint)
    d = M[oracle.encode(a), oracle.encode(a)].astype(np.int64)
    cut = int(np.searchsorted(np.cumsum(d), target - 40))
    rest = target - int(d[:cut].sum())
    k, rem = divmod(rest, 4)
    fill = {4: "A", 5: "R", 6: "N", 7: "P"}
    for v, ch in fill.items():
        c = int(oracle.encode(np.frombuffer(ch.encode(), dtype=np.uint8))[0])
        assert M[c, c] == v
    tail = "A" * (k - 1) + fill[4 + rem]
    return np.concatenate([a[:cut], np.frombuffer(tail.encode(), dtype=np.uint8)])


def test_packed_overflow_long_pairs(sw):
    # Whole-wave pairs run their forward pass in 16-bit cells with saturating
    # additions and fall back to int32 when a strip's maximum passes 65504.
    # Identical pairs with self-scores on either side of that limit (and of
    # the 16-bit ceiling), plus mutated pairs with gaps, all beyond the
    # 4096-residue packed limit of the smaller groups.
    rng = np.random.default_rng(21)
    M = oracle.matrix()
    seqs = []
    for t in (65503, 65504, 65505, 65535, 65536, 65540):
        x = _self_score_sequence(rng, M, t)
        seqs += [x, x.copy()]
    for L, rate in [(11000, 0.02), (12500, 0.01), (13400, 0.03), (16000, 0.05)]:
        a = P.background(rng, L)
        b = a.copy()
        hit = rng.random(L) < rate
        b[hit] = P.background(rng, int(hit.sum()))
        for _ in range(6):
            p = int(rng.integers(100, len(b) - 100))
            if rng.random() < 0.5:
                b = np.concatenate([b[:p], P.background(rng, int(rng.integers(1, 12))), b[p:]])
            else:
                b = np.concatenate([b[:p], b[p + int(rng.integers(1, 12)):]])
        seqs += [a, b]
    L = np.array([len(s) for s in seqs], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(L)])
    n = len(seqs) // 2
    pairs = np.arange(2 * n, dtype=np.int32).reshape(-1, 2)
    pairs = np.concatenate([pairs, pairs[:, ::-1]]).astype(np.int32)
    ps = P.PairSet(np.concatenate(seqs), offs, pairs, "overflow")
    exp = expect(ps)
    assert exp[:6, 0].tolist() == [65503, 65504, 65505, 65535, 65536, 65540]
    assert (exp[:, 0] <= 65504).sum() >= 4 and (exp[:, 0] > 65504).sum() >= 4
    say("packed overflow: %d pairs, scores %s" % (ps.n_pairs, exp[:n, 0].tolist()))
    assert_same(gpu_align(sw, ps), exp, ps, "packed overflow")


def planted_one_lane_set(seed):
    """One-lane pairs (16 query rows per super-strip) whose best cell lies in a
    chosen super-strip of the forward pass, at every distance from the pair's
    last super-strip: a reference segment copied into the query so that the
    copy ends in that super-strip; a weaker copy above or below a stronger
    one (the best row moves down, or stays while later super-strips pass);
    and exact ties (the reference is the segment itself, copied two or three
    times into the query: the first copy's cell must be reported)."""
    rng = np.random.default_rng(seed)
    seqs = []

    def plant(q, r, a, L, e):
        q[e - L + 1:e + 1] = r[a:a + L]

    for n_ss in range(1, 11):
        for s in range(n_ss):
            for variant in ("one", "higher_later", "lower_later", "tie"):
                m = int(16 * n_ss - rng.integers(0, 16))
                if s * 16 > m - 1:
                    continue
                e = int(rng.integers(16 * s, min(16 * s + 16, m)))
                q = P.background(rng, m)
                if variant == "tie":
                    L = min(24, e + 1)
                    r = P.background(rng, L)
                    plant(q, r, 0, L, e)
                    for s2 in range(s + 2, n_ss, 2):
                        e2 = min(16 * s2 + int(rng.integers(0, 16)), m - 1)
                        if e2 - L + 1 > e + 16:
                            plant(q, r, 0, L, e2)
                else:
                    n = int(rng.integers(60, 1000))
                    r = P.background(rng, n)
                    L = min(24, e + 1, n)
                    plant(q, r, int(rng.integers(0, n - L + 1)), L, e)
                    d = int(rng.integers(1, 6))
                    if variant != "one" and s + d < n_ss:
                        e2 = min(16 * (s + d) + int(rng.integers(0, 16)), m - 1)
                        L2 = 30 if variant == "higher_later" else 10
                        L2 = min(L2, e2 - e - 1, n)
                        if L2 >= 6:
                            plant(q, r, int(rng.integers(0, n - L2 + 1)), L2, e2)
                seqs += [q, r]
    L = np.array([len(x) for x in seqs], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(L)])
    prs = np.arange(len(seqs), dtype=np.int32).reshape(-1, 2)
    return P.PairSet(np.concatenate(seqs), offs, prs, "planted one-lane")


def test_one_lane_best_row_positions(sw):
    """The one-lane forward pass keeps its best super-strip's input row in a
    ring of four boundary buffers, copied aside when a later super-strip
    would overwrite it; planted best cells at every distance from the end,
    moving and staying picks and exact ties give the oracle's five outputs
    (two seeds, both pair orders)."""
    for seed in (41, 42):
        ps = planted_one_lane_set(seed)
        L = ps.lengths()
        assert max(L.max(), 0) <= 1024
        exp = expect(ps)
        say("planted one-lane set %d: %d pairs, scores %d..%d" % (seed, ps.n_pairs, exp[:, 0].min(),
                                                                   exp[:, 0].max()))
        assert_same(gpu_align(sw, ps, flags=sw.VALIDATE), exp, ps, "planted one-lane %d" % seed)
        rev = P.PairSet(ps.ascii, ps.offsets, ps.pairs[:, ::-1].copy(), "planted reversed")
        assert_same(gpu_align(sw, rev, flags=sw.VALIDATE), expect(rev), rev, "planted reversed %d" % seed)


def test_two_sets_match_one_set(sw):
    import torch
    ps = P.config_small(300)
    # queries = even sequences, references = odd sequences, in separate buffers
    L = ps.lengths()
    q_idx, r_idx = np.arange(0, ps.n_seqs, 2), np.arange(1, ps.n_seqs, 2)

    def take(ix):
        o = np.concatenate([[0], np.cumsum(L[ix])])
        return ps.ascii[P.gather_segments(ps.offsets[ix], L[ix])], o

    qa, qo = take(q_idx)
    ra, ro = take(r_idx)
    rng = np.random.default_rng(4)
    pairs = np.stack([rng.integers(0, len(q_idx), 500), rng.integers(0, len(r_idx), 500)], 1).astype(np.int32)
    qb, rb = sw.Batch(qa, qo), sw.Batch(ra, ro)
    got = sw.align_sets(qb.packed, qb.offsets, rb.packed, rb.offsets, torch.from_numpy(pairs).cuda()).cpu().numpy()
    one = P.PairSet(ps.ascii, ps.offsets, np.stack([q_idx[pairs[:, 0]], r_idx[pairs[:, 1]]], 1).astype(np.int32))
    assert_same(got, expect(one), one, "two sets")


def test_timed_calls(sw):
    """SW_TIMED changes no result; the timing read counts every timed call of
    each form once and then forgets them."""
    import torch
    ps = P.config_small(300)
    exp = expect(ps)
    stream = torch.cuda.current_stream()
    sw.timing_read(stream)
    for flags, label in [(0, "persistent+graph"), (sw.NO_GRAPH, "persistent"), (sw.PLAIN, "plain")]:
        say("timed, %s" % label)
        outer = 0.0
        for _ in range(2):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            got = gpu_align(sw, ps, flags=flags | sw.TIMED)
            e1.record(stream)
            torch.cuda.synchronize()
            outer += e0.elapsed_time(e1)
            assert_same(got, exp, ps, "timed " + label)
        if flags == sw.PLAIN:
            ms, calls = sw.timing_read(stream)
        else:
            fwd, start, calls = sw.timing_read_passes(stream)
            assert fwd > 0.0 and start > 0.0, (label, fwd, start)
            ms = fwd + start
        assert calls == 2 and ms > 0.0, (label, ms, calls)
        # the library's events sit inside the calls: their sum cannot exceed
        # the time between events recorded around the calls
        assert ms <= outer * 1.02 + 0.02, (label, ms, outer)
        assert sw.timing_read(stream) == (0.0, 0)
