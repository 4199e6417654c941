"""GPU candidate discovery (sw_discover) against the oracle: the set of
(query, reference, shared k-mer count) triples must be identical; the order
of the output is unspecified, so both sides are sorted before comparing."""
import numpy as np
import pytest

import oracle
from workloads import proteins as P

pytestmark = pytest.mark.gpu

LETTERS = "ARNDCQEGHILKMFPSTWYV"


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def sw():
    import torch
    assert torch.cuda.is_available()
    import paper_2303_01845_amd as m
    return m


def pack_set(seqs):
    asc = np.frombuffer("".join(seqs).encode(), dtype=np.uint8).copy()
    offs = np.zeros(len(seqs) + 1, dtype=np.int64)
    offs[1:] = np.cumsum([len(s) for s in seqs])
    return asc, offs


def on_gpu(sw, asc, offs):
    import torch
    return sw.pack(asc if len(asc) else b""), torch.from_numpy(offs).cuda()


def gpu_triples(sw, qp, qo, rp, ro, k, t, mode=0, capacity=None, budget=0):
    pairs, shared = sw.discover(qp, qo, rp, ro, k, t, mode, capacity, budget)
    a = np.concatenate([pairs.cpu().numpy().reshape(-1, 2), shared.cpu().numpy().reshape(-1, 1)], 1)
    return a[np.lexsort((a[:, 1], a[:, 0]))] if len(a) else a.reshape(0, 3)


def oracle_triples(qa, qo, ra, ro, k, t, mode=0):
    q, r, c = oracle.discover(qa, qo, ra, ro, k, t, mode)
    return np.stack([q, r, c], 1).astype(np.int32)


def rand_set(rng, n, alpha, lo, hi):
    return ["".join(rng.choice(list(alpha), size=int(rng.integers(lo, hi + 1)))) for _ in range(n)]


def test_small_sets_every_mode(sw):
    rng = np.random.default_rng(2024)
    for alpha, lo, hi in (("AC", 0, 40), ("ACDE", 0, 90), (LETTERS, 0, 300), ("W", 0, 12)):
        qs = rand_set(rng, 70, alpha, lo, hi)
        rs = rand_set(rng, 130, alpha, lo, hi)
        qa, qo = pack_set(qs)
        ra, ro = pack_set(rs)
        qp, qod = on_gpu(sw, qa, qo)
        rp, rod = on_gpu(sw, ra, ro)
        for k in (1, 2, 3, 6):
            for t in (1, 2, 3):
                say("set alpha=%s k=%d t=%d" % (alpha, k, t))
                got = gpu_triples(sw, qp, qod, rp, rod, k, t)
                exp = oracle_triples(qa, qo, ra, ro, k, t)
                assert np.array_equal(got, exp), (alpha, k, t)
                for mode in (1, 2):
                    got = gpu_triples(sw, rp, rod, rp, rod, k, t, mode)
                    exp = oracle_triples(ra, ro, ra, ro, k, t, mode)
                    assert np.array_equal(got, exp), (alpha, k, t, mode)


def test_edges(sw):
    import torch
    # sequences shorter than k, empty ones, a single query, identical copies
    qs = ["", "ACDEF", "ACDEFG", "W" * 50, "ACDEFGHIKL"]
    rs = ["ACDEFG", "", "ACDEFGHIKL", "W" * 6, "W" * 5, "ACDEFGHIKL", "GHIKLACDEF"]
    qa, qo = pack_set(qs)
    ra, ro = pack_set(rs)
    qp, qod = on_gpu(sw, qa, qo)
    rp, rod = on_gpu(sw, ra, ro)
    for k in (1, 5, 6):
        for t in (1, 2):
            assert np.array_equal(gpu_triples(sw, qp, qod, rp, rod, k, t), oracle_triples(qa, qo, ra, ro, k, t))
    one = torch.from_numpy(qo[-2:].copy()).cuda()  # the last query alone
    got = gpu_triples(sw, qp, one, rp, rod, 6, 1)
    exp = oracle_triples(qa[qo[-2]:], qo[-2:] - qo[-2], ra, ro, 6, 1)
    assert np.array_equal(got, exp)
    # nothing shared, empty sets
    assert len(gpu_triples(sw, qp, qod, rp, rod, 6, 99)) == 0
    e = torch.zeros(1, dtype=torch.int64, device="cuda")
    assert len(gpu_triples(sw, qp, e, rp, rod, 6, 1)) == 0


def test_capacity_and_errors(sw):
    import ctypes
    import torch
    rng = np.random.default_rng(9)
    rs = rand_set(rng, 200, "ACD", 20, 60)
    ra, ro = pack_set(rs)
    rp, rod = on_gpu(sw, ra, ro)
    exp = oracle_triples(ra, ro, ra, ro, 3, 2, 1)
    n = len(exp)
    assert n > 100
    L = sw.lib()
    found = ctypes.c_int64()
    args = (ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(rod.data_ptr()), len(rs),
            ctypes.c_void_p(rp.data_ptr()), ctypes.c_void_p(rod.data_ptr()), len(rs), 3, 2, 1)
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    assert L.sw_discover(*args, None, None, 0, ctypes.byref(found), 0, st) == sw.SW_ENOMEM
    assert found.value == n
    buf = torch.full((n, 2), -7, dtype=torch.int32, device="cuda")
    assert L.sw_discover(*args, ctypes.c_void_p(buf.data_ptr()), None, n - 10, ctypes.byref(found),
                         0, st) == sw.SW_ENOMEM
    assert found.value == n
    got = buf[:n - 10].cpu().numpy()
    assert (buf[n - 10:].cpu().numpy() == -7).all()            # nothing beyond the capacity
    assert set(map(tuple, got)) <= set(map(tuple, exp[:, :2]))  # a subset of the answer
    assert len(set(map(tuple, got))) == n - 10
    # exact capacity, no shared counts requested
    assert L.sw_discover(*args, ctypes.c_void_p(buf.data_ptr()), None, n, ctypes.byref(found), 0, st) == sw.SW_OK
    assert set(map(tuple, buf.cpu().numpy())) == set(map(tuple, exp[:, :2]))
    # offsets that run backwards, or past the packed residues
    bad = rod.clone()
    bad[5] = bad[3]
    bad[4] = bad[3] + 1000
    with pytest.raises(sw.SwError) as e:
        sw.discover(rp, bad, rp, rod, 3, 2)
    assert e.value.status == sw.SW_ERANGE
    bad = rod.clone()
    bad[-1] = int(ro[-1]) + 1
    with pytest.raises(sw.SwError) as e:
        sw.discover(rp, rod, rp, bad, 3, 2)
    assert e.value.status == sw.SW_ERANGE
    # a letter that is not a residue symbol (the packer flags it too)
    ja, jo = pack_set(["ACDEFGHIK", "ACDJFGHIK"])
    jp, jod = on_gpu(sw, ja, jo)
    with pytest.raises(sw.SwError) as e:
        sw.discover(jp, jod, jp, jod, 3, 1)
    assert e.value.status == sw.SW_ECODE
    with pytest.raises(sw.SwError):
        sw.check()  # the packer's flag of the same letter
    # the error paths leave the library usable
    assert np.array_equal(gpu_triples(sw, rp, rod, rp, rod, 3, 2, 1), exp)


def test_heavy_lists(sw):
    # 300 copies of one sequence: every k-mer list holds 300 references
    rng = np.random.default_rng(4)
    base = rand_set(rng, 1, LETTERS, 400, 400)[0]
    seqs = [base] * 300 + rand_set(rng, 200, LETTERS, 100, 400)
    a, o = pack_set(seqs)
    p, od = on_gpu(sw, a, o)
    p2, od2 = on_gpu(sw, a, o)  # the same set in a second buffer: not recognised as a self search
    for mode in (0, 1, 2):
        say("heavy mode=%d" % mode)
        exp = oracle_triples(a, o, a, o, 6, 2, mode)
        assert np.array_equal(gpu_triples(sw, p, od, p, od, 6, 2, mode), exp)
        assert np.array_equal(gpu_triples(sw, p, od, p2, od2, 6, 2, mode), exp)


def test_block_all_vs_all_full_size(sw):
    """The 2,000-family, 50k x 50k block workload: every candidate against the
    oracle, and the candidate list equals the one its generator builds."""
    import torch
    ps = P.config_block()
    nq = (ps.n_seqs + 1) // 2
    say("block: %d queries, %d references, %d generator pairs" % (nq, ps.n_seqs - nq, ps.n_pairs))
    offs = ps.offsets
    packed = sw.pack(ps.ascii)
    qo = torch.from_numpy(offs[:nq + 1].copy()).cuda()
    ro = torch.from_numpy(offs[nq:].copy()).cuda()
    got = gpu_triples(sw, packed, qo, packed, ro, 6, 2)
    cut = int(offs[nq])
    exp = oracle_triples(ps.ascii[:cut], offs[:nq + 1], ps.ascii[cut:], offs[nq:] - cut, 6, 2)
    say("block: %d candidates" % len(exp))
    assert np.array_equal(got, exp)
    gen = ps.pairs.astype(np.int64)
    gen = gen[np.lexsort((gen[:, 1], gen[:, 0]))]
    assert np.array_equal(got[:, :2], np.stack([gen[:, 0], gen[:, 1] - nq], 1))


def test_budget_splits_the_join(sw):
    """A small pair-table budget forms the product query range by query range;
    the result is the same set (here and on the full block set)."""
    import torch
    rng = np.random.default_rng(12)
    rs = rand_set(rng, 300, "ACDE", 20, 120)
    ra, ro = pack_set(rs)
    rp, rod = on_gpu(sw, ra, ro)
    for mode in (0, 1, 2):
        exp = oracle_triples(ra, ro, ra, ro, 3, 2, mode)
        for budget in (1, 4096, 1 << 16):
            assert np.array_equal(gpu_triples(sw, rp, rod, rp, rod, 3, 2, mode, budget=budget), exp), (mode, budget)
    ps = P.config_block()
    nq = (ps.n_seqs + 1) // 2
    packed = sw.pack(ps.ascii)
    qo = torch.from_numpy(ps.offsets[:nq + 1].copy()).cuda()
    ro = torch.from_numpy(ps.offsets[nq:].copy()).cuda()
    full = gpu_triples(sw, packed, qo, packed, ro, 6, 2)
    for budget in (64 << 20, 8 << 20):
        say("block with a %d MiB table budget" % (budget >> 20))
        assert np.array_equal(gpu_triples(sw, packed, qo, packed, ro, 6, 2, budget=budget), full)
