"""Seeded synthetic workloads (no GPU): shapes, distributions, determinism."""
import numpy as np

from workloads import proteins as P


def test_small_config_shape():
    s = P.config_small()
    assert s.n_pairs == 1000 and s.n_seqs == 2000
    L = s.lengths()
    q = L[0::2]
    assert q.min() >= 50 and q.max() <= 300
    assert L[1:1000:2].min() >= 50 and L[1:1000:2].max() <= 300     # unrelated refs
    assert set(np.unique(s.ascii).tobytes()) <= set(P.AA20)
    # homolog refs keep roughly the query length (5% indels)
    hq, hr = L[1000::2], L[1001::2]
    assert np.abs(hr - hq).mean() < 0.1 * hq.mean()


def test_background_frequencies():
    rng = P.rng_for(99, 0)
    x = P.background(rng, 400000)
    freq = np.array([(x == c).mean() for c in P.AA20])
    assert np.abs(freq - P.BACKGROUND).max() < 0.003


def test_mutation_model():
    rng = P.rng_for(98, 0)
    L = np.full(2000, 200)
    src, offs = P._from_lengths(rng, L)
    same, so = P.mutate_many(P.rng_for(98, 1), src, offs, 0.0, 0.0)
    assert (same == src).all() and (so == offs).all()
    sub, so = P.mutate_many(P.rng_for(98, 2), src, offs, 1.0, 0.0)
    assert (so == offs).all() and not (sub == src).any()
    half, so = P.mutate_many(P.rng_for(98, 3), src, offs, 0.3, 0.0)
    assert abs((half != src).mean() - 0.3) < 0.01
    ind, io = P.mutate_many(P.rng_for(98, 4), src, offs, 0.0, 0.3)
    d = np.diff(io) - 200
    assert d.std() > 3 and np.diff(io).min() >= 1


def test_determinism_and_prefix():
    a = P.config_1m(1000, workers=1)
    b = P.config_1m(1000, workers=1)
    assert (a.ascii == b.ascii).all() and (a.pairs == b.pairs).all()
    c = P.config_1m(P.CHUNK + 10, workers=2)
    k = a.offsets[-1]
    assert (c.ascii[:k] == a.ascii).all()
    L = c.lengths()[0::2]
    assert 250 < np.median(L) < 310 and L.min() >= 30 and L.max() <= 5000


def test_heavy_tail_mix():
    b = P.config_batching(400, workers=1)
    q = b.lengths()[0::2]
    longp = q >= 5000
    assert 0.01 < longp.mean() < 0.12
    assert q[longp].max() <= 35000


def test_shared_kmer_candidates():
    asc, offs, fam = P.families(77, 20, 200)
    q = np.arange(0, 200, 2)
    r = np.arange(1, 200, 2)
    L = np.diff(offs)

    def take(ix):
        o = np.zeros(len(ix) + 1, np.int64)
        np.cumsum(L[ix], out=o[1:])
        return asc[P.gather_segments(offs[ix], L[ix])], o

    qa, qo = take(q)
    ra, ro = take(r)
    qq, rr, shared = P.shared_kmer_pairs(qa, qo, ra, ro)
    assert len(qq) > 0

    def kmers(a, o, i):
        s = a[o[i]:o[i + 1]].tobytes()
        return {s[t:t + 6] for t in range(len(s) - 5)}

    got = set(zip(qq.tolist(), rr.tolist()))
    rng = np.random.default_rng(0)
    for i in rng.choice(len(q), 30, replace=False):
        for j in range(len(r)):
            k = len(kmers(qa, qo, i) & kmers(ra, ro, j))
            assert ((i, j) in got) == (k >= 2)


def test_c3_lpt_shard_is_the_seeded_chunks():
    """The query lengths the LPT assignment replays are those of the chunks
    config_batching draws, and the shards split the chunks exactly once."""
    L = P._c3_query_lengths((5, 300, 0.05))
    b = P.config_batching(300, first_chunk=5, workers=1)
    assert (b.lengths()[b.pairs[:, 0]] == L).all()
    shards, load, cost = P.c3_lpt_shards(3, n_pairs=5 * P.CHUNK + 1000, workers=1)
    assert sorted(c for s in shards for c in s) == list(range(6))
    assert abs(load.sum() - cost.sum()) < 1e-6 * cost.sum()
    assert load.max() - load.min() <= cost.max()
