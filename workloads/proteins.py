"""Seeded synthetic protein workloads shared by the tests, the smoke check and the
benchmark.  Holds no alignment arithmetic: it only draws residues, lengths,
mutations and candidate lists.

The paper's dataset (Metaclust, section "Similarity search at scale") is not
available, and it prints no length or identity distribution; these generators
stand in for it with the workload shapes the benchmark configurations name:

* residues are i.i.d. over the 20 standard amino acids at background
  frequencies (Robinson & Robinson 1991, renormalised);
* a homolog is made by ``mutate``: each position is substituted with
  probability ``s`` by a different background residue, then
  Binomial(len, rho/3) indel events are placed uniformly, each an insertion or
  a deletion with probability 1/2 and of length U{1..5} (mean 3, so about rho
  of the residues take part); inserted residues are background draws;
* every draw comes from ``numpy.random.Generator(PCG64(SeedSequence([1845,
  config, chunk])))`` so a chunk of pairs can be regenerated on its own.

Sequences are returned as one ASCII byte buffer plus int64 offsets
(``offsets[k]..offsets[k+1]`` is sequence k), and candidate pairs as int32
``[n_pairs, 2]`` (query index, reference index).
"""
from __future__ import annotations

import concurrent.futures
import dataclasses
import multiprocessing
import os

import numpy as np

AA20 = b"ARNDCQEGHILKMFPSTWYV"
_FREQ = np.array([.074, .052, .045, .053, .025, .034, .054, .074, .026, .068,
                  .099, .058, .025, .047, .039, .057, .051, .013, .032, .073])
BACKGROUND = _FREQ / _FREQ.sum()
_CDF = np.cumsum(BACKGROUND)
_CDF[-1] = 1.0
_LETTERS = np.frombuffer(AA20, dtype=np.uint8)
# Background draws use a 2^16-entry table: entry k holds the letter whose CDF
# interval contains (k + 0.5) / 2^16, so each letter's probability is exact to
# 2^-16.
_TABLE = _LETTERS[np.searchsorted(_CDF, (np.arange(65536) + 0.5) / 65536.0, side="right").clip(0, 19)]

CHUNK = 65536  # pairs per independently seeded chunk


def rng_for(config: int, chunk: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1845, config, chunk])))


@dataclasses.dataclass
class PairSet:
    ascii: np.ndarray    # uint8 [total residues]
    offsets: np.ndarray  # int64 [n_seqs + 1]
    pairs: np.ndarray    # int32 [n_pairs, 2]
    name: str = ""

    @property
    def n_seqs(self) -> int:
        return len(self.offsets) - 1

    @property
    def n_pairs(self) -> int:
        return len(self.pairs)

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def cells(self) -> int:
        L = self.lengths()
        return int((L[self.pairs[:, 0]].astype(np.int64) * L[self.pairs[:, 1]]).sum())

    def seq(self, k: int) -> bytes:
        return self.ascii[self.offsets[k]:self.offsets[k + 1]].tobytes()

    def subset(self, idx) -> "PairSet":
        """The pairs ``idx`` with only the sequences they use (renumbered)."""
        idx = np.asarray(idx)
        P = self.pairs[idx]
        used, inv = np.unique(P.reshape(-1), return_inverse=True)
        L = self.lengths()[used]
        offs = np.zeros(len(used) + 1, dtype=np.int64)
        np.cumsum(L, out=offs[1:])
        asc = self.ascii[gather_segments(self.offsets[used], L)]
        return PairSet(asc, offs, inv.reshape(-1, 2).astype(np.int32), self.name + "[sub]")


def concat(sets) -> PairSet:
    """Concatenate pair sets (sequence indices are shifted)."""
    asc, offs, prs, base_res, base_seq = [], [np.zeros(1, np.int64)], [], 0, 0
    for s in sets:
        asc.append(s.ascii)
        offs.append(s.offsets[1:] + base_res)
        prs.append(s.pairs + base_seq)
        base_res += int(s.offsets[-1])
        base_seq += s.n_seqs
    return PairSet(np.concatenate(asc), np.concatenate(offs),
                   np.concatenate(prs).astype(np.int32), "+".join(s.name for s in sets))


def background(rng: np.random.Generator, n: int) -> np.ndarray:
    """n i.i.d. background residues (uint8 ASCII)."""
    return _TABLE[rng.integers(0, 65536, n, dtype=np.uint16)]


def gather_segments(starts: np.ndarray, lengths: np.ndarray) -> np.ndarray:
    """Concatenated index ranges [starts[k], starts[k] + lengths[k])."""
    starts = np.asarray(starts, dtype=np.int64)
    lengths = np.asarray(lengths, dtype=np.int64)
    tot = int(lengths.sum())
    return np.repeat(starts - (np.cumsum(lengths) - lengths), lengths) + np.arange(tot)


def _from_lengths(rng, lengths: np.ndarray):
    lengths = np.asarray(lengths, dtype=np.int64)
    offs = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=offs[1:])
    return background(rng, int(offs[-1])), offs


def lognormal_lengths(rng, n: int, median: float, sigma: float, lo: int, hi: int) -> np.ndarray:
    L = np.rint(np.exp(rng.normal(np.log(median), sigma, n)))
    return np.clip(L, lo, hi).astype(np.int64)


def mutate_many(rng, src: np.ndarray, src_offs: np.ndarray, s, rho):
    """Mutate every sequence of a concatenated set.  ``s`` and ``rho`` are scalars
    or per-sequence arrays.  Returns (ascii, offsets) of the mutants."""
    n = len(src_offs) - 1
    L = np.diff(src_offs)
    s = np.broadcast_to(np.asarray(s, dtype=np.float64), (n,))
    rho = np.broadcast_to(np.asarray(rho, dtype=np.float64), (n,))
    seq_of = np.repeat(np.arange(n), L)
    # substitutions: a different background residue
    x = src.copy()
    hit = rng.random(len(x)) < s[seq_of]
    pos = np.flatnonzero(hit)
    new = background(rng, len(pos))
    clash = new == x[pos]
    while clash.any():
        new[clash] = background(rng, int(clash.sum()))
        clash = new == x[pos]
    x[pos] = new
    # indel events, placed on the original coordinates of each sequence
    n_ev = rng.binomial(L, rho / 3.0)
    ev_seq = np.repeat(np.arange(n), n_ev)
    n_events = len(ev_seq)
    is_ins = rng.random(n_events) < 0.5
    ev_len = rng.integers(1, 6, n_events)
    ev_pos = (rng.random(n_events) * (L[ev_seq] + is_ins)).astype(np.int64)  # ins may go at L
    total = int(src_offs[-1])
    # deletions: mark [pos, pos+len) of the original as removed (clipped to the sequence)
    dmask = np.zeros(total + 1, dtype=np.int64)
    d = ~is_ins
    d_start = src_offs[ev_seq[d]] + ev_pos[d]
    d_end = np.minimum(d_start + ev_len[d], src_offs[ev_seq[d] + 1])
    np.add.at(dmask, d_start, 1)
    np.add.at(dmask, d_end, -1)
    keep = np.cumsum(dmask[:-1]) == 0
    # never delete a whole sequence: keep the first residue if nothing survives
    kept_per_seq = np.bincount(seq_of, weights=keep, minlength=n)
    dead = np.flatnonzero((kept_per_seq == 0) & (L > 0))
    keep[src_offs[dead]] = True
    # insertions: ins_count[slot] residues go before original residue `slot`
    # (slot numbering: original position + sequence index, so each sequence has
    # L+1 slots and the last one is after its final residue)
    i = is_ins
    slot = src_offs[ev_seq[i]] + ev_seq[i] + ev_pos[i]
    ins_count = np.bincount(slot, weights=ev_len[i], minlength=total + n).astype(np.int64)
    # assemble: per sequence, for each slot t: inserted residues then original t
    orig_slot = np.arange(total) + seq_of                         # slot of each original residue
    unit = ins_count.copy()
    unit[orig_slot] += keep                                        # residues emitted per slot
    slot_seq = np.repeat(np.arange(n), L + 1)
    out_len = np.bincount(slot_seq, weights=unit, minlength=n).astype(np.int64)
    out_offs = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(out_len, out=out_offs[1:])
    out = background(rng, int(out_offs[-1]))                       # default: inserted residues
    start_of_slot = np.zeros(len(unit) + 1, dtype=np.int64)
    np.cumsum(unit, out=start_of_slot[1:])
    kept_idx = np.flatnonzero(keep)
    dst = start_of_slot[orig_slot[kept_idx]] + ins_count[orig_slot[kept_idx]]
    out[dst] = x[kept_idx]
    return out, out_offs


def _interleave_pairs(q_asc, q_offs, r_asc, r_offs) -> PairSet:
    """Sequence 2k is the query and 2k+1 the reference of pair k."""
    n = len(q_offs) - 1
    Lq, Lr = np.diff(q_offs), np.diff(r_offs)
    L = np.empty(2 * n, dtype=np.int64)
    L[0::2], L[1::2] = Lq, Lr
    offs = np.zeros(2 * n + 1, dtype=np.int64)
    np.cumsum(L, out=offs[1:])
    asc = np.empty(int(offs[-1]), dtype=np.uint8)
    qi = np.repeat(offs[0:-1:2] - q_offs[:-1], Lq) + np.arange(len(q_asc))
    ri = np.repeat(offs[1::2] - r_offs[:-1], Lr) + np.arange(len(r_asc))
    asc[qi] = q_asc
    asc[ri] = r_asc
    pairs = np.stack([np.arange(0, 2 * n, 2), np.arange(1, 2 * n, 2)], 1).astype(np.int32)
    return PairSet(asc, offs, pairs)


# --------------------------------------------------------------------------
# Benchmark configurations
# --------------------------------------------------------------------------

def config_small(n_pairs: int = 1000) -> PairSet:
    """1,000 pairs, lengths U{50..300}; first half unrelated, second half homologs
    with 30% substitutions and 5% indels of length 1-5."""
    rng = rng_for(1, 0)
    Lq = rng.integers(50, 301, n_pairs)
    q, qo = _from_lengths(rng, Lq)
    half = n_pairs // 2
    Lr_unrel = rng.integers(50, 301, half)
    r1, r1o = _from_lengths(rng, Lr_unrel)
    r2, r2o = mutate_many(rng, q[qo[half]:], qo[half:] - qo[half], 0.30, 0.05)
    r = np.concatenate([r1, r2])
    ro = np.concatenate([r1o, r2o[1:] + r1o[-1]])
    ps = _interleave_pairs(q, qo, r, ro)
    ps.name = "small-1k"
    return ps


def _homolog_chunk(config: int, chunk: int, n: int, long_frac: float, median: float,
                   long_lo: int = 5000, long_hi: int = 35000) -> PairSet:
    rng = rng_for(config, chunk)
    Lq = lognormal_lengths(rng, n, median, 0.6, 30, 5000)
    if long_frac > 0:
        is_long = rng.random(n) < long_frac
        Lq[is_long] = rng.integers(long_lo, long_hi + 1, int(is_long.sum()))
    q, qo = _from_lengths(rng, Lq)
    u = rng.uniform(0.10, 0.90, n)
    r, ro = mutate_many(rng, q, qo, 1.0 - u, 0.03)
    return _interleave_pairs(q, qo, r, ro)


def _c2_chunk(args):
    c, k = args
    full = _homolog_chunk(2, c, CHUNK, 0.0, 280.0)
    return full if k == CHUNK else full.subset(np.arange(k))


def _map_chunks(fn, jobs, workers):
    """Run independent seeded chunk jobs, in order, over a fork pool."""
    if workers is None:
        workers = min(len(os.sched_getaffinity(0)), 16)
    workers = max(1, min(workers, len(jobs)))
    if workers == 1:
        return [fn(j) for j in jobs]
    ctx = multiprocessing.get_context("fork")
    with concurrent.futures.ProcessPoolExecutor(workers, mp_context=ctx) as ex:
        return list(ex.map(fn, jobs))


def config_1m(n_pairs: int = 1_000_000, first_chunk: int = 0, workers: int | None = None) -> PairSet:
    """Log-normal lengths (median 280, sigma 0.6, clipped 30-5000); identity
    U(10%, 90%) by substitution plus 3% indels.  ``n_pairs`` smaller than the
    full million gives a prefix of the same seeded stream (chunk by chunk)."""
    jobs, done, c = [], 0, first_chunk
    while done < n_pairs:
        k = min(CHUNK, n_pairs - done)
        jobs.append((c, k))
        done += k
        c += 1
    ps = concat(_map_chunks(_c2_chunk, jobs, workers))
    ps.name = "1m-lognormal280" if n_pairs == 1_000_000 else "lognormal280-%d" % n_pairs
    return ps


def _c3_chunk(args):
    c, k, long_frac = args
    return _homolog_chunk(3, c, k, long_frac, 250.0)


def config_batching(n_pairs: int, first_chunk: int = 0, long_frac: float = 0.05,
                    workers: int | None = None) -> PairSet:
    """Heavy-tailed mix: 95% log-normal (median 250), 5% U{5,000..35,000}.  A
    final partial chunk is drawn at its own size from its chunk seed."""
    jobs, done, c = [], 0, first_chunk
    while done < n_pairs:
        k = min(CHUNK, n_pairs - done)
        jobs.append((c, k, long_frac))
        done += k
        c += 1
    ps = concat(_map_chunks(_c3_chunk, jobs, workers))
    ps.name = "heavy-tail-%d" % n_pairs
    return ps


C3_PAIRS = 10_000_000  # the whole heavy-tailed batching set


def _c3_chunk_sizes(n_pairs: int = C3_PAIRS):
    """Pairs per chunk of the first n_pairs of the heavy-tailed set."""
    full, rest = divmod(n_pairs, CHUNK)
    return [CHUNK] * full + ([rest] if rest else [])


def _c3_query_lengths(args):
    """Query lengths of one heavy-tail chunk: the first draws of
    _homolog_chunk replayed from the chunk's seed (no residues drawn)."""
    c, k, long_frac = args
    rng = rng_for(3, c)
    Lq = lognormal_lengths(rng, k, 250.0, 0.6, 30, 5000)
    if long_frac > 0:
        is_long = rng.random(k) < long_frac
        Lq[is_long] = rng.integers(5000, 35000 + 1, int(is_long.sum()))
    return Lq


def c3_lpt_shards(n_shards: int, n_pairs: int = C3_PAIRS, long_frac: float = 0.05, workers: int | None = None):
    """Longest-processing-time assignment of the heavy-tailed set's chunks to
    n_shards devices: chunks in decreasing order of cost (the sum of squared
    query lengths, replayed from each chunk's seed; a pair costs about m * n
    and the reference length is the query's within a few percent of indels),
    each to the device with the least cost so far.  Returns (chunk lists per
    shard, cost per shard, cost per chunk)."""
    sizes = _c3_chunk_sizes(n_pairs)
    Ls = _map_chunks(_c3_query_lengths, [(c, k, long_frac) for c, k in enumerate(sizes)], workers)
    cost = np.array([float((L.astype(np.float64) ** 2).sum()) for L in Ls])
    shards = [[] for _ in range(n_shards)]
    load = np.zeros(n_shards)
    for c in np.argsort(-cost, kind="stable"):
        g = int(np.argmin(load))
        shards[g].append(int(c))
        load[g] += cost[c]
    return [sorted(x) for x in shards], load, cost


def c3_shard(chunks, n_pairs: int = C3_PAIRS, long_frac: float = 0.05, workers: int | None = None) -> PairSet:
    """The pairs of the given chunks of the heavy-tailed set (each chunk drawn
    from its own seed at its own size, exactly as config_batching draws it)."""
    sizes = _c3_chunk_sizes(n_pairs)
    ps = concat(_map_chunks(_c3_chunk, [(c, sizes[c], long_frac) for c in chunks], workers))
    ps.name = "heavy-tail-shard-%dchunks" % len(chunks)
    return ps


def families(config: int, n_fam: int, n_members: int, d_lo: float = 0.20, d_hi: float = 0.60):
    """Family model: ancestors LN(280, 0.6) clipped 30-5000; each member picks a
    uniform family and is Mutation(ancestor, d ~ U(d_lo, d_hi), 0.03)."""
    rng = rng_for(config, 0)
    La = lognormal_lengths(rng, n_fam, 280.0, 0.6, 30, 5000)
    anc, anc_o = _from_lengths(rng, La)
    fam = rng.integers(0, n_fam, n_members)
    src_L = La[fam]
    src_o = np.zeros(n_members + 1, dtype=np.int64)
    np.cumsum(src_L, out=src_o[1:])
    src = anc[gather_segments(anc_o[fam], src_L)]
    d = rng.uniform(d_lo, d_hi, n_members)
    asc, offs = mutate_many(rng, src, src_o, d, 0.03)
    return asc, offs, fam


_KMER_BASE = 32


def kmer_sets(asc: np.ndarray, offs: np.ndarray, k: int = 6):
    """Distinct exact k-mers of every sequence: (kmer_code int64, seq int64)."""
    code = np.zeros(256, dtype=np.int64)
    code[_LETTERS] = np.arange(20)
    c = code[asc]
    n = len(offs) - 1
    L = np.diff(offs)
    nk = np.maximum(L - k + 1, 0)
    starts = np.repeat(offs[:-1], nk) + (np.arange(int(nk.sum())) - np.repeat(np.cumsum(nk) - nk, nk))
    km = np.zeros(len(starts), dtype=np.int64)
    for t in range(k):
        km = km * _KMER_BASE + c[starts + t]
    seq = np.repeat(np.arange(n), nk)
    key = np.unique(seq * (_KMER_BASE ** k) + km)
    return key % (_KMER_BASE ** k), key // (_KMER_BASE ** k)


def shared_kmer_pairs(q_asc, q_offs, r_asc, r_offs, k: int = 6, min_shared: int = 2,
                      max_per_query: int | None = None):
    """(query, reference, shared) for every pair sharing >= min_shared distinct
    exact k-mers (the candidate rule of the paper's discovery step: k = 6,
    common k-mer threshold 2).  Optionally keep the top ``max_per_query``."""
    qk, qs = kmer_sets(q_asc, q_offs, k)
    rk, rs = kmer_sets(r_asc, r_offs, k)
    order = np.argsort(rk, kind="stable")
    rk, rs = rk[order], rs[order]
    lo = np.searchsorted(rk, qk, side="left")
    hi = np.searchsorted(rk, qk, side="right")
    cnt = hi - lo
    qrep = np.repeat(qs, cnt)
    idx = np.repeat(lo - np.cumsum(cnt) + cnt, cnt) + np.arange(int(cnt.sum()))
    rmatch = rs[idx]
    nr = len(r_offs) - 1
    key, shared = np.unique(qrep * nr + rmatch, return_counts=True)
    keep = shared >= min_shared
    key, shared = key[keep], shared[keep]
    qq, rr = key // nr, key % nr
    if max_per_query is not None:
        o = np.lexsort((-shared, qq))
        qq, rr, shared = qq[o], rr[o], shared[o]
        first = np.searchsorted(qq, qq, side="left")
        rank = np.arange(len(qq)) - first
        m = rank < max_per_query
        qq, rr, shared = qq[m], rr[m], shared[m]
    return qq.astype(np.int64), rr.astype(np.int64), shared


def config_block(n_fam: int = 2000, n_members: int = 100_000) -> PairSet:
    """Block all-vs-all: family members split alternately into queries and
    references; candidates share >= 2 distinct exact 6-mers."""
    asc, offs, fam = families(4, n_fam, n_members)
    L = np.diff(offs)
    q_idx = np.arange(0, n_members, 2)
    r_idx = np.arange(1, n_members, 2)

    def take(ix):
        o = np.zeros(len(ix) + 1, dtype=np.int64)
        np.cumsum(L[ix], out=o[1:])
        a = asc[gather_segments(offs[ix], L[ix])]
        return a, o

    qa, qo = take(q_idx)
    ra, ro = take(r_idx)
    qq, rr, _ = shared_kmer_pairs(qa, qo, ra, ro)
    nq = len(q_idx)
    offs2 = np.concatenate([qo, ro[1:] + qo[-1]])
    ps = PairSet(np.concatenate([qa, ra]), offs2,
                 np.stack([qq, rr + nq], 1).astype(np.int32), "block-%dx%d" % (nq, len(r_idx)))
    return ps


# --------------------------------------------------------------------------
# Serving workload
# --------------------------------------------------------------------------

class KmerIndex:
    """Distinct exact k-mers of a reference set, as blocks of sorted keys
    k-mer * n + reference (one block per slice of references, built in
    parallel; each block sorted by k-mer, then reference)."""

    def __init__(self, asc, offs, k: int = 6, blocks=None):
        self.k, self.n = k, len(offs) - 1
        if blocks is None:
            km, seq = kmer_sets(asc, offs, k)
            blocks = [np.sort(km * self.n + seq)]
        self.blocks = blocks

    def candidates(self, q_asc, q_offs, min_shared: int = 2, top: int = 200):
        """(query, reference, shared) with >= min_shared distinct shared k-mers,
        at most `top` references per query (most shared first)."""
        qk, qs = kmer_sets(q_asc, q_offs, self.k)
        o = np.argsort(qk)  # sorted needles: numpy's binary search reuses the last bound
        qk, qs = qk[o], qs[o]
        keys = []
        for blk in self.blocks:
            lo = np.searchsorted(blk, qk * self.n, side="left")
            hi = np.searchsorted(blk, (qk + 1) * self.n, side="left")
            cnt = hi - lo
            qrep = np.repeat(qs, cnt)
            idx = np.repeat(lo - np.cumsum(cnt) + cnt, cnt) + np.arange(int(cnt.sum()))
            keys.append(qrep * self.n + blk[idx] % self.n)
        key, shared = np.unique(np.concatenate(keys), return_counts=True)
        keep = shared >= min_shared
        key, shared = key[keep], shared[keep]
        qq, rr = key // self.n, key % self.n
        o = np.lexsort((rr, -shared, qq))
        qq, rr, shared = qq[o], rr[o], shared[o]
        rank = np.arange(len(qq)) - np.searchsorted(qq, qq, side="left")
        m = rank < top
        return qq[m], rr[m], shared[m]


@dataclasses.dataclass
class ServeWorkload:
    ref_ascii: np.ndarray
    ref_offsets: np.ndarray
    batches: list          # (q_ascii uint8, q_offsets int64, cand int32 [n, 2])
    sizes: np.ndarray      # queries per batch


SERVE_FAMILY_BLOCK = 1250  # families per independently seeded block of the reference set


def serving(n_fam: int = 20000, per_fam: int = 50, n_batches: int = 200, max_batch: int = 10000,
            top: int = 200, seed: int = 0, workers: int | None = None, sizes=None) -> ServeWorkload:
    """Reference set: n_fam families x per_fam members (ancestors LN(280, 0.6)
    clipped 30-5000, members Mutation(ancestor, U(0.2, 0.6), 0.03), drawn in
    blocks of SERVE_FAMILY_BLOCK families, each from its own seed).  Query
    batches: sizes log-uniform on [1, max_batch] (or the given ``sizes``);
    each query a fresh member of a random family; candidates: references
    sharing >= 2 distinct exact 6-mers, the `top` most-shared first."""
    global _SERVE_STATE
    rng = rng_for(5, seed)
    La = lognormal_lengths(rng, n_fam, 280.0, 0.6, 30, 5000)
    anc, anc_o = _from_lengths(rng, La)
    blocks = [(seed, b, f0, min(f0 + SERVE_FAMILY_BLOCK, n_fam), per_fam)
              for b, f0 in enumerate(range(0, n_fam, SERVE_FAMILY_BLOCK))]
    _SERVE_STATE = (anc, anc_o, La)
    try:
        parts = _map_chunks(_serve_ref_block, blocks, workers)
    finally:
        _SERVE_STATE = None
    ref = np.concatenate([p[0] for p in parts])
    ref_o = np.zeros(n_fam * per_fam + 1, dtype=np.int64)
    np.cumsum(np.concatenate([np.diff(p[1]) for p in parts]), out=ref_o[1:])
    n_ref = len(ref_o) - 1
    _SERVE_STATE = (ref, ref_o, n_ref)
    try:
        index = KmerIndex(None, ref_o, 6, blocks=_map_chunks(_serve_index_block, blocks, workers))
    finally:
        _SERVE_STATE = None
    drawn = np.exp(rng.uniform(0.0, np.log(max_batch + 1), n_batches)).astype(np.int64).clip(1, max_batch)
    sizes = drawn if sizes is None else np.asarray(sizes, dtype=np.int64)
    n_batches = len(sizes)
    _SERVE_STATE = (anc, anc_o, La, n_fam, index, top)
    try:
        batches = _map_chunks(_serve_batch, [(seed, b, int(sizes[b])) for b in range(n_batches)], workers)
    finally:
        _SERVE_STATE = None
    return ServeWorkload(ref, ref_o, batches, sizes)


def _serve_ref_block(job):
    """Members of families [f0, f1) of the reference set, per_fam each."""
    seed, b, f0, f1, per_fam = job
    anc, anc_o, La = _SERVE_STATE
    rng = rng_for(7, seed * 100003 + b)
    fam = np.repeat(np.arange(f0, f1), per_fam)
    src = anc[gather_segments(anc_o[fam], La[fam])]
    src_o = np.concatenate([[0], np.cumsum(La[fam])])
    return mutate_many(rng, src, src_o, rng.uniform(0.2, 0.6, len(fam)), 0.03)


def _serve_index_block(job):
    """Sorted distinct (k-mer, reference) keys of one block's references."""
    _, _, f0, f1, per_fam = job
    ref, ref_o, n_ref = _SERVE_STATE
    r0, r1 = f0 * per_fam, f1 * per_fam
    km, seq = kmer_sets(ref[ref_o[r0]:ref_o[r1]], ref_o[r0:r1 + 1] - ref_o[r0], 6)
    return np.sort(km * n_ref + (seq + r0))


_SERVE_STATE = None  # shared with the forked workers of serving()


def _serve_batch(job):
    """One query batch of serving(): fresh members of random families and
    their candidate references (seeded by batch number)."""
    seed, b, size = job
    anc, anc_o, La, n_fam, index, top = _SERVE_STATE
    r2 = rng_for(6, seed * 100003 + b)
    f = r2.integers(0, n_fam, size)
    s2 = anc[gather_segments(anc_o[f], La[f])]
    s2o = np.concatenate([[0], np.cumsum(La[f])])
    q, qo = mutate_many(r2, s2, s2o, r2.uniform(0.2, 0.6, len(f)), 0.03)
    qq, rr, _ = index.candidates(q, qo, 2, top)
    return (q, qo, np.stack([qq, rr], 1).astype(np.int32))
