"""GPU test of the per-bucket autotuner (sw_autotune): on a mixed set it
times each length bucket with every lane count the bucket allows, keeps a
choice per bucket, writes them to its JSON cache, picks the current tuning or
one of the two tables, and leaves results equal to the oracle's; a second call
finds every bucket in the cache and times none."""
import json
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
    yield lib
    lib.set_tuning(16, 1024, -1, 2048, 2048)


def buckets_of(ps):
    L = ps.lengths().astype(np.int64)
    mx = np.maximum(L[ps.pairs[:, 0]], L[ps.pairs[:, 1]])
    return sorted({int(np.ceil(np.log2(x))) if x > 1 else 0 for x in mx})


def test_autotune_per_bucket_and_cache(sw, tmp_path):
    import torch
    ps = P.concat([P.config_small(300), P.config_1m(3000, first_chunk=3),
                   P.config_batching(24, first_chunk=21, long_frac=0.3)])
    present = buckets_of(ps)
    say("autotune set: %d pairs, buckets %s, %.3g cells" % (ps.n_pairs, present, ps.cells()))
    b = sw.Batch(ps.ascii, ps.offsets)
    pairs = torch.from_numpy(ps.pairs).cuda()
    exp = oracle.batch_ascii(ps.ascii, ps.offsets, ps.pairs, 11, 1)
    cache = tmp_path / "sw_tune.json"
    out = torch.empty((ps.n_pairs, 5), dtype=torch.int32, device="cuda")
    chosen, ms, trials = sw.autotune(b.packed, b.offsets, pairs, reps=1, out=out, cache_path=str(cache))
    say("first call: %d trials, chosen %s, %.2f ms" % (trials, chosen, ms))
    assert (out.cpu().numpy() == exp).all()
    assert trials >= 2 * len(present)
    assert sw.get_tuning() == chosen
    lanes = chosen["bucket_lanes"]
    R = chosen["rows_per_lane"]
    doc = json.loads(cache.read_text())
    keys = {(e["rows_per_lane"], e["bucket"]) for e in doc["entries"]}
    assert {(r, bk) for r in (16, 8) for bk in present} <= keys
    assert all(e["gap_open"] == 11 and e["gap_extend"] == 1 for e in doc["entries"])
    # the candidates: the tuning in force before the call (no table, the
    # length thresholds decide) and the table found for each rows_per_lane
    tables = {r: [0] * 17 for r in (16, 8)}
    for e in doc["entries"]:
        if e["bucket"] in present:
            tables[e["rows_per_lane"]][e["bucket"]] = e["lanes"]
    for r, t in tables.items():
        for bk in present:
            assert t[bk] in (1, 8, 16, 64), (r, bk, t)
            if t[bk] == 1:
                assert (1 << bk) <= min(1024, 64 * r)
            if t[bk] in (8, 16):
                assert (1 << bk) <= 4096
    assert lanes == [0] * 17 or (lanes == tables[R]), (R, lanes, tables)
    # results with the chosen table through the plain call as well
    got = sw.align(b.packed, b.offsets, pairs, 11, 1, sw.VALIDATE).cpu().numpy()
    assert (got == exp).all()
    out2 = torch.full((ps.n_pairs, 5), -9, dtype=torch.int32, device="cuda")
    chosen2, ms2, trials2 = sw.autotune(b.packed, b.offsets, pairs, reps=1, out=out2, cache_path=str(cache))
    say("second call: %d trials, chosen %s" % (trials2, chosen2))
    assert trials2 == 0
    # timed again on the whole workload: the same candidates
    assert chosen2["bucket_lanes"] in (lanes, tables[16], tables[8]), (chosen2, lanes, tables)
    assert (out2.cpu().numpy() == exp).all()


def test_bucket_override_table(sw):
    """Every lane count a bucket allows, set by hand, gives the oracle's
    results (pairs of 513-1024 and 1025-2048 residues)."""
    import torch
    ps = P.concat([P.config_1m(1500, first_chunk=4), P.config_small(200)])
    exp = oracle.batch_ascii(ps.ascii, ps.offsets, ps.pairs, 11, 1)
    b = sw.Batch(ps.ascii, ps.offsets)
    pairs = torch.from_numpy(ps.pairs).cuda()
    try:
        for l10, l11, l9 in [(1, 8, 1), (8, 16, 8), (16, 64, 16), (64, 8, 64), (1, 64, 8)]:
            table = [0] * 17
            table[9], table[10], table[11] = l9, l10, l11
            sw.set_tuning(16, 1024, -1, 2048, 2048, bucket_lanes=table)
            for fl in (sw.PERSISTENT, sw.PLAIN):
                got = sw.Batch(ps.ascii, ps.offsets).align(ps.pairs, 11, 1, fl | sw.VALIDATE).cpu().numpy()
                bad = np.flatnonzero((got != exp).any(axis=1))
                assert len(bad) == 0, (table[9:12], fl, bad[:5])
            say("bucket lanes 9/10/11 = %d/%d/%d: equal to the oracle" % (l9, l10, l11))
    finally:
        sw.set_tuning(16, 1024, -1, 2048, 2048)
