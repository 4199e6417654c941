"""GPU parity of the caller-owned workspace form (sw_align_sets_ws): the same
results as the library-owned form and the oracle, with a workspace of the
size sw_workspace_size reports and with smaller ones that run fewer blocks
at once; a workspace too small for one slot is refused."""
import sys

import numpy as np
import pytest

import oracle
from workloads import proteins as P

pytestmark = pytest.mark.gpu

SLOT_BYTES = 327680 * 4  # the least boundary-row slot (1,280 KiB)


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


def test_caller_workspace_matches_library_and_oracle(sw):
    import torch
    ps = P.concat([P.config_small(400), P.config_batching(48, first_chunk=9, long_frac=0.15)])
    L = ps.lengths()
    say("workspace set: %d pairs, longest %d, %.3g cells" % (ps.n_pairs, L.max(), ps.cells()))
    b = sw.Batch(ps.ascii, ps.offsets)
    pairs = torch.from_numpy(ps.pairs).cuda()
    ref = sw.align_sets(b.packed, b.offsets, b.packed, b.offsets, pairs, flags=sw.VALIDATE).cpu().numpy()
    exp = oracle.batch_ascii(ps.ascii, ps.offsets, ps.pairs, 11, 1)
    assert (ref == exp).all()
    full = sw.workspace_size(ps.n_pairs, int(L.max()))
    assert full >= sw.workspace_size(ps.n_pairs, 100)
    assert sw.workspace_size(ps.n_pairs + 1000, 100) > sw.workspace_size(ps.n_pairs, 100)
    # bytes before the slots: the full grid of least slots subtracted
    grid = torch.cuda.get_device_properties(0).multi_processor_count * sw.get_tuning()["blocks_per_cu"]
    head = sw.workspace_size(ps.n_pairs, 0) - grid * SLOT_BYTES
    assert 0 < head < (8 << 20), head
    for label, nbytes, flags in [("full", full, 0), ("full, no graph", full, sw.NO_GRAPH),
                                 ("full, plain", full, sw.PLAIN), ("three slots", head + 3 * SLOT_BYTES, 0),
                                 ("one slot", head + SLOT_BYTES, 0), ("one slot, plain", head + SLOT_BYTES, sw.PLAIN)]:
        ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        assert ws.data_ptr() % 256 == 0
        say("caller workspace: %s (%d bytes)" % (label, nbytes))
        for rep in range(2):  # the second call replays the captured graphs
            got = sw.align_sets_ws(b.packed, b.offsets, b.packed, b.offsets, pairs, ws,
                                   flags=flags | sw.VALIDATE).cpu().numpy()
            bad = np.flatnonzero((got != ref).any(axis=1))
            assert len(bad) == 0, "%s: pair %d gpu %s library form %s" % (label, bad[0], got[bad[0]].tolist(),
                                                                          ref[bad[0]].tolist())
        del ws
    tiny = torch.empty(head + SLOT_BYTES - 256, dtype=torch.uint8, device="cuda")
    with pytest.raises(sw.SwError) as e:
        sw.align_sets_ws(b.packed, b.offsets, b.packed, b.offsets, pairs, tiny)
    assert e.value.status == sw.SW_ENOMEM


def test_small_slots_long_similar_pairs(sw):
    """Pairs beyond 54,600 residues whose scores pass 16 bits, in a workspace
    of least slots (1,280 KiB): three int32 boundary rows of such a pair do
    not fit a slot, so after the packed pass stops (and for the start pass)
    they run the in-place sweep; the results equal the library form (whose
    slots take the int32 scan) and the oracle."""
    import torch
    rng = np.random.default_rng(33)
    seqs = []
    for L, rate in [(55000, 0.0), (56000, 0.02)]:
        a = P.background(rng, L)
        b = a.copy()
        hit = rng.random(L) < rate
        b[hit] = P.background(rng, int(hit.sum()))
        seqs += [a, b]
    Ls = np.array([len(x) for x in seqs], dtype=np.int64)
    offs = np.concatenate([[0], np.cumsum(Ls)])
    pairs = np.array([[0, 1], [1, 0], [2, 3], [3, 2]], dtype=np.int32)
    ps = P.PairSet(np.concatenate(seqs), offs, pairs, "long similar")
    exp = oracle.batch_ascii(ps.ascii, ps.offsets, ps.pairs, 11, 1)
    assert (exp[:, 0] > 65504).all(), exp[:, 0]
    say("long similar pairs: scores %s" % exp[:, 0].tolist())
    b = sw.Batch(ps.ascii, ps.offsets)
    pairs_d = torch.from_numpy(ps.pairs).cuda()
    ref = sw.align_sets(b.packed, b.offsets, b.packed, b.offsets, pairs_d, flags=sw.VALIDATE).cpu().numpy()
    assert (ref == exp).all(), (ref.tolist(), exp.tolist())
    grid = torch.cuda.get_device_properties(0).multi_processor_count * sw.get_tuning()["blocks_per_cu"]
    head = sw.workspace_size(ps.n_pairs, 0) - grid * SLOT_BYTES
    ws = torch.empty(head + 2 * SLOT_BYTES, dtype=torch.uint8, device="cuda")
    got = sw.align_sets_ws(b.packed, b.offsets, b.packed, b.offsets, pairs_d, ws, flags=sw.VALIDATE).cpu().numpy()
    assert (got == exp).all(), (got.tolist(), exp.tolist())
    say("long similar pairs: in-place sweeps in least slots equal the oracle")
