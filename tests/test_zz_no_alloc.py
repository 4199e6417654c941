"""GPU test of sw_align_sets_static, the entry point that allocates nothing:
its results equal those of sw_align_sets (and so the oracle's) on two calls
in a row, the second with a smaller input, through the C ABI; device memory
does not shrink during a call; refused flags and sizes return their errors."""
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


def test_static_workspace_matches_library_form(sw):
    import torch
    big = P.concat([P.config_small(600), P.config_batching(64, first_chunk=11, long_frac=0.2)])
    small = P.config_1m(300)
    sets = [("first call", big), ("second call, smaller", small)]
    prepared = []
    for label, ps in sets:
        b = sw.Batch(ps.ascii, ps.offsets)
        pairs = torch.from_numpy(ps.pairs).cuda()
        ref = sw.align_sets(b.packed, b.offsets, b.packed, b.offsets, pairs, flags=sw.VALIDATE).cpu().numpy()
        exp = oracle.batch_ascii(ps.ascii, ps.offsets, ps.pairs, 11, 1)
        assert (ref == exp).all(), label
        out = torch.full((ps.n_pairs, 5), -7, dtype=torch.int32, device="cuda")
        prepared.append((label, ps, b, pairs, ref, out))
    torch.cuda.synchronize()
    for label, ps, b, pairs, ref, out in prepared:
        say("%s: %d pairs, longest %d, %.3g cells" % (label, ps.n_pairs, ps.lengths().max(), ps.cells()))
        free0 = torch.cuda.mem_get_info()[0]
        sw.align_sets_static(b.packed, b.offsets, b.packed, b.offsets, pairs, flags=sw.VALIDATE, out=out)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        got = out.cpu().numpy()
        bad = np.flatnonzero((got != ref).any(axis=1))
        assert len(bad) == 0, "%s: pair %d static %s library %s" % (label, bad[0], got[bad[0]].tolist(),
                                                                   ref[bad[0]].tolist())
        assert free1 >= free0 - (1 << 20), "%s: free device memory fell by %d bytes" % (label, free0 - free1)
        say("%s: equal to sw_align_sets on every pair" % label)


def test_static_refusals(sw):
    import torch
    ps = P.config_small(20)
    b = sw.Batch(ps.ascii, ps.offsets)
    pairs = torch.from_numpy(ps.pairs).cuda()
    for fl in (sw.PLAIN, sw.TIMED):
        with pytest.raises(sw.SwError) as e:
            sw.align_sets_static(b.packed, b.offsets, b.packed, b.offsets, pairs, flags=fl)
        assert e.value.status == sw.SW_EINVAL
    many = torch.zeros(((1 << 22) + 1, 2), dtype=torch.int32, device="cuda")
    out = torch.empty((1, 5), dtype=torch.int32, device="cuda")
    with pytest.raises(sw.SwError) as e:
        sw.align_sets_static(b.packed, b.offsets, b.packed, b.offsets, many, out=out)
    assert e.value.status == sw.SW_ENOMEM
    assert "at most" in sw.lib().sw_last_device_error().decode()
