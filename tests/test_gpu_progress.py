"""GPU test of the progress read and the bounded wait (sw_get_progress,
sw_wait): a persistent call with long pairs is still running right after it
is enqueued, the wait with no time left reports SW_ETIMEOUT with a partial
count of its work items, and the unbounded wait ends with every item of the
start pass done; the results are the oracle's."""
import sys

import numpy as np
import pytest

import oracle
from workloads import proteins as P

# On its first GPU run this test went silent for 180 s and was stopped: a
# progress read (a device-to-host copy on a second stream while the
# persistent kernel held every compute unit) and a bounded host wait were
# new in that run, and no cause was shown.  The progress entry points were
# taken out of the library; the test stays, skipped, with this reason.
pytestmark = [pytest.mark.gpu,
              pytest.mark.skip(reason="progress read taken out: its first GPU run went silent (180 s), "
                                      "cause not shown")]


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


def test_progress_and_bounded_wait(sw):
    import torch
    ps = P.concat([P.config_1m(4000, first_chunk=6), P.config_batching(60, first_chunk=30, long_frac=0.5)])
    L = ps.lengths().astype(np.int64)
    mx = np.maximum(L[ps.pairs[:, 0]], L[ps.pairs[:, 1]])
    say("progress set: %d pairs, longest %d, %.3g cells" % (ps.n_pairs, mx.max(), ps.cells()))
    b = sw.Batch(ps.ascii, ps.offsets)
    pairs = torch.from_numpy(ps.pairs).cuda()
    stream = torch.cuda.current_stream()
    out = torch.empty((ps.n_pairs, 5), dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    sw.align_sets(b.packed, b.offsets, b.packed, b.offsets, pairs, out=out, stream=stream)
    done, p0 = sw.wait(0, stream)
    say("right after enqueue: completed %s, progress %s" % (done, p0))
    assert not done
    assert p0["pass"] in (0, 1, 2) and 0 <= p0["items_done"] <= max(p0["items_total"], 0)
    seen = [p0]
    while True:
        done, p = sw.wait(50, stream)
        seen.append(p)
        if done:
            break
    say("completed: progress %s after %d reads" % (p, len(seen)))
    assert p["pass"] == 2 and p["idle"] == 1
    assert p["items_total"] > 0 and p["items_done"] == p["items_total"]
    # within one pass the count never goes down
    for x, y in zip(seen, seen[1:]):
        if x["pass"] == y["pass"] and x["pass"] > 0:
            assert y["items_done"] >= x["items_done"]
    got = out.cpu().numpy()
    short = np.flatnonzero(mx <= 4096)
    sub = ps.subset(short)
    exp = oracle.batch_ascii(sub.ascii, sub.offsets, sub.pairs, 11, 1)
    assert (got[short] == exp).all()
    plain = sw.align_sets(b.packed, b.offsets, b.packed, b.offsets, pairs, flags=sw.PLAIN).cpu().numpy()
    assert (got == plain).all()
    q = sw.progress(stream)
    assert q["idle"] == 1 and q["items_done"] == q["items_total"]
