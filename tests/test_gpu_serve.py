"""GPU serving: every request's results equal the oracle and are the same
alone and when served concurrently with others; admission by slots and HBM
budget."""
import sys

import numpy as np
import pytest

import oracle
from workloads import proteins as P

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def setup():
    import torch
    assert torch.cuda.is_available()
    import paper_2303_01845_amd as sw
    from paper_2303_01845_amd.serve import Server, run_open_loop
    w = P.serving(n_fam=300, per_fam=50, n_batches=24, max_batch=400, seed=1)
    refs = sw.Batch(w.ref_ascii, w.ref_offsets)
    return sw, Server, run_open_loop, w, refs


def oracle_for(w, q, qo, cand):
    # one pair set: queries first, then the whole reference set
    asc = np.concatenate([q, w.ref_ascii])
    offs = np.concatenate([qo, w.ref_offsets[1:] + qo[-1]])
    pairs = cand.copy()
    pairs[:, 1] += len(qo) - 1
    return oracle.batch_ascii(asc, offs, pairs, 11, 1)


def test_requests_alone_and_mixed(setup):
    import torch
    sw, Server, run_open_loop, w, refs = setup
    srv = Server(refs.packed, refs.offsets, hbm_budget=1 << 30, max_slots=4)
    try:
        alone = []
        for k, (q, qo, cand) in enumerate(w.batches):
            t = srv.submit(q, qo, cand)
            assert t is not None
            alone.append(srv.wait(t))
        say("alone done")
        for k, (q, qo, cand) in enumerate(w.batches):
            exp = oracle_for(w, q, qo, cand)
            assert (alone[k] == exp).all(), "request %d differs from the oracle" % k
        rng = np.random.default_rng(0)
        arrivals = np.cumsum(rng.exponential(0.0005, len(w.batches)))
        rec = run_open_loop(srv, w.batches, arrivals)
        say("mixed done")
        for k, r in enumerate(rec):
            assert (r["result"] == alone[k]).all(), "request %d differs in the mix" % k
        assert max(r["submit"] for r in rec) > 0
    finally:
        srv.close()


def test_admission_limits(setup):
    sw, Server, run_open_loop, w, refs = setup
    q, qo, cand = max(w.batches, key=lambda b: len(b[2]))
    need = Server.request_bytes(len(q), len(qo) - 1, len(cand))
    srv = Server(refs.packed, refs.offsets, hbm_budget=need + need // 2, max_slots=4)
    try:
        t1 = srv.submit(q, qo, cand)
        assert t1 is not None
        assert srv.submit(q, qo, cand) is None          # budget: the second does not fit now
        assert srv.stats()["inflight"] == 1
        srv.wait(t1)
        t2 = srv.submit(q, qo, cand)                     # memory freed: admitted
        assert t2 is not None
        srv.wait(t2)
        assert srv.stats()["bytes_in_use"] == 0
    finally:
        srv.close()
    tiny = Server(refs.packed, refs.offsets, hbm_budget=1024, max_slots=1)
    try:
        with pytest.raises(sw.SwError) as e:
            tiny.submit(q, qo, cand)
        assert e.value.status == sw.SW_ENOMEM
    finally:
        tiny.close()
    one = Server(refs.packed, refs.offsets, hbm_budget=1 << 30, max_slots=1)
    try:
        exp = oracle_for(w, q, qo, cand)
        t = one.submit(q, qo, cand)
        # the slot is busy: these queue and run merged into one later launch
        more = [one.submit(*b) for b in w.batches[:5]]
        assert all(x is not None for x in more)
        assert (one.wait(t) == exp).all()
        for x, b in zip(more, w.batches[:5]):
            assert (one.wait(x) == oracle_for(w, *b)).all()
        assert one.stats()["inflight"] == 0
    finally:
        one.close()


def test_c5_shaped_set_under_admission_pressure():
    """200,000 resident references (4,000 families x 50), query batches of
    1 to 2,000 sequences with their k-mer candidate lists, all offered at
    once to a server whose budget holds about one large request: requests
    wait for admission (SW_EAGAIN) and memory, yet every request's results
    equal the oracle's and its results when served alone."""
    import os
    import torch
    import paper_2303_01845_amd as sw
    from paper_2303_01845_amd.serve import Server, run_open_loop
    sizes = [2000, 1200, 700, 300, 120, 50, 20, 8, 3, 1, 2000, 450]
    say("generating the C5-shaped serving set (200k references)")
    w = P.serving(n_fam=4000, per_fam=50, sizes=sizes, seed=2)
    say("references %d, requests %d, candidates %d" % (len(w.ref_offsets) - 1, len(w.batches),
                                                      sum(len(b[2]) for b in w.batches)))
    refs = sw.Batch(w.ref_ascii, w.ref_offsets)
    need = max(Server.request_bytes(len(q), len(qo) - 1, len(c)) for q, qo, c in w.batches)
    srv = Server(refs.packed, refs.offsets, hbm_budget=need + need // 4, max_slots=4)

    class Counting:
        rejected = 0

        def submit(self, *a):
            t = srv.submit(*a)
            if t is None:
                Counting.rejected += 1
            return t

        def poll(self, t):
            return srv.poll(t)

    try:
        alone = []
        for q, qo, cand in w.batches:
            t = srv.submit(q, qo, cand)
            assert t is not None
            alone.append(srv.wait(t))
        say("alone done")
        threads = max(1, min(16, len(os.sched_getaffinity(0))))
        for k, (q, qo, cand) in enumerate(w.batches):
            asc = np.concatenate([q, w.ref_ascii])
            offs = np.concatenate([qo, w.ref_offsets[1:] + qo[-1]])
            pairs = cand.copy()
            pairs[:, 1] += len(qo) - 1
            exp = oracle.batch_ascii(asc, offs, pairs, 11, 1, threads=threads)
            assert (alone[k] == exp).all(), "request %d (%d queries) differs from the oracle" % (k, sizes[k])
        say("oracle equal on every request")
        rec = run_open_loop(Counting(), w.batches, np.zeros(len(w.batches)))
        say("all offered at once: %d submits refused for budget" % Counting.rejected)
        assert Counting.rejected > 0
        for k, r in enumerate(rec):
            assert (r["result"] == alone[k]).all(), "request %d differs in the mix" % k
        rng = np.random.default_rng(3)
        rec = run_open_loop(Counting(), w.batches, np.cumsum(rng.exponential(0.002, len(w.batches))))
        for k, r in enumerate(rec):
            assert (r["result"] == alone[k]).all(), "request %d differs under Poisson arrivals" % k
        assert srv.stats()["bytes_in_use"] == 0
    finally:
        srv.close()
