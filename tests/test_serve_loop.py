"""The open-loop serving driver against a fake server with an injectable clock
(no GPU): FIFO admission under a slot limit and a memory budget, retry on
'not admissible', latency bookkeeping."""
import numpy as np

from paper_2303_01845_amd.serve import run_open_loop, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def advance(self, dt=1e-3):
        self.t += dt


class FakeServer:
    """Admits while a slot and budget are free; a request completes `dur`
    seconds after admission."""

    def __init__(self, clock, slots, budget, dur):
        self.clock, self.slots, self.budget, self.dur = clock, slots, budget, dur
        self.inflight = {}
        self.used = 0
        self.next = 1
        self.admitted = []
        self.max_inflight = 0

    def submit(self, q_ascii, q_offsets, cand):
        need = len(q_ascii) + 8 * len(cand)
        if len(self.inflight) >= self.slots or self.used + need > self.budget:
            return None
        t = self.next
        self.next += 1
        self.inflight[t] = (self.clock() + self.dur, need, len(cand))
        self.used += need
        self.admitted.append(len(q_ascii))
        self.max_inflight = max(self.max_inflight, len(self.inflight))
        return t

    def poll(self, t):
        end, need, n = self.inflight[t]
        if self.clock() < end:
            return None
        del self.inflight[t]
        self.used -= need
        return np.full((n, 5), 7, np.int32)


def make_requests(sizes):
    reqs = []
    for k, s in enumerate(sizes):
        asc = np.full(s, ord("A"), np.uint8)
        reqs.append((asc, np.array([0, s], np.int64), np.zeros((s // 10 + 1, 2), np.int32)))
    return reqs


def test_fifo_admission_slots_and_latency():
    clock = FakeClock()
    srv = FakeServer(clock, slots=2, budget=10 ** 9, dur=0.010)
    reqs = make_requests([100] * 6)
    arrivals = [0.0, 0.0, 0.0, 0.001, 0.002, 0.030]
    rec = run_open_loop(srv, reqs, arrivals, clock=clock, idle=lambda: clock.advance(1e-3))
    assert srv.max_inflight == 2
    # request 2 waits for a slot: admitted when 0 or 1 completes (~10 ms)
    assert rec[2]["submit"] >= 0.010 - 1e-9
    assert all(r["latency"] >= 0.010 - 1e-9 for r in rec)
    assert rec[5]["latency"] < 0.013  # arrives to an idle server
    assert [r["result"].shape[0] for r in rec] == [11] * 6
    s = summarize(rec, [1e6] * 6)
    assert s["requests"] == 6 and s["p99_ms"] >= s["p50_ms"] > 0


def test_budget_blocks_big_request_until_memory_frees():
    clock = FakeClock()
    srv = FakeServer(clock, slots=8, budget=2000, dur=0.005)
    reqs = make_requests([600, 600, 100])
    rec = run_open_loop(srv, reqs, [0.0, 0.0, 0.0], clock=clock, idle=lambda: clock.advance(5e-4))
    # the second 600-residue request does not fit next to the first; FIFO keeps
    # the third behind it even though it would fit
    assert srv.admitted == [600, 600, 100]
    assert rec[1]["submit"] >= 0.005 - 1e-9
    assert rec[2]["submit"] >= rec[1]["submit"]
