"""Host logic of the continuous-batching EM service (no GPU): admission by
slots and memory, FIFO order with bounded bypass, rejection of requests that
can never fit, and continuous admission while other requests run, driven
through ``serve`` with a simulated executor and clock."""
import pytest

from paper_2301_09710_amd import serve as sv


def _req(rid, size="a", arrival=0.0, iters=4):
    return sv.Request(rid, size, rid, arrival, iters)


NEED = {"a": 3, "b": 5, "huge": 100}


def test_admission_by_slots_and_memory():
    s = sv.Scheduler(budget_bytes=10, max_slots=3, need=lambda r: NEED[r.size])
    for i, size in enumerate(["b", "b", "a", "a"]):
        s.arrive(_req(i, size))
    got = [r.rid for r in s.admit()]
    assert got == [0, 1]                      # 5 + 5 = 10: the "a" behind must wait (strict FIFO)
    assert s.in_use == 10 and s.peak == 10
    s.release(0)
    assert [r.rid for r in s.admit()] == [2]  # 5 + 3 = 8 <= 10
    assert [r.rid for r in s.admit()] == []   # 8 + 3 > 10
    s.release(1)
    assert [r.rid for r in s.admit()] == [3]
    assert s.peak <= 10


def test_slot_limit_and_bypass():
    s = sv.Scheduler(budget_bytes=8, max_slots=2, need=lambda r: NEED[r.size], bypass=1)
    for i, size in enumerate(["b", "b", "a", "a"]):
        s.arrive(_req(i, size))
    assert [r.rid for r in s.admit()] == [0, 2]     # head b fits, second b does not, a bypasses
    assert [r.rid for r in s.admit()] == []         # both slots taken
    s.release(2)
    assert [r.rid for r in s.admit()] == [3]        # b still does not fit (5 + 5 > 8); one bypass
    s.release(0)
    s.release(3)
    assert [r.rid for r in s.admit()] == [1]


def test_oversized_request_rejected():
    s = sv.Scheduler(budget_bytes=10, max_slots=2, need=lambda r: NEED[r.size])
    s.arrive(_req(0, "huge"))
    s.arrive(_req(1, "a"))
    assert [r.rid for r in s.admit()] == [1]
    assert s.rejected == [0]


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3          # every look at the clock advances simulated time by 1 ms
        return self.t


class FakeExecutor:
    """Each request takes `dur[size]` simulated seconds after it starts."""

    def __init__(self, clock, dur):
        self.clock, self.dur = clock, dur
        self.running = {}
        self.starts = {}
        self.max_concurrent = 0

    def start(self, req, now):
        self.running[req.rid] = (req, now)
        self.starts[req.rid] = now
        self.max_concurrent = max(self.max_concurrent, len(self.running))

    def step(self):
        pass

    def finished(self, now):
        out = []
        for rid, (req, t0) in list(self.running.items()):
            if now - t0 >= self.dur[req.size]:
                out.append(sv.Done(rid, req.size, req.arrival, t0, now))
                del self.running[rid]
        return out


def test_serve_continuous_admission(monkeypatch):
    clock = FakeClock()
    monkeypatch.setattr(sv.time, "sleep", lambda s: None)
    ex = FakeExecutor(clock, {"a": 0.05, "b": 0.2})
    sched = sv.Scheduler(budget_bytes=10, max_slots=3, need=lambda r: NEED[r.size])
    trace = [_req(0, "b", 0.0), _req(1, "a", 0.01), _req(2, "a", 0.02), _req(3, "b", 0.03),
             _req(4, "a", 0.04)]
    done = sv.serve(trace, sched, ex, clock=clock)
    assert sorted(d.rid for d in done) == [0, 1, 2, 3, 4]
    assert sched.peak <= 10 and sched.idle()
    # request 3 (b) cannot fit next to 0 (b) and two a's; it is admitted when
    # memory frees up -- before request 0 (the long one) has finished
    fin = {d.rid: d.finished for d in done}
    assert ex.starts[3] < fin[0]
    assert ex.max_concurrent >= 2
    for d in done:
        assert d.latency >= {"a": 0.05, "b": 0.2}[d.size]


def test_poisson_trace_and_summary():
    tr = sv.poisson_trace(200, 20.0, seed=1)
    assert len(tr) == 200 and all(b.arrival > a.arrival for a, b in zip(tr, tr[1:]))
    assert 7.0 < tr[-1].arrival < 14.0                       # mean 10 s at 20 req/s
    assert set(r.size for r in tr) == set(sv.SIZES)
    done = [sv.Done(i, "paper", 0.0, 0.0, 0.01 * (i + 1)) for i in range(100)]
    s = sv.summarize(done, 2.0)
    assert s["requests"] == 100 and abs(s["p50_ms"] - 505.0) < 1e-6 and s["throughput_req_s"] == 50.0
