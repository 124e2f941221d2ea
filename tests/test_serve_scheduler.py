"""CPU tests of the serving scheduler with a fake backend and a virtual clock (no GPU)."""
import pytest

from paper_1404_5253_amd.serve import run_stream


class VirtualClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += max(dt, 1e-6)


class FakeBackend:
    """Slots finish after ceil(E) steps; each step costs step_s of virtual time."""

    def __init__(self, clock, slots, step_s=0.001):
        self.clock = clock
        self.slots = [None] * slots
        self.step_s = step_s
        self.admitted = 0
        self.max_live = 0

    def admit(self, E):
        for k, s in enumerate(self.slots):
            if s is None:
                self.slots[k] = [E, int(E) + 1]
                self.admitted += 1
                self.max_live = max(self.max_live, self.live())
                return k
        return None

    def live(self):
        return sum(s is not None for s in self.slots)

    def step(self):
        self.clock.t += self.step_s
        out = []
        for k, s in enumerate(self.slots):
            if s is None:
                continue
            s[1] -= 1
            if s[1] <= 0:
                out.append((k, {"E": s[0]}))
                self.slots[k] = None
        return out


def test_all_requests_served_with_budgeted_slots():
    clk = VirtualClock()
    backs = [FakeBackend(clk, 3), FakeBackend(clk, 5)]
    reqs = [(0.0005 * k, k % 2, 1.0 + (k % 7)) for k in range(60)]
    done, st = run_stream(backs, reqs, clock=clk, sleep=clk.sleep, threaded=False)
    assert st["n"] == 60
    assert backs[0].max_live <= 3 and backs[1].max_live <= 5
    for r in done:
        assert r.result["E"] == r.E_lab           # each request gets its own result
        assert r.t_arrival <= r.t_admit <= r.t_done
    assert st["p50_ms"] <= st["p99_ms"]


def test_latency_accounting_single_request():
    clk = VirtualClock()
    back = FakeBackend(clk, 2, step_s=0.002)
    done, st = run_stream([back], [(0.0, 0, 3.0)], clock=clk, sleep=clk.sleep, threaded=False)
    # 4 steps of 2 ms each
    assert done[0].t_done - done[0].t_arrival == pytest.approx(0.008, abs=1e-9)


def test_arrivals_wait_for_free_slots():
    clk = VirtualClock()
    back = FakeBackend(clk, 1, step_s=0.001)
    reqs = [(0.0, 0, 5.0), (0.0, 0, 0.5)]
    done, _ = run_stream([back], reqs, clock=clk, sleep=clk.sleep, threaded=False)
    first, second = sorted(done, key=lambda r: r.t_admit)
    assert second.t_admit >= first.t_done


class ThreadedFakeBackend:
    """Real-time fake for the threaded scheduler: slots finish after ceil(E) steps of step_s
    seconds; admission yields the GIL between taking the slot and returning (widening the window
    in which a request is neither queued nor in flight, had the scheduler not held the lock)."""

    def __init__(self, slots, step_s=0.0002):
        import threading
        import time
        self.time = time
        self.slots = [None] * slots
        self.step_s = step_s
        self.mu = threading.Lock()

    def admit(self, E):
        with self.mu:
            for k, s in enumerate(self.slots):
                if s is None:
                    self.slots[k] = [E, int(E) + 1]
                    self.time.sleep(0)
                    return k
        return None

    def live(self):
        return sum(s is not None for s in self.slots)

    def step(self):
        self.time.sleep(self.step_s)
        out = []
        with self.mu:
            for k, s in enumerate(self.slots):
                if s is None:
                    continue
                s[1] -= 1
                if s[1] <= 0:
                    out.append((k, {"E": s[0]}))
                    self.slots[k] = None
        return out


def test_threaded_stream_serves_every_request():
    """Threaded run_stream (one thread per lattice, as the bench runs it): every request is served
    exactly once with its own result, also the last ones of the stream, and the warm-up window is
    served but not counted."""
    backs = [ThreadedFakeBackend(3), ThreadedFakeBackend(4), ThreadedFakeBackend(2)]
    reqs = [(0.0004 * k, k % 3, 1.0 + (k % 5)) for k in range(300)]
    done, st = run_stream(backs, reqs, threaded=True, measure_from=0.04)
    assert st["n_served"] == st["n_requests"] == 300
    assert sorted(r.rid for r in done) == list(range(300))
    for r in done:
        assert r.result["E"] == r.E_lab and r.t_arrival <= r.t_admit <= r.t_done
    assert st["n"] == sum(1 for r in done if r.t_arrival >= 0.04) < 300


def test_divide_budget_is_proportional_and_fits():
    from paper_1404_5253_amd.serve import divide_budget
    sb = [10, 20, 40, 80]
    sl = divide_budget(1000, sb, [1, 1, 1, 1], max_slots=32)
    assert sum(k * b for k, b in zip(sl, sb)) <= 1000
    assert all(1 <= k <= 32 for k in sl)
    assert sl[0] == sl[1] == sl[2] == sl[3]          # equal weights: equal slot counts
    big = divide_budget(10 ** 9, sb, [1, 1, 1, 1], max_slots=32)
    assert big == [32, 32, 32, 32]                   # capped
    w = divide_budget(4000, [10, 10], [3, 1], max_slots=1000)
    assert w[0] == 3 * w[1] or abs(w[0] - 3 * w[1]) <= 3
    import pytest
    with pytest.raises(ValueError):
        divide_budget(100, [60, 60], [1, 1], max_slots=4)


def test_worker_admits_the_queue_in_one_call():
    """With admit_many the worker hands the whole queue to the backend at once and admits the
    first len(slots) requests in order."""
    from paper_1404_5253_amd.serve import LatticeWorker, Request

    class Many:
        def __init__(self, free):
            self.free = list(range(free))
            self.calls = []

        def admit_many(self, Es):
            self.calls.append(list(Es))
            k = min(len(Es), len(self.free))
            got, self.free = self.free[:k], self.free[k:]
            return got

        def step(self):
            return []

        def live(self):
            return 0

    b = Many(3)
    w = LatticeWorker(b, clock=lambda: 1.0)
    for i in range(5):
        w.submit(Request(i, 0.0, 0, 10.0 + i))
    w.pump()
    assert b.calls == [[10.0, 11.0, 12.0, 13.0, 14.0]]
    assert sorted(w.inflight) == [0, 1, 2]
    assert [r.E_lab for r in w.queue] == [13.0, 14.0]
    assert [w.inflight[k].E_lab for k in (0, 1, 2)] == [10.0, 11.0, 12.0]
