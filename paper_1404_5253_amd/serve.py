"""Continuous-batching serving loop over resident lattices (faddeev_batch_* of libwpcd, FP64 or
mixed precision).

Each resident lattice owns one batch (a fixed number of energy slots sized by a device-memory
budget) and one worker thread with its own HIP stream, so the steps of different lattices
overlap on the GPU (ctypes releases the GIL inside library calls). A request
(arrival time, lattice, E_lab) waits in its lattice's queue until a slot is free, is admitted
between two steps of that batch, advances with every step of the batch and retires as soon as
its Pade estimate is accepted; latency = retirement time - arrival time.

Admission takes every queued request that fits in one call (admit_many: runs of adjacent free
slots, one G1 launch and one right-hand-side product per run, enqueued on the lattice's own
stream). One device-memory budget is divided among the lattices' batches (divide_budget), in
units of each lattice's slot size.

The scheduler only talks to a backend object with admit(E) -> slot | None (or admit_many(Es) ->
slots), step() -> list of (slot, result) and live(), so it is tested on the CPU with a fake
backend and a virtual clock.
"""
from __future__ import annotations

import ctypes as C
import threading
import time
from collections import deque
from dataclasses import dataclass, field


@dataclass
class Request:
    rid: int
    t_arrival: float
    lattice: int
    E_lab: float
    t_admit: float = -1.0
    t_done: float = -1.0
    result: dict = field(default=None)


class BatchBackend:
    """One lattice's continuous batch on the GPU: mode "fp64" (Pade-summed Neumann terms, `terms`
    per step) or "mixed" / "mixed_split" (one FP64-refined mixed-precision cycle of refine_every
    Arnoldi steps per step)."""

    def __init__(self, lattice, slots, hbm_budget, terms=4, tol=1e-12, accept=1e-7, max_iter=200, stream=None,
                 mode="fp64", refine_every=0):
        import paper_1404_5253_amd as wp
        self.wp = wp
        self.L = lattice
        self.terms = terms
        self.mode = mode
        o = wp._SolveOpts(wp.SOLVE_MODES[mode], tol, accept, max_iter, refine_every, 0, 0, 0)
        self.h = C.c_void_p()
        wp._check(wp._lib.faddeev_batch_create(lattice.h, slots, hbm_budget, C.byref(o), C.byref(self.h)))
        self.slots = slots
        self.stream = stream
        self._done = (C.c_int * slots)()

    def admit_many(self, Es):
        """Slots of the first len(result) energies of Es (fewer when the batch is full)."""
        n = len(Es)
        if n == 0:
            return []
        E = (C.c_double * n)(*Es)
        sl = (C.c_int * n)()
        got = C.c_int()
        self.wp._check(self.wp._lib.faddeev_batch_admit_many(self.h, n, E, self.stream, sl, C.byref(got)))
        return list(sl[:got.value])

    def admit(self, E_lab):
        got = self.admit_many([E_lab])
        return got[0] if got else None

    def live(self):
        n = C.c_int()
        self.wp._check(self.wp._lib.faddeev_batch_live(self.h, C.byref(n)))
        return n.value

    def step(self):
        n = C.c_int()
        self.wp._check(self.wp._lib.faddeev_batch_step(self.h, self.stream, self.terms, C.byref(n), self._done))
        out = []
        for k in range(n.value):
            sl = self._done[k]
            hs = C.c_void_p()
            st = self.wp._lib.faddeev_batch_take(self.h, sl, C.byref(hs))
            if st not in (self.wp.WP_OK, self.wp.WP_ENOCONV):
                self.wp._check(st)
            res = self.wp.amplitude(hs, 0)
            res["accepted"] = st == self.wp.WP_OK
            self.wp._lib.wp_solution_free(hs)
            out.append((sl, res))
        return out

    def close(self):
        if self.h is not None and self.h.value:
            self.wp._lib.faddeev_batch_free(self.h)
            self.h = None


class LatticeWorker:
    """Admission + stepping loop of one lattice; runs in its own thread."""

    def __init__(self, backend, clock):
        self.b = backend
        self.clock = clock
        self.queue = deque()
        self.inflight = {}
        self.finished = []
        self.lock = threading.Lock()
        self.steps = 0

    def submit(self, req):
        with self.lock:
            self.queue.append(req)

    def busy(self):
        """True while a submitted request has not retired (read under the lock, so that a request
        between the queue and the in-flight table is still seen)."""
        with self.lock:
            return bool(self.queue or self.inflight)

    def pump(self):
        """Admit what fits, then one step. Returns True if any work was done."""
        with self.lock:
            if hasattr(self.b, "admit_many"):
                slots = self.b.admit_many([r.E_lab for r in self.queue]) if self.queue else []
                t = self.clock()
                for sl in slots:
                    req = self.queue.popleft()
                    req.t_admit = t
                    self.inflight[sl] = req
            else:
                while self.queue:
                    sl = self.b.admit(self.queue[0].E_lab)
                    if sl is None:
                        break
                    req = self.queue.popleft()
                    req.t_admit = self.clock()
                    self.inflight[sl] = req
        if not self.inflight:
            return False
        for sl, res in self.b.step():
            req = self.inflight[sl]
            req.t_done = self.clock()
            req.result = res
            with self.lock:   # finished before it leaves the in-flight table
                self.finished.append(req)
                del self.inflight[sl]
        self.steps += 1
        return True


def run_stream(backends, requests, clock=time.perf_counter, sleep=time.sleep, threaded=True, measure_from=0.0):
    """Serve (t_arrival, lattice, E_lab) requests in arrival order; returns finished Requests and stats.

    With threaded=True each lattice is stepped by its own thread; with False a single loop
    round-robins the lattices (deterministic, used with a virtual clock). The stats cover the
    requests arriving at or after measure_from (seconds into the stream: the warm-up before it
    is served but not counted).
    """
    reqs = [Request(k, t, lat, E) for k, (t, lat, E) in enumerate(sorted(requests))]
    t0 = clock()
    now = lambda: clock() - t0
    workers = [LatticeWorker(b, now) for b in backends]
    pending = deque(reqs)
    stop = threading.Event()

    def feed():
        while pending and pending[0].t_arrival <= now():
            r = pending.popleft()
            workers[r.lattice].submit(r)

    def worker_loop(w):
        while not stop.is_set():
            if not w.pump():
                sleep(0.0002)

    if threaded:
        threads = [threading.Thread(target=worker_loop, args=(w,), daemon=True) for w in workers]
        for t in threads:
            t.start()
        while pending or any(w.busy() for w in workers):
            feed()
            wait = pending[0].t_arrival - now() if pending else 0.0
            sleep(min(0.001, wait) if wait > 0 else 0.0005)
        stop.set()
        for t in threads:
            t.join()
    else:
        while pending or any(w.busy() for w in workers):
            feed()
            busy = False
            for w in workers:
                busy |= w.pump()
            if not busy and pending:
                sleep(max(0.0, pending[0].t_arrival - now()))   # clamped: the clock moves on
    t_end = now()
    done = [r for w in workers for r in w.finished]
    done.sort(key=lambda r: r.rid)
    counted = [r for r in done if r.t_arrival >= measure_from]
    lat = sorted(r.t_done - r.t_arrival for r in counted)

    def pct(p):
        if not lat:
            return float("nan")
        k = min(len(lat) - 1, max(0, int(round(p / 100.0 * (len(lat) - 1)))))
        return lat[k]
    span = (max(r.t_done for r in counted) - min(r.t_arrival for r in counted)) if counted else 0.0
    stats = dict(n=len(counted), n_served=len(done), n_requests=len(reqs), p50_ms=pct(50) * 1e3,
                 p99_ms=pct(99) * 1e3, mean_ms=(sum(lat) / len(lat) * 1e3) if lat else 0,
                 solves_per_s=len(counted) / span if span > 0 else 0.0, wall_s=t_end,
                 steps=[w.steps for w in workers])
    return done, stats


def slot_bytes(lattice, mode="fp64", refine_every=0):
    """Device bytes one batch slot takes on this lattice (faddeev_batch_slot_bytes)."""
    import paper_1404_5253_amd as wp
    o = wp._SolveOpts(wp.SOLVE_MODES[mode], 1e-8, 1e-8, 200, refine_every, 0, 0, 0)
    b = C.c_size_t()
    wp._check(wp._lib.faddeev_batch_slot_bytes(lattice.h, C.byref(o), C.byref(b)))
    return b.value


def divide_budget(total_bytes, slot_bytes, weights, max_slots):
    """Slots per lattice from one device-memory budget: proportional to the weights (each
    lattice's share of the expected load), at least one and at most max_slots each, with
    sum(slots[i] * slot_bytes[i]) <= total_bytes. Raises if not even one slot each fits."""
    n = len(slot_bytes)
    if sum(slot_bytes) > total_bytes:
        raise ValueError("budget smaller than one slot per lattice")
    wsum = float(sum(weights))

    def slots_at(scale):
        return [min(max_slots, max(1, int(scale * w / wsum))) for w in weights]

    def cost(sl):
        return sum(k * b for k, b in zip(sl, slot_bytes))

    lo, hi = 0.0, float(max_slots) * n * 4 + 1.0
    for _ in range(100):   # largest scale whose slots fit
        mid = 0.5 * (lo + hi)
        if cost(slots_at(mid)) <= total_bytes:
            lo = mid
        else:
            hi = mid
    return slots_at(lo)
