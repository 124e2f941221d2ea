"""Solver autotuning on a resident lattice.

For a target absolute amplitude error, pick the solve mode, the stop tolerance and (for the
mixed paths) the Arnoldi cycle length that give the most solves per second on a calibration
batch of energies. The reference amplitudes come from the FP64 path run to its rounding floor
(tol 1e-12), so the accuracy a configuration reaches is measured, not assumed; a margin keeps
the chosen configuration below the target on other draws of energies.
"""
from __future__ import annotations

import time

import numpy as np

TOL_LADDER = (1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7, 3e-8, 1e-8, 3e-9, 1e-9)
CYCLES = (6, 8, 10, 12)


def _amps(sol, n):
    return np.array([sol.amplitude(k)["A"].ravel() for k in range(n)])


def _timed(L, Es, mode, tol, m, sync, reps):
    L.solve(Es, mode, tol=tol, refine_every=m, allow_noconv=True)
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        sol = L.solve(Es, mode, tol=tol, refine_every=m, allow_noconv=True)
    sync()
    return sol, (time.perf_counter() - t0) / reps


def tune(L, Es, target=1e-6, margin=0.5, modes=("fp64", "mixed", "mixed_split"), sync=lambda: None, reps=2,
         ref=None):
    """Returns {mode: dict(tol, refine_every, s_per_batch, max_err)} for the fastest passing
    configuration of each mode, and the reference amplitudes used."""
    Es = np.asarray(Es, dtype=np.float64)
    if ref is None:
        ref = _amps(L.solve(Es, "fp64", tol=1e-12, allow_noconv=True), len(Es))
    best = {}
    for mode in modes:
        cycles = (0,) if mode == "fp64" else CYCLES
        for m in cycles:
            for tol in TOL_LADDER:   # loosest first: the first passing tolerance is the fastest
                sol = L.solve(Es, mode, tol=tol, refine_every=m, allow_noconv=True)
                err = float(np.max(np.abs(_amps(sol, len(Es)) - ref)))
                if err <= margin * target:
                    _, dt = _timed(L, Es, mode, tol, m, sync, reps)
                    if mode not in best or dt < best[mode]["s_per_batch"]:
                        best[mode] = dict(tol=tol, refine_every=m, s_per_batch=dt, max_err=err)
                    break
    return best, ref
