"""Solver autotuning on a resident lattice.

For a target absolute amplitude error, pick the solve mode, the stop tolerance and (for the
mixed paths) the Arnoldi cycle length that give the most solves per second on a calibration
batch of energies. The reference amplitudes come from the FP64 path run to its rounding floor
(tol 1e-12), so the accuracy a configuration reaches is measured, not assumed; a margin keeps
the chosen configuration below the target on other draws of energies.

A second stage tunes how the chosen configuration is launched, one choice at a time (each kept
only if it is faster and still within the margin): the FP64 step kernel (`step_tile`: MFMA with
8 or 16 columns per workgroup, the row-parallel MFMA kernel, or the VALU kernel), with more than
4 channels the column count from which the block-CSR products run lanes over the columns
(`spmm_cols`), HIP-graph replay of the term chunks / Arnoldi sweeps (`graph`), and the batch
width (energies per call; the batch is solved in calls of that many energies).
"""
from __future__ import annotations

import time

import numpy as np

TOL_LADDER = (1e-4, 3e-5, 1e-5, 3e-6, 1e-6, 3e-7, 1e-7, 3e-8, 1e-8, 3e-9, 1e-9)
CYCLES = (6, 8, 10, 12)
STEP_TILES = ("auto", "mfma8", "mfma16", "rows", "valu")
SPMM_COLS = (0, 8, 32, 1 << 20)          # 0: the library's default (16); 1 << 20: never
WIDTH_DIVISORS = (1, 2, 4)
LAUNCH_DEFAULTS = dict(step_tile="auto", spmm_cols=0, graph=False, width=None)


def _amps(sol, n):
    return np.array([sol.amplitude(k)["A"].ravel() for k in range(n)])


def solve_amplitudes(L, Es, mode, tol, refine_every=0, width=None, iters=False, **launch):
    """Amplitude arrays of every energy, the batch solved in calls of `width` energies (all at
    once when None); `launch` takes graph, step_tile and spmm_cols. With iters, also the largest
    number of operator applications any energy took."""
    Es = np.asarray(Es, dtype=np.float64)
    w = len(Es) if not width else int(width)
    out, it = [], 0
    for k in range(0, len(Es), w):
        part = Es[k:k + w]
        sol = L.solve(part, mode, tol=tol, refine_every=refine_every, allow_noconv=True, **launch)
        out.append(_amps(sol, len(part)))
        if iters:
            it = max(it, max(int(np.max(sol.amplitude(e)["iters"])) for e in range(len(part))))
    return (np.concatenate(out), it) if iters else np.concatenate(out)


def _launch(cfg):
    return {k: cfg[k] for k in ("graph", "step_tile", "spmm_cols") if k in cfg}


def _timed(L, Es, mode, cfg, sync, reps):
    run = lambda: solve_amplitudes(L, Es, mode, cfg["tol"], cfg["refine_every"], cfg.get("width"), **_launch(cfg))
    run()
    sync()
    t0 = time.perf_counter()
    for _ in range(reps):
        amps = run()
    sync()
    return amps, (time.perf_counter() - t0) / reps


def tune(L, Es, target=1e-6, margin=0.5, modes=("fp64", "mixed", "mixed_split"), sync=lambda: None, reps=2,
         ref=None, launch=True):
    """Returns {mode: dict(tol, refine_every, step_tile, spmm_cols, graph, width, s_per_batch,
    max_err)} for the fastest passing configuration of each mode, and the reference amplitudes
    used."""
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
                    cfg = dict(LAUNCH_DEFAULTS, tol=tol, refine_every=m)
                    _, dt = _timed(L, Es, mode, cfg, sync, reps)
                    if mode not in best or dt < best[mode]["s_per_batch"]:
                        best[mode] = dict(cfg, s_per_batch=dt, max_err=err)
                    break
    if not launch:
        return best, ref
    widths = sorted({max(1, len(Es) // d) for d in WIDTH_DIVISORS}, reverse=True)
    choices = (("step_tile", STEP_TILES), ("spmm_cols", SPMM_COLS if L.nch > 4 else (0,)),
               ("graph", (False, True)), ("width", [None] + widths[1:]))
    for mode, cfg in best.items():
        for key, options in choices:
            for opt in options:
                if opt == cfg[key]:
                    continue
                trial = dict(cfg, **{key: opt})
                amps, dt = _timed(L, Es, mode, trial, sync, reps)
                err = float(np.max(np.abs(amps - ref)))
                if err <= margin * target and dt < cfg["s_per_batch"]:
                    cfg.update(trial, s_per_batch=dt, max_err=err)
    return best, ref
