"""Host logic of the autotuner (tune.py) on a stand-in lattice: no GPU.

The stand-in's amplitude error depends only on the stop tolerance and its run time on every
choice, so the configuration the tuner must pick is known in advance.
"""
import time

import numpy as np

from paper_1404_5253_amd.tune import tune, solve_amplitudes


class _Sol:
    def __init__(self, n, err):
        self.n, self.err = n, err

    def amplitude(self, k):
        return {"A": np.array([[1.0 + self.err]]), "iters": np.array([10])}


class _FakeLattice:
    nch = 18
    # seconds per call of each choice (defaults: 2 ms)
    COST = {("step_tile", "mfma16"): -0.001, ("graph", True): -0.0005, ("spmm_cols", 32): +0.002}

    def __init__(self):
        self.calls = []

    def solve(self, Es, mode, tol=1e-12, refine_every=0, allow_noconv=False, graph=False, step_tile="auto",
              spmm_cols=0):
        self.calls.append((len(Es), mode, tol, refine_every, graph, step_tile, spmm_cols))
        t = 0.002 + self.COST.get(("step_tile", step_tile), 0) + self.COST.get(("graph", graph), 0) + \
            self.COST.get(("spmm_cols", spmm_cols), 0)
        if mode != "fp64":
            t *= 0.5
        time.sleep(max(t, 0.0))
        err = 0.0 if tol <= 1e-12 else tol * (0.3 if mode == "fp64" else 3.0)
        return _Sol(len(Es), err)


def test_tuner_picks_fastest_passing_configuration():
    L = _FakeLattice()
    Es = np.linspace(1, 50, 8)
    best, ref = tune(L, Es, target=1e-6, margin=0.5, modes=("fp64", "mixed"), reps=1)
    # the loosest tolerance with error <= 5e-7
    assert best["fp64"]["tol"] == 1e-6
    assert best["mixed"]["tol"] == 1e-7
    for cfg in best.values():
        assert cfg["step_tile"] == "mfma16"
        assert cfg["graph"] is True
        assert cfg["spmm_cols"] != 32
        assert cfg["max_err"] <= 5e-7


def test_solve_amplitudes_splits_the_batch():
    L = _FakeLattice()
    A = solve_amplitudes(L, np.arange(10.0), "fp64", 1e-12, width=4)
    assert A.shape == (10, 1)
    assert [c[0] for c in L.calls] == [4, 4, 2]
