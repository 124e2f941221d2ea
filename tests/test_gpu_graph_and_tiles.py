"""Graph replay and launch choices of the solve (wp_solve_opts graph / step_tile / spmm_cols).

A launch choice changes how the kernels are issued or which variant runs, never what is
computed: HIP-graph replay of the FP64 term chunks and of the mixed Arnoldi sweeps must give the
launched path's results bit for bit, on every replay (the graph is kept by the lattice and
replayed by later calls, with eager solves in between); every step-kernel variant and both kinds
of many-channel product must match the oracle's series terms at the FP64 tolerance
(tests/parity_util.py).
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import paper_1404_5253_amd as wp

from oracle import pipeline
from parity_util import SERIES_TOL, series_mismatch

SPECS = {
    "doublet_mt_20": pipeline.Spec(M=20, N=20, two_J=1, pot="mt"),
    "pw18_mt_6": pipeline.Spec(M=6, N=7, two_J=1, j_max=2, swave_only=False, pot="mt"),
}
_cache = {}


def _lattice(name, prec="fp64"):
    key = (name, prec)
    if key not in _cache:
        spec = SPECS[name]
        L = wp.Lattice(spec.M, spec.N, two_J=spec.two_J, j_max=spec.j_max, swave_only=spec.swave_only,
                       n_x=spec.n_x, n_phi=spec.n_phi)
        L.pseudostates(kind="mt", V_R=spec.V_R, mu_R=spec.mu_R, mu_A=spec.mu_A, singlet_ratio=spec.singlet_ratio)
        L.build_perm(prec)
        _cache[key] = L
    return _cache[key]


def _state(sol, n, series=True):
    out = []
    for k in range(n):
        a = sol.amplitude(k)
        out.append(a["A"].copy())
        out.append(np.asarray(a["iters"]).copy())
        if series:
            for b in range(a["A"].shape[1]):
                out.append(sol.series(k, b).copy())
    return out


def _same(x, y):
    return len(x) == len(y) and all(np.array_equal(a, b) for a, b in zip(x, y))


@pytest.mark.parametrize("name,Es", [("doublet_mt_20", [14.1]),
                                     ("doublet_mt_20", list(np.random.default_rng(5).uniform(1, 50, 40))),
                                     ("pw18_mt_6", [3.0, 22.7])])
def test_fp64_graph_replay_is_bit_identical(name, Es):
    L = _lattice(name)
    ref = _state(L.solve(Es, "fp64", tol=1e-12, accept=1e-6), len(Es))
    for rep in range(3):   # the first call captures, the next ones replay the kept graphs
        got = _state(L.solve(Es, "fp64", tol=1e-12, accept=1e-6, graph=True), len(Es))
        assert _same(got, ref), (name, rep)
        eager = _state(L.solve(Es, "fp64", tol=1e-12, accept=1e-6), len(Es))
        assert _same(eager, ref), (name, rep)


@pytest.mark.parametrize("mode", ["mixed", "mixed_split"])
@pytest.mark.parametrize("name,Es", [("doublet_mt_20", [3.0, 14.1]), ("pw18_mt_6", [3.0, 22.7])])
def test_mixed_graph_replay_is_bit_identical(name, Es, mode):
    L = _lattice(name)
    ref = _state(L.solve(Es, mode, tol=1e-10, accept=1e-6), len(Es), series=False)
    for rep in range(3):
        got = _state(L.solve(Es, mode, tol=1e-10, accept=1e-6, graph=True), len(Es), series=False)
        assert _same(got, ref), (name, mode, rep)
        eager = _state(L.solve(Es, mode, tol=1e-10, accept=1e-6), len(Es), series=False)
        assert _same(eager, ref), (name, mode, rep)


def _series_parity(name, Es, **launch):
    s = pipeline.build_system(SPECS[name])
    P0full = s.P0geo.full(s.C)
    L = _lattice(name)
    sol = L.solve(Es, "fp64", tol=1e-12, accept=1e-6, **launch)
    assert sol.converged
    worst = 0.0
    for k, E in enumerate(Es):
        ref = pipeline.solve_energy(s, E, P0full=P0full)
        for b in range(len(ref["series"])):
            worst = max(worst, series_mismatch(sol.series(k, b), ref["series"][b]))
    return worst


@pytest.mark.parametrize("tile", ["mfma8", "mfma16", "rows", "valu"])
def test_every_step_kernel_matches_oracle(tile):
    Es = list(np.random.default_rng(11).uniform(1, 50, 24))
    d = _series_parity("doublet_mt_20", Es, step_tile=tile)
    assert d <= SERIES_TOL, (tile, d)


@pytest.mark.parametrize("spmm_cols", [4, 1 << 20])
def test_many_channel_product_choice_matches_oracle(spmm_cols):
    """20 energies x 2 open channels = 40 columns: lanes over the columns (spmm_cols 4) or passes
    of 4 columns (never lanes over columns)."""
    Es = list(np.random.default_rng(13).uniform(1, 50, 20))
    d = _series_parity("pw18_mt_6", Es, spmm_cols=spmm_cols)
    assert d <= SERIES_TOL, (spmm_cols, d)
