"""GPU parity of the breakup transition elements (faddeev_breakup, mixed modes): the cells must be
the oracle's exactly (integer work), and each element <Z_kj^g|U|Z_0j0> = (O y)_{gkj} must match
the oracle's dense solve to 1e-7 of the largest element (the refined mixed solution at tol 1e-11
agrees with FP64 to ~1e-9 in the amplitude)."""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import paper_1404_5253_amd as wp

from oracle import pipeline

SPECS = {
    "doublet_mt_20": pipeline.Spec(M=20, N=20, two_J=1, pot="mt"),
    "pw18_mt_6": pipeline.Spec(M=6, N=7, two_J=1, j_max=2, swave_only=False, pot="mt"),
}


def _lattice(spec):
    L = wp.Lattice(spec.M, spec.N, two_J=spec.two_J, j_max=spec.j_max, swave_only=spec.swave_only,
                   n_x=spec.n_x, n_phi=spec.n_phi)
    L.pseudostates(kind="mt", V_R=spec.V_R, mu_R=spec.mu_R, mu_A=spec.mu_A, singlet_ratio=spec.singlet_ratio)
    L.build_perm("fp64")
    return L


@pytest.mark.parametrize("name,Es", [("doublet_mt_20", [14.1, 30.0]), ("pw18_mt_6", [22.7]),
                                     ("doublet_mt_20", [1.0])])
@pytest.mark.parametrize("mode", ["mixed", "mixed_split"])
def test_breakup_elements_match_oracle(name, Es, mode):
    spec = SPECS[name]
    s = pipeline.build_system(spec)
    P0full = s.P0geo.full(s.C)
    L = _lattice(spec)
    sol = L.solve(Es, mode, tol=1e-11, accept=1e-8, breakup=True)
    assert sol.converged
    for k, E in enumerate(Es):
        ref_cells, ref = pipeline.breakup_elements(s, E, P0full=P0full)
        for b in ref:
            cells, U = sol.breakup(k, b)
            assert [tuple(c) for c in cells.tolist()] == ref_cells, (name, E)
            if ref_cells:
                scale = np.max(np.abs(ref[b]))
                assert np.max(np.abs(U - ref[b])) <= 1e-7 * scale, (name, E, b, np.max(np.abs(U - ref[b])) / scale)


def test_fp64_solutions_hold_no_breakup_cells():
    L = _lattice(SPECS["doublet_mt_20"])
    sol = L.solve([14.1], "fp64", breakup=True)
    cells, U = sol.breakup(0, 0)
    assert cells.shape == (0, 3) and U.size == 0
