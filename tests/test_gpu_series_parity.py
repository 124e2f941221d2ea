"""GPU parity of the FP64 solve, one case per kernel variant the solve dispatches, through the C ABI.

The FP64 path's arithmetic is deterministic: the on-shell series terms a_n = e_f^T O K^n b
(Sec. II.A; Sec. V.A step 5) are compared with the oracle's terms element by element, before
any Pade summation, at 1e-10 relative for the first ten terms and linearly growing after them
(tests/parity_util.py). Every solve must be accepted (no
WP_ENOCONV). Amplitudes (Pade, Sec. II.B.4): 1e-10 relative against the oracle where the series
converges; where it diverges, 1e-8 relative against the dense LU solution of the same discrete
system, the accuracy of Pade summation of such a series (tests/parity_util.py).

The solve kernels are chosen by the grid a call makes (columns = energies x open channels):

| case | columns | FP64 step | SpMV / SpMM |
|---|---|---|---|
| doublet_mt_20, 1 energy | 1 | k_step64r (MFMA, all row tiles per workgroup) | k_spmv, 2 channels |
| doublet_mt_20, 64 energies | 64 | k_step64m<1> (MFMA, >= 256 workgroups) | k_spmm, 2 channels |
| pw18_mt_6, 1 energy | 2 | k_step64r | k_spmv_pk<18, 2 columns> |
| pw18_mt_6, 2 energies | 4 | k_step64r | k_spmv_pk<18, 4 columns> |
| pw18_mt_6, 20 energies | 40 | k_step64m<2> | k_spmm_pk |
| pw10_mt_8, 2 energies | 4 | k_step64r | k_spmv_pk<10, 4 columns> |
| doublet_mt_136x8, 1 energy | 1 | k_step64 (VALU, M > 128) | k_spmv, 2 channels |
| quartet_yam_24, 3 energies | 3 | k_step64r | k_spmv, 1 channel |
| pw30_mt_4, 3 and 12 energies | 3 x open channels | k_step64r / k_step64m | k_spmv_pk<30, 4> (more than 24 channels) |

Many-channel P0 (more than 4 channels) is stored packed: only the channel pairs with a nonzero
recoupling coefficient, in a permuted channel order (k_spmv_pk, k_spmm_pk).
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import paper_1404_5253_amd as wp

from oracle import pipeline
from parity_util import SERIES_TOL, amplitude_tolerance, series_mismatch

SPECS = {
    "doublet_mt_20": pipeline.Spec(M=20, N=20, two_J=1, pot="mt"),
    "pw18_mt_6": pipeline.Spec(M=6, N=7, two_J=1, j_max=2, swave_only=False, pot="mt"),
    "pw10_mt_8": pipeline.Spec(M=8, N=8, two_J=1, j_max=1, swave_only=False, pot="mt"),
    "doublet_mt_136x8": pipeline.Spec(M=136, N=8, two_J=1, pot="mt"),
    "quartet_yam_24": pipeline.Spec(M=24, N=24, two_J=3, pot="yamaguchi"),
    "pw30_mt_4": pipeline.Spec(M=4, N=5, two_J=3, j_max=2, swave_only=False, pot="mt"),
}

CASES = {
    "doublet_mt_20-E1": ("doublet_mt_20", [14.1]),
    "doublet_mt_20-E64": ("doublet_mt_20", list(np.random.default_rng(1234).uniform(1.0, 50.0, 64))),
    "pw18_mt_6-E1": ("pw18_mt_6", [22.7]),
    "pw18_mt_6-E2": ("pw18_mt_6", [3.0, 22.7]),
    "pw18_mt_6-E20": ("pw18_mt_6", list(np.random.default_rng(7).uniform(1.0, 50.0, 20))),
    "pw10_mt_8-E2": ("pw10_mt_8", [3.0, 22.7]),
    "doublet_mt_136x8-E1": ("doublet_mt_136x8", [14.1]),
    "quartet_yam_24-E3": ("quartet_yam_24", [1.0, 3.0, 10.0]),
    "pw30_mt_4-E3": ("pw30_mt_4", [3.0, 14.1, 22.7]),
    "pw30_mt_4-E12": ("pw30_mt_4", list(np.random.default_rng(3).uniform(4.0, 50.0, 12))),
}

_systems = {}


def _system(name):
    if name not in _systems:
        s = pipeline.build_system(SPECS[name])
        _systems[name] = (s, s.P0geo.full(s.C))
    return _systems[name]


def _lib_lattice(spec):
    L = wp.Lattice(spec.M, spec.N, two_J=spec.two_J, j_max=spec.j_max, swave_only=spec.swave_only,
                   n_x=spec.n_x, n_phi=spec.n_phi)
    if spec.pot == "yamaguchi":
        L.pseudostates(kind="yamaguchi", beta=spec.beta)
    else:
        L.pseudostates(kind="mt", V_R=spec.V_R, mu_R=spec.mu_R, mu_A=spec.mu_A, singlet_ratio=spec.singlet_ratio)
    L.build_perm("fp64")
    return L


@pytest.mark.parametrize("case", list(CASES))
def test_fp64_series_and_amplitudes_match_oracle(case):
    name, Es = CASES[case]
    spec = SPECS[name]
    s, P0full = _system(name)
    L = _lib_lattice(spec)
    # accept: a Pade sum may stop on its rounding plateau once its relative change is below 1e-6
    sol = L.solve(Es, "fp64", tol=1e-12, accept=1e-6, max_iter=300)
    assert sol.converged
    small = spec.M * spec.N * len(s.chans) <= 1000
    worst = 0.0
    for k, E in enumerate(Es):
        ref = pipeline.solve_energy(s, E, P0full=P0full)
        got = sol.amplitude(k)
        for b in range(len(got["A"])):
            d = series_mismatch(sol.series(k, b), ref["series"][b])
            worst = max(worst, d)
            assert d <= SERIES_TOL, (case, E, b, d)
        tol = amplitude_tolerance(ref["series"])
        A = got["A"]
        Ar = pipeline.solve_energy(s, E, direct=True, P0full=P0full)["A"] if small else ref["A"]
        assert np.max(np.abs(A - Ar)) <= tol * np.max(np.abs(Ar)), (case, E, tol, np.max(np.abs(A - Ar)))
    print(f"{case}: max series mismatch {worst:.2e}")


def test_series_terms_are_summed_by_the_host_pade():
    """The amplitude is the Pade (Wynn epsilon) value of the captured terms: the oracle's Wynn table
    run over the library's own terms, up to the term at which the library stopped, gives the
    library's U to rounding (both stop on two successive relative changes <= tol here)."""
    from oracle import lattice as olat, solve as osolve
    spec = SPECS["quartet_yam_24"]
    L = _lib_lattice(spec)
    s, _ = _system("quartet_yam_24")
    for E in (1.0, 3.0, 10.0):
        sol = L.solve([E], "fp64", tol=1e-12)
        a = sol.series(0, 0)[:, 0]
        est, _ = osolve.pade_sum(a)
        q0 = olat.q_onshell(E, spec.h2m)
        j0 = olat.onshell_bin(s.q_edges, q0)
        U = sol.amplitude(0)["A"][0, 0] * (3.0 * spec.h2m * q0) / 2.0 * (s.q_edges[j0 + 1] - s.q_edges[j0])
        # the inverse differences of nearly equal partial sums amplify the last-bit differences of two
        # implementations of complex arithmetic
        assert abs(U - est) <= 1e-11 * abs(est), (E, abs(U - est) / abs(est))
