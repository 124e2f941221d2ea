"""GPU parity of the energy-weight packets (Sec. III.B, footnote to eqs. dg1a, dg1b: weights
w(p) ~ sqrt(p), f(q) ~ sqrt(q)) through the C ABI, against the oracle.

* P0 on every build path the lattices below dispatch (node tables: s-wave; per-box node tables:
  144 nodes; fused MFMA build: 10 and 18 channels with 64 nodes; moment + combine: 10 channels
  with 30 nodes): |dP| <= 1e-12 max|P0|, as for unit weights.
* G1 (closed forms, k_g1_energy) at the library's energy and bins against the oracle's 40-digit
  closed forms: |dG| <= 1e-13 max|G| for every element, below, at and above breakup.
* FP64 solve: series terms and amplitudes to the unit-weight tolerances (tests/parity_util.py);
  S unitary below breakup.
* Mixed path against the FP64 path: |dA| <= 1e-6.
* Continuous batching (G1 per slot at admission): bit-identical alone and in a mix, FP64 and
  split-BF16.
"""
import numpy as np
import pytest

from conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import paper_1404_5253_amd as wp

from oracle import pipeline, resolvent
from parity_util import amplitude_tolerance, series_mismatch

SPECS = {
    "quartet_yam_24": pipeline.Spec(M=24, N=24, two_J=3, pot="yamaguchi", weights="energy"),
    "quartet_yam_ragged_17x13": pipeline.Spec(M=17, N=13, two_J=3, pot="yamaguchi", n_x=6, n_phi=10,
                                              weights="energy"),
    "doublet_mt_nodes144": pipeline.Spec(M=9, N=8, two_J=1, pot="mt", n_x=12, n_phi=12, weights="energy"),
    "doublet_mt_20": pipeline.Spec(M=20, N=20, two_J=1, pot="mt", weights="energy"),
    "pw10_mt_8": pipeline.Spec(M=8, N=8, two_J=1, j_max=1, swave_only=False, pot="mt", weights="energy"),
    "pw18_mt_6": pipeline.Spec(M=6, N=7, two_J=1, j_max=2, swave_only=False, pot="mt", weights="energy"),
    # 30 nodes (not a multiple of four): the moment + combine build instead of the fused one
    "pw10_mt_8_nodes30": pipeline.Spec(M=8, N=8, two_J=1, j_max=1, swave_only=False, pot="mt", n_x=6, n_phi=5,
                                       weights="energy"),
}

_sys = {}


def _system(name):
    if name not in _sys:
        _sys[name] = pipeline.build_system(SPECS[name])
    return _sys[name]


def _lib_lattice(spec, precision="fp64"):
    L = wp.Lattice(spec.M, spec.N, two_J=spec.two_J, j_max=spec.j_max, swave_only=spec.swave_only,
                   n_x=spec.n_x, n_phi=spec.n_phi, weights="energy")
    if spec.pot == "yamaguchi":
        L.pseudostates(kind="yamaguchi", beta=spec.beta)
    else:
        L.pseudostates(kind="mt", V_R=spec.V_R, mu_R=spec.mu_R, mu_A=spec.mu_A, singlet_ratio=spec.singlet_ratio)
    L.build_perm(precision)
    return L


@pytest.mark.parametrize("name", list(SPECS))
def test_energy_p0_matches_oracle(name):
    s = _system(name)
    print(f"energy-weight P0 {name}", flush=True)
    L = _lib_lattice(SPECS[name])
    rp, col, val = L.export_perm()
    got = {}
    for r in range(len(rp) - 1):
        for b in range(rp[r], rp[r + 1]):
            got[(r, int(col[b]))] = val[b]
    P = s.P0geo
    vals = np.einsum("abm,nm->nab", s.C, P.moms)
    ref = {(int(r), int(c)): vals[k] for k, (r, c) in enumerate(zip(P.rows, P.cols))}
    scale = max(np.abs(v).max() for v in ref.values())
    nch = len(s.chans)
    worst = 0.0
    for k in set(got) | set(ref):
        a = got.get(k, np.zeros((nch, nch)))
        b = ref.get(k, np.zeros((nch, nch)))
        worst = max(worst, np.abs(a - b).max())
    assert worst <= 1e-12 * scale, (name, worst / scale)
    assert L.perm_stats["blocks"] == len(got)


@pytest.mark.parametrize("name", ["quartet_yam_24", "pw18_mt_6"])
@pytest.mark.parametrize("E_lab", [1.0, 3.0, 3.336, 3.4, 14.1, 45.0])
def test_energy_g1_matches_oracle(name, E_lab):
    s = _system(name)
    L = _lib_lattice(SPECS[name])
    E_lib = L.eps0 + 2.0 * E_lab / 3.0
    for a, ch in enumerate(L.channels):
        G = L.resolvent(E_lab, a)
        nb, _, _, bins = L.pseudostate_data(a)
        Gq = resolvent.channel_diagonal_energy(s.q_edges, E_lib, [L.eps0] if nb else [], bins)
        err = np.max(np.abs(G - Gq)) / np.max(np.abs(Gq))
        assert err <= 1e-13, (ch, E_lab, err)


@pytest.mark.parametrize("name,Es", [("quartet_yam_24", [1.0, 3.0, 10.0]), ("doublet_mt_20", [3.0, 14.1]),
                                     ("pw18_mt_6", [3.0, 22.7]), ("pw10_mt_8", [9.0])])
def test_energy_fp64_solve_matches_oracle(name, Es):
    s = _system(name)
    spec = SPECS[name]
    L = _lib_lattice(spec)
    sol = L.solve(Es, "fp64", tol=1e-12, accept=1e-6, max_iter=300)
    assert sol.converged
    small = spec.M * spec.N * len(s.chans) <= 1000
    for k, E in enumerate(Es):
        ref = pipeline.solve_energy(s, E)
        got = sol.amplitude(k)
        for b in range(len(got["A"])):
            d = series_mismatch(sol.series(k, b), ref["series"][b])
            assert d <= 1e-10, (name, E, b, d)
        Ar = pipeline.solve_energy(s, E, direct=True)["A"] if small else ref["A"]
        tol = amplitude_tolerance(ref["series"])
        assert np.max(np.abs(got["A"] - Ar)) <= tol * np.max(np.abs(Ar)), (name, E)
        if E < 1.5 * 2.2246 and len(got["S"]) == 1:
            assert abs(abs(got["S"][0, 0]) - 1.0) < 1e-9


@pytest.mark.parametrize("mode", ["mixed", "mixed_split"])
def test_energy_mixed_matches_fp64(mode):
    L = _lib_lattice(SPECS["doublet_mt_20"])
    Es = [1.5, 3.0, 9.0, 14.1, 33.0]
    ref = L.solve(Es, "fp64", accept=1e-6)
    mix = L.solve(Es, mode, tol=1e-8)
    compared = 0
    for k in range(len(Es)):
        a, b = mix.amplitude(k), ref.amplitude(k)
        if max(b["err"]) > 1e-9:
            continue
        assert np.max(np.abs(a["A"] - b["A"])) <= 1e-6, (mode, Es[k])
        compared += 1
    assert compared >= 2


@pytest.mark.parametrize("mode", ["fp64", "mixed_split"])
def test_energy_batch_alone_equals_in_mix(mode):
    """Continuous batching with energy-weight packets (each slot's closed-form G1 computed at
    admission): a request's amplitude is bit-identical alone or among seven others, and agrees with
    the plain solve."""
    from test_gpu_parity import _run_batch
    L = _lib_lattice(SPECS["doublet_mt_20"])
    mix = [3.0, 14.1, 2.5, 40.0, 9.0, 22.7, 1.5, 33.0]
    tol = 1e-12 if mode == "fp64" else 1e-8
    together = _run_batch(L, mix, slots=8, mode=mode, tol=tol)
    assert len(together) == len(mix)
    for E in (3.0, 22.7):
        alone = _run_batch(L, [E], slots=8, mode=mode, tol=tol)[E]
        assert np.array_equal(alone["A"], together[E]["A"]), (mode, E)
        solo = L.solve([E], mode, tol=tol, accept=1e-6).amplitude(0)
        assert np.max(np.abs(alone["A"] - solo["A"])) <= (1e-8 if mode == "fp64" else 1e-6), (mode, E)
