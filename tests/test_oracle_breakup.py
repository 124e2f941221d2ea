"""Pins of the oracle's breakup elements (oracle.pipeline.breakup_elements), CPU only.

* The elements come from the factorised lattice-space solve y = b + K y rotated to the SWP basis
  (z = O y). An independent route solves the matrix equation U = P V1 + P V1 G1 U (eq. m_pvg)
  directly in the SWP basis, with P V1 = O P0 v O^T assembled as an explicit dense matrix, and
  must give the same z on every cell (breakup cells and the elastic element alike).
* The cells are those where the oracle's G1 has an imaginary part; they must be exactly the cells
  whose corner energies h2m p^2 + (3/4) h2m q^2 straddle E (the energy shell crosses the cell).
* Below the breakup threshold there is no such cell.
"""
import numpy as np
import pytest

from oracle import lattice, pipeline, solve

SPEC = pipeline.Spec(M=7, N=6, two_J=1, pot="mt")


@pytest.fixture(scope="module")
def sysm():
    return pipeline.build_system(SPEC)


def _swp_route(s, E_lab):
    """z = (I - A G1)^{-1} A e0 in the SWP basis (g, j, k), A = O P0 W as a dense matrix."""
    E = lattice.total_energy(E_lab, s.eps0)
    q0 = lattice.q_onshell(E_lab, SPEC.h2m)
    j0 = lattice.onshell_bin(s.q_edges, q0)
    M, N, n = SPEC.M, SPEC.N, len(s.chans)
    P0 = s.P0geo.full(s.C).toarray()
    D = n * N * M
    Ob = np.zeros((D, D))   # z[g, j, k] = sum_i O_g[k, i] y[g, j, i]
    Wb = np.zeros((D, D))   # s[g, j, i] = sum_k W_g[i, k] z[g, j, k]
    G1 = pipeline.g1_lists(s, E)
    gdiag = np.zeros(D, dtype=complex)
    for g, c in enumerate(s.chans):
        d = s.pair[(c[0], c[1])]
        for j in range(N):
            base = (g * N + j) * M
            Ob[base:base + M, base:base + M] = d["O"]
            Wb[base:base + M, base:base + M] = d["W"]
            gdiag[base:base + M] = G1[(c[0], c[1])][:, j]
    A = Ob @ P0 @ Wb
    out = {}
    for b, g0 in enumerate(pipeline.initial_channels(s)):
        e0 = np.zeros(D)
        e0[(g0 * N + j0) * M + 0] = 1.0
        z = np.linalg.solve(np.eye(D) - A * gdiag[None, :], A @ e0)
        out[b] = z.reshape(n, N, M)
    return out, j0


def test_breakup_elements_match_the_swp_basis_solve(sysm):
    E_lab = 22.7
    cells, el = pipeline.breakup_elements(sysm, E_lab)
    assert len(cells) > 0
    z, j0 = _swp_route(sysm, E_lab)
    for b in el:
        ref = np.array([z[b][g, j, k] for (g, k, j) in cells])
        assert np.max(np.abs(el[b] - ref)) <= 1e-12 * np.max(np.abs(ref)), b
        # the elastic element of the same solution is the one the amplitude uses
        U = pipeline.solve_energy(sysm, E_lab, direct=True)["U"]
        g0 = pipeline.initial_channels(sysm)[b]
        assert abs(z[b][g0, j0, 0] - U[b, b]) <= 1e-12 * abs(U[b, b])


def test_breakup_cells_are_the_energy_shell(sysm):
    E_lab = 22.7
    E = lattice.total_energy(E_lab, sysm.eps0)
    cells, _ = pipeline.breakup_elements(sysm, E_lab)
    h, b3 = SPEC.h2m, 0.75 * SPEC.h2m
    want = []
    for g, c in enumerate(sysm.chans):
        d = sysm.pair[(c[0], c[1])]
        nb, bins = d["nb"], d["bins"]
        for k in range(nb, SPEC.M):
            pa, pb = bins[k - nb], bins[k - nb + 1]
            for j in range(SPEC.N):
                qa, qb = sysm.q_edges[j], sysm.q_edges[j + 1]
                if h * pa * pa + b3 * qa * qa < E < h * pb * pb + b3 * qb * qb:
                    want.append((g, k, j))
    assert cells == want


def test_no_breakup_cells_below_threshold(sysm):
    cells, el = pipeline.breakup_elements(sysm, 1.0)   # E_lab = 1 MeV < 3.34 MeV breakup threshold
    assert cells == []
