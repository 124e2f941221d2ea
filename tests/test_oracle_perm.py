"""Pins for the oracle's P0 (Appendix): selection, rule, symmetry, exact values, operator bounds."""
import numpy as np
import pytest

from oracle import channels, lattice, perm, recoupling
from oracle.perm import P0Lattice, channel_terms

S_KEY = (0, 0, 0, 0, 0)


def _grid(M, N=None):
    return lattice.tangent_edges(M), lattice.tangent_edges(N or M)


def test_candidate_set_equals_exhaustive():
    pe, qe = _grid(12)
    chans = channels.enumerate_channels(1, +1, 1)
    gt = {(a, b): recoupling.g_table(chans[a], chans[b], 1) for a in range(3) for b in range(3)}
    keys, _ = channel_terms(chans[:3], gt)
    A = P0Lattice(pe, qe, keys, exhaustive=True)
    B = P0Lattice(pe, qe, keys, exhaustive=False)
    assert np.array_equal(A.rows, B.rows) and np.array_equal(A.cols, B.cols)
    assert np.allclose(A.moms, B.moms, rtol=1e-13, atol=1e-15)


def test_rule_symmetry_and_fill():
    pe, qe = _grid(20)
    P = P0Lattice(pe, qe, [S_KEY]).full(np.ones((1, 1, 1)))
    assert abs(P - P.T).max() < 1e-13 * abs(P).max()
    fill = P.nnz / P.shape[0] ** 2
    assert 0.002 < fill < 0.1     # the paper quotes about 1% on its own lattices


def test_multichannel_symmetry():
    """P0^{gg'}_{ab} = P0^{g'g}_{ba} for l > 0 channels (phi -> pi/2 - phi maps the rule onto itself)."""
    pe, qe = _grid(8)
    chans = channels.enumerate_channels(1, +1, 1)
    gt = {(a, b): recoupling.g_table(chans[a], chans[b], 1)
          for a in range(len(chans)) for b in range(len(chans))}
    keys, C = channel_terms(chans, gt)
    P = P0Lattice(pe, qe, keys).full(C)
    assert abs(P - P.T).max() < 1e-12 * abs(P).max()


@pytest.mark.parametrize("seed", [0, 1])
def test_rule_converges_to_semianalytic_and_bruteforce(seed):
    pe, qe = _grid(6)
    A = P0Lattice(pe, qe, [S_KEY])
    rng = np.random.default_rng(seed)
    for idx in rng.choice(A.geo_nnz, 2, replace=False):
        j, i = divmod(int(A.rows[idx]), 6)
        jp, ip = divmod(int(A.cols[idx]), 6)
        exact = perm.element_semianalytic_s(pe, qe, i, j, ip, jp)
        r8 = perm.element_rule(pe, qe, i, j, ip, jp, S_KEY, 8, 8)
        assert r8 == pytest.approx(A.moms[idx, 0], rel=1e-14)
        r160 = perm.element_rule(pe, qe, i, j, ip, jp, S_KEY, 160, 160)
        assert abs(r160 - exact) < 2e-3 * abs(exact) + 1e-6
        bf = perm.element_bruteforce_s(pe, qe, i, j, ip, jp, 160)
        assert abs(bf - exact) < 3e-2 * abs(exact) + 1e-5


def _high_order_swave(M, C, n=24):
    pe, qe = _grid(M)
    return P0Lattice(pe, qe, [S_KEY], n_x=n, n_phi=n).full(C).toarray()


@pytest.mark.parametrize("name", ["quartet", "doublet"])
def test_operator_bounds(name):
    """On P23-antisymmetric states P = C + C^-1 with C^3 = 1: spectrum {-1, 2}, P^2 = 2 + P.

    Any compression (finite lattice, truncated channels) keeps its spectrum in [-1, 2] and obeys
    the Bessel row bound sum_b P_ab^2 <= 2 + P_aa.
    """
    ch = channels.swave_quartet() if name == "quartet" else channels.swave_doublet()
    two_J = 3 if name == "quartet" else 1
    n = len(ch)
    C = np.zeros((n, n, 1))
    for a in range(n):
        for b in range(n):
            C[a, b, 0] = recoupling.g_table(ch[a], ch[b], two_J).get((0, 0, 0), 0.0)
    P = _high_order_swave(10, C)
    ev = np.linalg.eigvalsh(0.5 * (P + P.T))
    assert ev[0] > -1.0 - 2e-3 and ev[-1] < 2.0 + 2e-3
    row = (P * P).sum(axis=1)
    assert np.all(row <= 2.0 + np.diag(P) + 2e-3)


def test_planted_mistake_is_caught():
    """A sign error in zeta2 (a plausible slip) breaks the exact-value pin."""
    pe, qe = _grid(6)
    i, j, ip, jp = 3, 4, 4, 4
    exact = perm.element_semianalytic_s(pe, qe, i, j, ip, jp)
    orig = perm.box_nodes

    def bad(q_edges, j_, jp_, nx, nphi):
        d = orig(q_edges, j_, jp_, nx, nphi)
        c, s, X = d["c"], d["s"], d["x"]
        d["z2"] = np.sqrt(0.25 * c * c + s * s - X * c * s)
        return d
    perm.box_nodes = bad
    try:
        wrong = perm.element_rule(pe, qe, i, j, ip, jp, S_KEY, 160, 160)
    finally:
        perm.box_nodes = orig
    assert abs(wrong - exact) > 1e-2 * abs(exact)
