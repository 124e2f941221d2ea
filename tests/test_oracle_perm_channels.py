"""Pins for the oracle's P0 rule beyond s-wave (Appendix, final formula; eq. P_kern).

The channel-pair value of the rule, sum_m C[g, g', m] * moment_m, is checked against the 3D
kernel integrated without the polar substitution, with G taken from the m-scheme evaluation
(explicit spin/isospin permutation matrices and spherical harmonics, no 6j/9j symbols, no moment
exponents). That route shares nothing with the rule's (k, a, b, l, l') moment decomposition, so
a misplaced zeta power, a swapped cos/sin power or a wrong coefficient contraction fails it.

The multichannel operator pins use only the algebra of the exact P on P23-antisymmetric states
(P = C + C^-1, C^3 = 1, eigenvalues 2 and -1): every compression has its spectrum in [-1, 2],
obeys the Bessel bound sum_b P_ab^2 <= 2 + P_aa, and approaches the two eigenvalues and the
identity P^2 = 2 + P as the partial-wave truncation and the lattice grow.
"""
import numpy as np
import pytest

from oracle import channels, lattice, mscheme, perm, recoupling
from oracle.perm import P0Lattice, channel_terms

M6 = 6
# (row channel, column channel) indices into the J = 1/2+, j <= 2 list: l -> l' = 0->3, 0->2,
# 1->3, 2->3, 3->2, 0->1 (lam = 2 -> 3), 2->2 and 1->1
PAIRS = [(0, 17), (2, 13), (4, 17), (8, 16), (16, 8), (3, 11), (9, 14), (1, 1)]


def _chans():
    return channels.enumerate_channels(1, +1, 2)


def _pair_setup(a, b):
    ch = _chans()
    ca, cb = ch[a], ch[b]
    gt = {(0, 0): recoupling.g_table(ca, ca, 1), (0, 1): recoupling.g_table(ca, cb, 1),
          (1, 0): recoupling.g_table(cb, ca, 1), (1, 1): recoupling.g_table(cb, cb, 1)}
    keys, C = channel_terms([ca, cb], gt)
    return ca, cb, keys, C[0, 1]


def _elements(pe, qe, keys, Cab, picks):
    """Cell pairs of the rule's largest, and some smaller, channel-pair values."""
    A = P0Lattice(pe, qe, keys)
    v = A.moms @ Cab
    order = np.argsort(-np.abs(v))
    out = []
    for r in picks:
        idx = order[r]
        j, i = divmod(int(A.rows[idx]), M6)
        jp, ip = divmod(int(A.cols[idx]), M6)
        out.append((i, j, ip, jp))
    return out, float(np.abs(v).max())


@pytest.mark.parametrize("a,b", PAIRS)
def test_rule_converges_to_kernel_integral(a, b):
    """Rule at 160 x 160 nodes vs the 3D kernel with the m-scheme G (semi-analytic), and the
    3D midpoint brute force, on a 6 x 6 lattice."""
    pe, qe = lattice.tangent_edges(M6), lattice.tangent_edges(M6)
    ca, cb, keys, Cab = _pair_setup(a, b)
    G = mscheme.G_polynomial(ca, cb, 1)
    els, vmax = _elements(pe, qe, keys, Cab, (0, 10))
    for (i, j, ip, jp) in els:
        exact = perm.element_semianalytic(pe, qe, i, j, ip, jp, G, ca[0], cb[0], n_sub=48)
        r160 = perm.element_rule_channel(pe, qe, i, j, ip, jp, keys, Cab, 160, 160)
        assert abs(r160 - exact) < 2e-3 * vmax, (ca, cb, (i, j, ip, jp), r160, exact)
        bf = perm.element_bruteforce(pe, qe, i, j, ip, jp, G, ca[0], cb[0], 100)
        assert abs(bf - exact) < 6e-2 * vmax, (ca, cb, (i, j, ip, jp), bf, exact)


def _planted(monkeypatch, fn):
    orig = perm.moment_weight
    monkeypatch.setattr(perm, "moment_weight", lambda nodes, key, weights="unit": orig(nodes, fn(key), weights))


@pytest.mark.parametrize("mistake", ["zeta_powers_swapped", "cos_sin_powers_swapped"])
def test_planted_exponent_mistakes_are_caught(monkeypatch, mistake):
    """Two plausible misreadings of the final formula, planted in the oracle's moment weight,
    each break the kernel-integral pin (while P0 = P0^T holds for both)."""
    fn = {"zeta_powers_swapped": lambda k: (k[0], k[1], k[2], k[4], k[3]),
          "cos_sin_powers_swapped": lambda k: (k[0], k[2], k[1], k[3], k[4])}[mistake]
    pe, qe = lattice.tangent_edges(M6), lattice.tangent_edges(M6)
    worst = 0.0
    for a, b in [(0, 17), (8, 16)]:
        ca, cb, keys, Cab = _pair_setup(a, b)
        G = mscheme.G_polynomial(ca, cb, 1)
        els, vmax = _elements(pe, qe, keys, Cab, (0, 3))
        exact = [perm.element_semianalytic(pe, qe, *e, G, ca[0], cb[0], n_sub=48) for e in els]
        with monkeypatch.context() as mp:
            _planted(mp, fn)
            wrong = [perm.element_rule_channel(pe, qe, *e, keys, Cab, 160, 160) for e in els]
        worst = max(worst, max(abs(w - x) for w, x in zip(wrong, exact)) / vmax)
    assert worst > 2e-2


def _full(M, chans, two_J, n):
    pe, qe = lattice.tangent_edges(M), lattice.tangent_edges(M)
    gt = {(a, b): recoupling.g_table(chans[a], chans[b], two_J)
          for a in range(len(chans)) for b in range(len(chans))}
    keys, C = channel_terms(chans, gt)
    return P0Lattice(pe, qe, keys, n_x=n, n_phi=n).full(C).toarray()


@pytest.mark.parametrize("j_max", [1, 2])
def test_multichannel_operator_bounds(j_max):
    """10 and 18 channels (J = 1/2+), high-order rule: symmetric, spectrum in [-1, 2], and the
    Bessel row bound."""
    P = _full(6, channels.enumerate_channels(1, +1, j_max), 1, 24)
    assert abs(P - P.T).max() < 1e-12 * abs(P).max()
    ev = np.linalg.eigvalsh(0.5 * (P + P.T))
    assert ev[0] > -1.0 - 2e-3 and ev[-1] < 2.0 + 2e-3
    assert np.all((P * P).sum(axis=1) <= 2.0 + np.diag(P) + 2e-3)


def test_identity_gap_shrinks_with_partial_waves():
    """Rows of the two channels present for every j_max: the Bessel gap 2 + P_aa - sum_b P_ab^2
    (zero for P^2 = 2 + P) decreases strictly from j_max = 0 to 1 to 2, and the spectrum edges
    move towards -1 and 2."""
    gaps, lo, hi = [], [], []
    D = M6 * M6
    for j_max in (0, 1, 2):
        P = _full(M6, channels.enumerate_channels(1, +1, j_max), 1, 24)
        gap = 2.0 + np.diag(P) - (P * P).sum(axis=1)
        gaps.append(gap[:2 * D].sum())
        ev = np.linalg.eigvalsh(0.5 * (P + P.T))
        lo.append(ev[0])
        hi.append(ev[-1])
    assert gaps[0] > gaps[1] > gaps[2] > 0.0
    assert lo[0] > lo[1] > lo[2] > -1.0 - 2e-3
    assert hi[0] < hi[1] < hi[2] < 2.0 + 2e-3


def test_spectrum_edges_approach_the_exact_eigenvalues():
    """18 channels: as M = N grows 4 -> 6 -> 8 -> 10 the extreme eigenvalues of the compression
    approach the exact P's -1 and 2 from inside."""
    lo, hi = [], []
    for M in (4, 6, 8, 10):
        P = _full(M, _chans(), 1, 16)
        ev = np.linalg.eigvalsh(0.5 * (P + P.T))
        lo.append(ev[0])
        hi.append(ev[-1])
    assert all(a > b for a, b in zip(lo, lo[1:])) and lo[-1] > -1.0 - 2e-3
    assert all(a < b for a, b in zip(hi, hi[1:])) and hi[-1] < 2.0 + 2e-3
    assert lo[-1] < -0.96 and hi[-1] > 1.92
