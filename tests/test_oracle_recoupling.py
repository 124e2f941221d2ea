"""Pins for the oracle's channel algebra and recoupling coefficients (Appendix, eqs. ggaga, gal).

The m-scheme evaluation (explicit three-nucleon spin and isospin spaces, explicit cyclic
permutation matrices, spherical harmonics) shares nothing with the 6j/9j formula of eq. gal.
"""
import numpy as np
import pytest

from oracle import channels, mscheme, recoupling


def test_channel_counts_match_paper():
    # 18 channels for J = 1/2+ with all pair waves j <= 2 (Sec. V.B, the J = 1/2+ run)
    assert len(channels.enumerate_channels(1, +1, 2)) == 18
    assert len(channels.enumerate_channels(1, +1, 1)) == 10
    assert len(channels.enumerate_channels(1, +1, 0)) == 2
    for c in channels.enumerate_channels(1, +1, 3):
        l, s, j, lam, two_I, t = c
        assert (l + s + t) % 2 == 1
        assert (-1) ** (l + lam) == 1


def test_swave_constants():
    q = channels.swave_quartet()
    assert q == [(0, 1, 1, 0, 1, 0)]
    assert recoupling.g_table(q[0], q[0], 3) == pytest.approx({(0, 0, 0): -0.5}, abs=1e-15)
    d = channels.swave_doublet()
    expect = [[0.25, -0.75], [-0.75, 0.25]]
    for a in range(2):
        for b in range(2):
            tab = recoupling.g_table(d[a], d[b], 1)
            assert tab[(0, 0, 0)] == pytest.approx(expect[a][b], abs=1e-15)


def _pairs(chans, n):
    rng = np.random.default_rng(7)
    idx = [(a, b) for a in range(len(chans)) for b in range(len(chans))]
    sel = rng.choice(len(idx), min(n, len(idx)), replace=False)
    return [idx[i] for i in sel]


@pytest.mark.parametrize("two_J,j_max,npairs", [(1, 1, 100), (1, 2, 40), (3, 2, 30)])
def test_gal_matches_mscheme(two_J, j_max, npairs):
    chans = channels.enumerate_channels(two_J, +1, j_max)
    rng = np.random.default_rng(11)
    for a, b in _pairs(chans, npairs):
        tab = recoupling.g_table(chans[a], chans[b], two_J)
        q, qp, x = rng.uniform(0.2, 2.0), rng.uniform(0.2, 2.0), rng.uniform(-1, 1)
        re, im = mscheme.G_mscheme(chans[a], chans[b], two_J, q, qp, x)
        gf = recoupling.G_from_table(tab, chans[a], chans[b], q, qp, x)
        assert abs(im) < 1e-12
        assert gf == pytest.approx(re, abs=1e-12), (chans[a], chans[b])


def test_printed_exponent_order_fails_the_pin():
    """The q/q' exponents as printed in eq. ggaga (q^(l2+l2') q'^(l1+l1')) disagree with G."""
    from numpy.polynomial import legendre as L
    chans = channels.enumerate_channels(1, +1, 1)
    a, b = chans[0], chans[4]   # 1S0 and 1P1 with lam = 1: l' = 1
    tab = recoupling.g_table(a, b, 1)
    q, qp, x = 0.7, 1.3, 0.3
    re, _ = mscheme.G_mscheme(a, b, 1, q, qp, x)
    mirrored = sum(v * q ** ((a[0] - l1) + (b[0] - l1p)) * qp ** (l1 + l1p) * L.legval(x, [0] * k + [1])
                   for (l1, l1p, k), v in tab.items())
    assert abs(mirrored - re) > 1e-3


def test_g_transpose_symmetry():
    """P = P^T implies G_{gg'}(q, q', x) = G_{g'g}(q', q, x)."""
    chans = channels.enumerate_channels(1, +1, 2)
    rng = np.random.default_rng(3)
    for a, b in _pairs(chans, 60):
        q, qp, x = rng.uniform(0.2, 2.0), rng.uniform(0.2, 2.0), rng.uniform(-1, 1)
        t_ab = recoupling.g_table(chans[a], chans[b], 1)
        t_ba = recoupling.g_table(chans[b], chans[a], 1)
        g1 = recoupling.G_from_table(t_ab, chans[a], chans[b], q, qp, x)
        g2 = recoupling.G_from_table(t_ba, chans[b], chans[a], qp, q, x)
        assert g1 == pytest.approx(g2, abs=1e-12)
