"""Pins for the oracle's elastic nd observables (Sec. IV: the I -> Sigma transformation, phase
shifts, differential cross section, neutron analysing power).

* The printed transformation equals the m-scheme overlap <(j 1/2) Sigma, lam; J | j, (lam 1/2) I; J>
  (explicit Clebsch-Gordan sums over projections) for every lam <= 4 and J <= 9/2; the three other
  coupling orders of the channel-spin state disagree with it in sign somewhere (so the pin fixes the
  convention the amplitude is written in).
* The amplitude built in the channel-spin basis and the one built in the product basis (m_d, sigma)
  straight from the jj channels (no Sigma step) give the same dsigma/dOmega and A_y.
* int dsigma/dOmega dOmega equals the partial-wave sum (pi/k^2) sum (2J+1)/6 |S - 1|^2, and for a
  unitary S the optical theorem (4 pi / k) Im Tr M(0) / 6.
* Two s-wave blocks alone give the textbook isotropic (1/k^2)(1/3 sin^2 delta_d + 2/3 sin^2 delta_q)
  with A_y = 0; A_y vanishes at 0 and 180 degrees.
* Eigenphases reconstruct S.
"""
import numpy as np
import pytest
from sympy import Rational
from sympy.physics.wigner import clebsch_gordan

from oracle import channels
from oracle import observables as ob

H = Rational(1, 2)


def _cg(j1, m1, j2, m2, j3, m3):
    return clebsch_gordan(j1, j2, j3, m1, m2, m3)


def _overlap(lam, I, J, Sg, order):
    """<Sigma state | jj state> at M = J; order 'c' = (j 1/2) Sigma then lam, the others permuted."""
    M = J
    jj = {}
    for md in (-1, 0, 1):
        mI = M - md
        if abs(mI) > I:
            continue
        for sg in (H, -H):
            ml = mI - sg
            if abs(ml) <= lam:
                jj[(md, ml, sg)] = _cg(1, md, I, mI, J, M) * _cg(lam, ml, H, sg, I, mI)
    tot = 0
    for (md, ml, sg), v in jj.items():
        nu = md + sg
        if abs(nu) > Sg:
            continue
        spin = _cg(1, md, H, sg, Sg, nu) if order in "ac" else _cg(H, sg, 1, md, Sg, nu)
        orb = _cg(Sg, nu, lam, ml, J, M) if order in "cd" else _cg(lam, ml, Sg, nu, J, M)
        tot += v * spin * orb
    return float(tot)


def test_printed_transformation_is_the_channel_spin_overlap():
    bad = {"a": 0, "b": 0, "d": 0}
    n = 0
    for two_J in range(1, 10, 2):
        for par in (1, -1):
            chans = [(c[3], c[4]) for c in channels.enumerate_channels(two_J, par, 1)
                     if c[0] == 0 and c[1] == 1 and c[2] == 1]
            sig, T = ob.sigma_transform(two_J, chans)
            assert np.allclose(T @ T.T, np.eye(len(sig)), atol=1e-14)
            for a, (lam, two_S) in enumerate(sig):
                for b, (lamb, two_I) in enumerate(chans):
                    if lam != lamb:
                        continue
                    args = (lam, Rational(two_I, 2), Rational(two_J, 2), Rational(two_S, 2))
                    assert abs(T[a, b] - _overlap(*args, "c")) < 1e-14, (two_J, par, lam, two_I, two_S)
                    for o in bad:
                        bad[o] += abs(T[a, b] - _overlap(*args, o)) > 1e-12
                    n += 1
    assert n > 30 and all(v > 0 for v in bad.values()), bad


def _blocks(seed, twoJs=(1, 3, 5, 7), unitary=True):
    rng = np.random.default_rng(seed)
    out = []
    for two_J in twoJs:
        for par in (1, -1):
            chans = [(c[3], c[4]) for c in channels.enumerate_channels(two_J, par, 1)
                     if c[0] == 0 and c[1] == 1 and c[2] == 1]
            n = len(chans)
            O, _ = np.linalg.qr(rng.normal(size=(n, n)))
            d = np.exp(2j * rng.uniform(-1.5, 1.5, n))
            if not unitary:
                d *= rng.uniform(0.5, 1.0, n)
            out.append((two_J, chans, O @ np.diag(d) @ O.T))
    return out


@pytest.mark.parametrize("unitary", [True, False])
def test_channel_spin_and_product_basis_routes_agree(unitary):
    blocks = _blocks(1, unitary=unitary)
    k = 0.6
    th = np.linspace(0.03, np.pi - 0.03, 9)
    ds, ay = ob.observables(blocks, k, th)
    syp = ob.sigma_y_product_basis()
    for t, d0, a0 in zip(th, ds, ay):
        M = ob.amplitude_product_basis(blocks, k, t)
        den = np.trace(M @ M.conj().T).real
        assert abs(den / 6.0 - d0) <= 1e-12 * d0
        assert abs((np.trace(M @ syp @ M.conj().T) / den).real - a0) <= 1e-12


def test_integrated_cross_section_and_optical_theorem():
    blocks = _blocks(2)
    k = 0.45
    x, w = np.polynomial.legendre.leggauss(48)
    ds, ay = ob.observables(blocks, k, np.arccos(x))
    integral = 2.0 * np.pi * float(np.sum(w * ds))
    pw = ob.elastic_cross_section_partial_waves(blocks, k)
    assert abs(integral - pw) <= 1e-11 * pw
    M0 = ob.amplitude_sigma([(tJ,) + ob.to_sigma(tJ, c, S) for tJ, c, S in blocks], k, 0.0)
    assert abs(4.0 * np.pi / k * np.trace(M0).imag / 6.0 - pw) <= 1e-11 * pw
    _, ay_ends = ob.observables(blocks, k, np.array([0.0, np.pi]))
    assert np.max(np.abs(ay_ends)) <= 1e-12


def test_swave_blocks_give_the_textbook_cross_section():
    dd, dq = 0.7, -1.1
    blocks = [(1, [(0, 1)], np.array([[np.exp(2j * dd)]])), (3, [(0, 1)], np.array([[np.exp(2j * dq)]]))]
    k = 0.3
    th = np.linspace(0.0, np.pi, 5)
    ds, ay = ob.observables(blocks, k, th)
    ref = (np.sin(dd) ** 2 / 3.0 + 2.0 * np.sin(dq) ** 2 / 3.0) / k ** 2
    assert np.allclose(ds, ref, rtol=1e-13)
    assert np.max(np.abs(ay)) <= 1e-14


def test_eigenphases_reconstruct_s():
    for two_J, chans, S in _blocks(3):
        d, O = ob.eigenphases(S)
        assert np.allclose(O @ np.diag(np.exp(2j * d)) @ O.T, S, atol=1e-13)
        assert np.allclose(O.T @ O, np.eye(len(d)), atol=1e-13)


def _spin_free_blocks(s_lam, two_J_max=9):
    """Blocks whose channel-spin S is s_lam[lam] on the diagonal for every J and Sigma (scattering
    that does not see the spins), returned in the jj basis (S_jj = T^T S_Sigma T)."""
    out = []
    for two_J in range(1, two_J_max + 1, 2):
        for par in (1, -1):
            chans = [(c[3], c[4]) for c in channels.enumerate_channels(two_J, par, 1)
                     if c[0] == 0 and c[1] == 1 and c[2] == 1]
            sig, T = ob.sigma_transform(two_J, chans)
            Ss = np.diag([s_lam[lam] for lam, _ in sig])
            out.append((two_J, chans, T.T @ Ss @ T))
    return out


def spinless_cross_section(s_lam, k, theta):
    """|f|^2 with f = sum_lam (2 lam + 1) (s_lam - 1) / (2 i k) P_lam(cos theta)."""
    from numpy.polynomial import legendre
    c = [(2 * l + 1) * (s_lam[l] - 1.0) / (2j * k) for l in range(len(s_lam))]
    return np.abs(legendre.legval(np.cos(theta), c)) ** 2


def test_spin_free_scattering_has_no_analysing_power():
    """S independent of Sigma and J (per lam): the amplitude is spin-independent, A_y = 0 and
    dsigma/dOmega is the spinless |f|^2."""
    rng = np.random.default_rng(4)
    # lam <= 3 scatter: up to J = 9/2 every (lam, Sigma, J) of these lam is present; higher lam
    # (incomplete shells) do not scatter
    s_lam = np.ones(8, dtype=complex)
    s_lam[:4] = np.exp(2j * rng.uniform(-1.2, 1.2, 4)) * rng.uniform(0.6, 1.0, 4)
    blocks = _spin_free_blocks(s_lam)
    th = np.linspace(0.0, np.pi, 11)
    k = 0.8
    ds, ay = ob.observables(blocks, k, th)
    assert np.max(np.abs(ay)) <= 1e-12
    assert np.allclose(ds, spinless_cross_section(s_lam, k, th), rtol=1e-11)
