"""Pins for the oracle's lattice, kinematics, potentials and pseudostates."""
import mpmath
import numpy as np
import pytest
from scipy import integrate, optimize

from oracle import lattice, potential, pseudostates

H = lattice.H2M


def test_tangent_grid_and_h0():
    e = lattice.tangent_edges(40)
    assert e[0] == 0.0 and e[-1] == pytest.approx(10.0, abs=0)
    assert np.all(np.diff(e) > 0)
    h0 = lattice.h0_diagonal(e)
    for i in (0, 7, 39):
        val, _ = integrate.quad(lambda p: H * p * p, e[i], e[i + 1])
        assert h0[i] == pytest.approx(val / (e[i + 1] - e[i]), rel=1e-13)


def test_kinematics_threshold_and_bin():
    # breakup threshold: E = eps0 + (2/3) E_lab = 0 at E_lab = 1.5 * 2.2246
    assert lattice.total_energy(1.5 * 2.2246, -2.2246) == pytest.approx(0.0, abs=1e-15)
    q0 = lattice.q_onshell(10.0)
    assert 0.75 * H * q0 ** 2 == pytest.approx(2.0 * 10.0 / 3.0, rel=1e-14)
    e = lattice.tangent_edges(40)
    j0 = lattice.onshell_bin(e, q0)
    assert e[j0] < q0 <= e[j0 + 1]
    assert lattice.onshell_bin(e, e[5]) == 4          # half-open (q_{j-1}, q_j]


def test_yamaguchi_secular_roots():
    """Rank-1 potential: eigenvalues solve 1 = lam sum_i G_i^2 / (e_i - eps) (no eigh)."""
    e = lattice.tangent_edges(30)
    beta = 1.394
    lam = potential.tune_yamaguchi(e, beta, 2.2246)
    G = potential.yamaguchi_form(e)(beta)
    h0 = lattice.h0_diagonal(e)
    f = lambda x: 1.0 - lam * np.sum(G * G / (h0 - x))
    roots = [optimize.brentq(f, -200.0, h0[0] - 1e-12, xtol=1e-14, rtol=1e-15)]
    for i in range(3):
        roots.append(optimize.brentq(f, h0[i] + 1e-9, h0[i + 1] - 1e-9, xtol=1e-14, rtol=1e-15))
    eps, O = pseudostates.diagonalize(e, potential.yamaguchi_wp(e, beta, lam))
    assert roots[0] == pytest.approx(-2.2246, abs=1e-10)
    assert np.allclose(eps[:4], roots, rtol=1e-11, atol=1e-11)
    assert np.allclose(O @ O.T, np.eye(len(eps)), atol=1e-13)


def test_yamaguchi_strength_tends_to_continuum_value():
    """lam -> 4 H beta (beta + kappa)^2 / pi (continuum bound-state condition) as M grows."""
    beta = 1.394
    kappa = np.sqrt(2.2246 / H)
    lam_star = 4.0 * H * beta * (beta + kappa) ** 2 / np.pi
    errs = [abs(potential.tune_yamaguchi(lattice.tangent_edges(M), beta, 2.2246) / lam_star - 1.0)
            for M in (20, 80)]
    assert errs[1] < errs[0] and errs[1] < 0.02


def test_yukawa_gauss_vs_closed_form():
    e = lattice.tangent_edges(24)
    a = potential.yukawa_wp(e, 0, 1.55, n_gauss=32)
    b = potential.yukawa_wp_swave_closed(e, 1.55)
    assert np.allclose(a, b, rtol=1e-11, atol=1e-13)


@pytest.mark.parametrize("l", [0, 1, 2, 3])
def test_legendre_q_vs_mpmath(l):
    for z in (1.001, 1.3, 1.99, 2.01, 7.5, 400.0):
        ref = float(mpmath.legenq(l, 0, z, type=3).real)
        assert potential.legendre_q(l, np.array([z]))[0] == pytest.approx(ref, rel=1e-11)


def _numerov_bound_VA(V_R, mu_R, mu_A, BE, rmax=30.0, n=30000):
    """V_A giving an l = 0 bound state at -BE in r space (shooting, independent of the WP basis)."""
    r = np.linspace(rmax / n, rmax, n)
    h = r[1] - r[0]
    kap2 = BE / H

    def end_value(VA):
        V = (V_R * np.exp(-mu_R * r) - VA * np.exp(-mu_A * r)) / r
        k = -(V / H + kap2)   # u'' = (V/H + kappa^2) u
        u = np.zeros(n)
        u[0], u[1] = r[0], r[1]
        for i in range(1, n - 1):
            u[i + 1] = (2 * u[i] * (1 - 5 * h * h * k[i] / 12) - u[i - 1] * (1 + h * h * k[i - 1] / 12)) / (1 + h * h * k[i + 1] / 12)
        return u[-1] * np.exp(-np.sqrt(kap2) * 0)  # sign change marks the eigenvalue
    return optimize.brentq(end_value, 400.0, 900.0, xtol=1e-8)


def test_mt_strength_vs_numerov():
    """The WP-basis tuned V_A approaches the r-space value as the lattice grows."""
    V_R = 1438.72
    ref = _numerov_bound_VA(V_R, 3.11, 1.55, 2.2246)
    vals = [potential.tune_mt(lattice.tangent_edges(M), V_R, 3.11, 1.55, 2.2246) for M in (40, 120)]
    assert abs(vals[1] - ref) < abs(vals[0] - ref) + 1e-9
    assert vals[1] == pytest.approx(ref, rel=0.01)


def test_scattering_bins_contain_pseudostates():
    e = lattice.tangent_edges(30)
    v = potential.yamaguchi_wp(e, 1.394, potential.tune_yamaguchi(e, 1.394, 2.2246))
    eps, _ = pseudostates.diagonalize(e, v)
    b = pseudostates.scattering_bins(eps[1:])
    ps = np.sqrt(eps[1:] / H)
    assert b[0] == 0.0 and np.all((b[:-1] < ps) & (ps < b[1:]))
