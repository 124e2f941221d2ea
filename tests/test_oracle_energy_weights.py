"""Pins for the oracle's energy-weight packets (Sec. III.B, footnote to eqs. dg1a, dg1b: weights
w(p) ~ sqrt(p), f(q) ~ sqrt(q), for which the channel resolvent has closed formulas).

* P0: the rule with F = U^4 - L^4, the node factor sqrt(cos sin zeta1 zeta2) and the norm from the
  squared-momentum widths, against the 3D kernel integrated with the weights and energy widths
  applied as defined (semi-analytic and midpoint routes), s-wave and l, l' > 0 channel pairs; a
  planted omission of the node factor or of the U^2 + L^2 term fails it.
* G1: the closed forms (40-digit) against direct quadrature off the shell, against a 1D quadrature
  of the inner logarithm on the shell, and the i0 prescription against E + i eta as eta -> 0; the
  bound-continuum row against a Cauchy principal-value quadrature.
* Two-body: the energy-weight h0 and potential matrices against adaptive quadrature of their
  defining integrals.
* End to end: S = 1 - 2 pi i A with A = U / B_j0 is unitary below breakup to rounding.
"""
import mpmath
import numpy as np
import pytest
from scipy import integrate

from oracle import channels, lattice, mscheme, perm, pipeline, potential, recoupling, resolvent
from oracle.perm import P0Lattice, channel_terms

H = lattice.H2M
M6 = 6


def _top_elements(pe, qe, keys, Cab, picks, weights):
    A = P0Lattice(pe, qe, keys, weights=weights)
    v = A.moms @ Cab
    order = np.argsort(-np.abs(v))
    out = []
    for r in picks:
        idx = order[r]
        j, i = divmod(int(A.rows[idx]), M6)
        jp, ip = divmod(int(A.cols[idx]), M6)
        out.append((i, j, ip, jp))
    return out, float(np.abs(v).max())


def _pair(a, b):
    ch = channels.enumerate_channels(1, +1, 2)
    ca, cb = ch[a], ch[b]
    gt = {(0, 0): recoupling.g_table(ca, ca, 1), (0, 1): recoupling.g_table(ca, cb, 1),
          (1, 0): recoupling.g_table(cb, ca, 1), (1, 1): recoupling.g_table(cb, cb, 1)}
    keys, C = channel_terms([ca, cb], gt)
    return ca, cb, keys, C[0, 1]


@pytest.mark.parametrize("a,b", [(0, 0), (0, 17), (2, 13), (8, 16)])
def test_energy_rule_converges_to_kernel_integral(a, b):
    pe, qe = lattice.tangent_edges(M6), lattice.tangent_edges(M6)
    ca, cb, keys, Cab = _pair(a, b)
    G = mscheme.G_polynomial(ca, cb, 1)
    els, vmax = _top_elements(pe, qe, keys, Cab, (0, 10), "energy")
    for (i, j, ip, jp) in els:
        exact = perm.element_semianalytic(pe, qe, i, j, ip, jp, G, ca[0], cb[0], n_sub=48, weights="energy")
        r160 = perm.element_rule_channel(pe, qe, i, j, ip, jp, keys, Cab, 160, 160, weights="energy")
        assert abs(r160 - exact) < 2e-3 * vmax, (ca, cb, (i, j, ip, jp), r160, exact)
        bf = perm.element_bruteforce(pe, qe, i, j, ip, jp, G, ca[0], cb[0], 100, weights="energy")
        assert abs(bf - exact) < 6e-2 * vmax, (ca, cb, (i, j, ip, jp), bf, exact)


@pytest.mark.parametrize("mistake", ["node_factor", "F_square_sum"])
def test_planted_energy_mistakes_are_caught(monkeypatch, mistake):
    pe, qe = lattice.tangent_edges(M6), lattice.tangent_edges(M6)
    ca, cb, keys, Cab = _pair(0, 17)
    G = mscheme.G_polynomial(ca, cb, 1)
    els, vmax = _top_elements(pe, qe, keys, Cab, (0, 10), "energy")
    exact = [perm.element_semianalytic(pe, qe, *e, G, ca[0], cb[0], n_sub=48, weights="energy") for e in els]
    if mistake == "node_factor":
        orig = perm.moment_weight
        monkeypatch.setattr(perm, "moment_weight", lambda n, k, w="unit": orig(n, k, "unit"))
    else:
        orig = perm.F_values
        monkeypatch.setattr(perm, "F_values",
                            lambda pe_, n, ii, iip, w="unit": 2.0 * orig(pe_, n, ii, iip, "unit"))
    worst = max(abs(perm.element_rule_channel(pe, qe, *e, keys, Cab, 160, 160, weights="energy") - x)
                for e, x in zip(els, exact))
    assert worst > 2e-2 * vmax, (mistake, worst, vmax)


def test_energy_p0_is_symmetric_and_bounded():
    pe, qe = lattice.tangent_edges(10), lattice.tangent_edges(10)
    keys = [(0, 0, 0, 0, 0)]
    A = P0Lattice(pe, qe, keys, weights="energy").full(np.ones((1, 1, 1)))
    D = A.toarray()
    assert np.max(np.abs(D - D.T)) <= 1e-13 * np.max(np.abs(D))
    ev = np.linalg.eigvalsh(D)
    assert ev.min() >= -1.0 - 1e-6 and ev.max() <= 2.0 + 1e-6, (ev.min(), ev.max())


# --------------------------------------------------------------------------- G1 closed forms

BOX = (0.3, 0.5, 0.2, 0.45)


def _corners(pa, pb, qa, qb):
    return H * pa * pa, H * pb * pb, 0.75 * H * qa * qa, 0.75 * H * qb * qb


@pytest.mark.parametrize("E", [-3.0, 0.5, 40.0, 120.0])
def test_continuum_closed_form_off_shell_matches_quadrature(E):
    x1, x2, y1, y2 = _corners(*BOX)
    assert not (x1 + y1 <= E <= x2 + y2)
    val, _ = integrate.dblquad(lambda y, x: 1.0 / (E - x - y), x1, x2, y1, y2, epsabs=0.0, epsrel=1e-13)
    g = resolvent.continuum_element_energy(*BOX, E)
    assert g.imag == 0.0
    assert abs(g.real - val / ((x2 - x1) * (y2 - y1))) <= 1e-12 * abs(g.real)


@pytest.mark.parametrize("frac", [0.05, 0.3, 0.5, 0.77, 0.99])
def test_continuum_closed_form_on_shell(frac):
    x1, x2, y1, y2 = _corners(*BOX)
    E = x1 + y1 + frac * ((x2 - x1) + (y2 - y1))
    g = resolvent.continuum_element_energy(*BOX, E)
    # real part: the y integral is ln|E - x - y1| - ln|E - x - y2|; the x integral by adaptive
    # quadrature with the two logarithmic points as breakpoints
    f = lambda x: np.log(abs(E - x - y1)) - np.log(abs(E - x - y2))
    pts = [p for p in (E - y1, E - y2) if x1 < p < x2]
    re, _ = integrate.quad(f, x1, x2, points=pts or None, epsabs=0.0, epsrel=1e-12, limit=400)
    assert abs(g.real - re / ((x2 - x1) * (y2 - y1))) <= 1e-10 * abs(g)
    # imaginary part: the E + i eta limit of the same antiderivative with the principal logarithm
    with mpmath.workdps(40):
        Ez = mpmath.mpf(E) + 1j * mpmath.mpf("1e-25")
        phi = lambda z: z * mpmath.log(z)
        s = phi(Ez - x1 - y1) - phi(Ez - x2 - y1) - phi(Ez - x1 - y2) + phi(Ez - x2 - y2)
        lim = complex(s / ((x2 - x1) * (y2 - y1)))
    assert abs(g.imag - lim.imag) <= 1e-12 * abs(g.imag) and g.imag < 0.0
    assert abs(g.real - lim.real) <= 1e-12 * abs(g)


def test_bound_continuum_matches_principal_value():
    qe = lattice.tangent_edges(12)
    eps0, E = -2.2246, 3.0
    row = resolvent.bound_continuum_energy(qe, E, eps0)
    b3 = 0.75 * H
    for j in range(12):
        y1, y2 = b3 * qe[j] ** 2, b3 * qe[j + 1] ** 2
        c = E - eps0
        if y1 < c < y2:
            # int dy / (c - y) = -PV int dy / (y - c)
            pv, _ = integrate.quad(lambda y: -1.0, y1, y2, weight="cauchy", wvar=c, epsabs=0.0, epsrel=1e-13)
            assert abs(row[j].imag + np.pi / (y2 - y1)) <= 1e-13 * np.pi / (y2 - y1)
        else:
            pv, _ = integrate.quad(lambda y: 1.0 / (c - y), y1, y2, epsabs=0.0, epsrel=1e-13)
            assert row[j].imag == 0.0
        assert abs(row[j].real - pv / (y2 - y1)) <= 1e-11 * abs(row[j]), (j, row[j], pv / (y2 - y1))


# --------------------------------------------------------------------------- two-body

def test_energy_h0_and_potentials_match_their_integrals():
    pe = lattice.tangent_edges(8)
    C = H * (pe[1:] ** 2 - pe[:-1] ** 2)
    # h0: (1/C_i) int |w|^2 H p^2 dp with |w|^2 = 2 H p
    for i in range(8):
        v, _ = integrate.quad(lambda p: 2.0 * H * p * H * p * p, pe[i], pe[i + 1])
        assert abs(lattice.h0_diagonal_energy(pe)[i] - v / C[i]) <= 1e-13 * abs(v / C[i])
    # Yamaguchi form factor: C_i^(-1/2) int w(p) p g(p) dp
    beta = 1.394
    Gy = potential.yamaguchi_form_energy(pe, beta)
    for i in range(8):
        v, _ = integrate.quad(lambda p: np.sqrt(2.0 * H * p) * p / (p * p + beta * beta), pe[i], pe[i + 1],
                              epsabs=0.0, epsrel=1e-12)
        assert abs(Gy[i] - v / np.sqrt(C[i])) <= 1e-11 * abs(Gy[i])
    # Yukawa (l = 0 and 2): off-diagonal bin pairs have smooth integrands and agree tightly with a
    # nested adaptive quadrature; diagonal ones carry the log singularity at p = p' and agree to
    # the Gauss rule's accuracy there
    mu = 1.55
    for l in (0, 2):
        Y = potential.yukawa_wp_energy(pe, l, mu)
        for (i, k, tol) in ((2, 5, 1e-10), (0, 7, 1e-10), (3, 3, 2e-4), (6, 6, 2e-4)):
            def inner(pp, p):
                z = (p * p + pp * pp + mu * mu) / (2.0 * p * pp)
                return np.sqrt(2 * H * p) * np.sqrt(2 * H * pp) * potential.legendre_q(l, np.array([z]))[0] / np.pi
            pts = None
            if i == k:
                v = 0.0
                for (a, b) in ((pe[i], pe[i + 1]),):
                    v, _ = integrate.quad(lambda p: integrate.quad(lambda pp: inner(pp, p), a, b, points=[p],
                                                                  limit=200, epsrel=1e-10)[0],
                                          a, b, limit=200, epsrel=1e-10)
            else:
                v, _ = integrate.dblquad(inner, pe[i], pe[i + 1], pe[k], pe[k + 1], epsabs=0.0, epsrel=1e-12)
            ref = v / np.sqrt(C[i] * C[k])
            assert abs(Y[i, k] - ref) <= tol * abs(ref), (l, i, k, Y[i, k], ref)


@pytest.mark.parametrize("pot", ["yamaguchi", "mt"])
def test_energy_weight_s_matrix_is_unitary_below_breakup(pot):
    spec = pipeline.Spec(M=12, N=12, two_J=3 if pot == "yamaguchi" else 1, pot=pot, weights="energy")
    s = pipeline.build_system(spec)
    for E in (1.0, 2.0, 3.0):
        r = pipeline.solve_energy(s, E, direct=True)
        S = r["S"]
        assert np.max(np.abs(S.conj().T @ S - np.eye(S.shape[0]))) <= 1e-12, (pot, E)
