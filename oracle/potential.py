"""NN potentials in the free WP basis (the v1 of eq. Ueq). Oracle: test-only.

With unit-weight packets <p | p_i> = 1/(p sqrt(d_i)) on D_i (measure p^2 dp), a partial-wave
kernel v_l(p, p') (normalisation <p|p'> = delta(p - p')/p^2) has WP elements

    v_ii' = (d_i d_i')^(-1/2) int_{D_i} dp int_{D_i'} dp'  p p' v_l(p, p').

* Yamaguchi (separable): v(p, p') = -lam g(p) g(p'), g = 1/(p^2 + beta^2); closed form.
* Yukawa term V e^{-mu r}/r: v_l(p, p') = (V / (pi p p')) Q_l(z), z = (p^2 + p'^2 + mu^2)/(2 p p').
  The Malfliet-Tjon form is V_R Yuk(mu_R) - V_A Yuk(mu_A).

Energy-weight packets (weight w(p) = sqrt(2 H2M p), |w|^2 = d eps/dp, norm C_i = H2M (p_i^2 -
p_{i-1}^2); Sec. III.B, footnote) give

    v_ii' = (C_i C_i')^(-1/2) int int w(p) w(p') p p' v_l(p, p') dp dp'
          = 2 (dp2_i dp2_i')^(-1/2) int int sqrt(p p') p p' v_l(p, p') dp dp',

dp2_i = p_i^2 - p_{i-1}^2 (H2M cancels).
"""
from __future__ import annotations

import numpy as np
from scipy import integrate
from scipy.optimize import brentq
from scipy.special import gamma, hyp2f1

from .lattice import H2M, h0_diagonal


def yamaguchi_form(edges):
    """G_i = (1/sqrt(d_i)) int_{D_i} p/(p^2+beta^2) dp is returned as a function of beta."""
    a, b = edges[:-1], edges[1:]

    def G(beta):
        return np.log((b ** 2 + beta ** 2) / (a ** 2 + beta ** 2)) / (2.0 * np.sqrt(b - a))
    return G


def yamaguchi_wp(edges, beta, lam):
    G = yamaguchi_form(edges)(beta)
    return -lam * np.outer(G, G)


def legendre_q(l: int, z):
    """Legendre function of the second kind Q_l(z), z > 1.

    Large z: the hypergeometric series
      Q_l(z) = sqrt(pi) l! / (Gamma(l + 3/2) (2z)^(l+1)) 2F1((l+1)/2, (l+2)/2; l+3/2; 1/z^2);
    z < 2: upward recurrence from Q_0 = atanh(1/z), Q_1 = z Q_0 - 1 (stable there).
    """
    z = np.asarray(z, dtype=float)
    out = np.empty_like(z)
    small = z < 2.0
    if np.any(small):
        zs = z[small]
        q0 = 0.5 * np.log((zs + 1.0) / (zs - 1.0))
        if l == 0:
            out[small] = q0
        else:
            qm, qc = q0, zs * q0 - 1.0
            for n in range(1, l):
                qm, qc = qc, ((2 * n + 1) * zs * qc - n * qm) / (n + 1)
            out[small] = qc
    big = ~small
    if np.any(big):
        zb = z[big]
        c = np.sqrt(np.pi) * gamma(l + 1) / gamma(l + 1.5)
        out[big] = c / (2.0 * zb) ** (l + 1) * hyp2f1((l + 1) / 2.0, (l + 2) / 2.0, l + 1.5, 1.0 / zb ** 2)
    return out


def yukawa_wp(edges, l: int, mu: float, n_gauss: int = 32):
    """Unit-strength (V = 1 MeV fm) Yukawa WP matrix for orbital l by n x n Gauss per bin pair."""
    x, w = np.polynomial.legendre.leggauss(n_gauss)
    a, b = edges[:-1], edges[1:]
    h = 0.5 * (b - a)
    m = 0.5 * (b + a)
    P = (m[:, None] + h[:, None] * x[None, :])  # (M, n) nodes
    W = h[:, None] * w[None, :]
    M = len(a)
    pp = P.reshape(M, 1, -1, 1)
    pq = P.reshape(1, M, 1, -1)
    z = (pp ** 2 + pq ** 2 + mu ** 2) / (2.0 * pp * pq)
    # p p' v_l = (1/pi) Q_l(z)
    f = legendre_q(l, z.reshape(-1)).reshape(z.shape) / np.pi
    I = np.einsum("ijab,ia,jb->ij", f, W, W)
    d = b - a
    return I / np.sqrt(np.outer(d, d))


def yukawa_wp_swave_closed(edges, mu: float):
    """Closed form of the l = 0 unit Yukawa WP matrix (pin for the Gauss route).

    p p' v_0 = (1/(2 pi)) [ln((p+p')^2 + mu^2) - ln((p-p')^2 + mu^2)]; the double integral of
    ln(u^2 + mu^2) over a rectangle follows from the second antiderivative
      L2(u) = (u^2 - mu^2)/2 ln(u^2 + mu^2) - 3u^2/2 + 2 mu u atan(u/mu).
    """
    def L2(u):
        return 0.5 * (u * u - mu * mu) * np.log(u * u + mu * mu) - 1.5 * u * u + 2.0 * mu * u * np.arctan(u / mu)
    a, b = edges[:-1], edges[1:]
    A, B = a[:, None], b[:, None]
    C, D = a[None, :], b[None, :]
    plus = L2(B + D) - L2(B + C) - L2(A + D) + L2(A + C)
    minus = L2(B - C) - L2(B - D) - L2(A - C) + L2(A - D)
    d = b - a
    return (plus - minus) / (2.0 * np.pi) / np.sqrt(np.outer(d, d))


def yamaguchi_form_energy(edges, beta):
    """Energy weights: G_i = sqrt(2 / dp2_i) int_{D_i} p^(3/2) / (p^2 + beta^2) dp (adaptive quadrature)."""
    a, b = edges[:-1], edges[1:]
    out = np.empty(len(a))
    for i in range(len(a)):
        val, _ = integrate.quad(lambda p: p ** 1.5 / (p * p + beta * beta), a[i], b[i], epsabs=0.0, epsrel=1e-13,
                                limit=200)
        out[i] = val * np.sqrt(2.0 / (b[i] ** 2 - a[i] ** 2))
    return out


def yamaguchi_wp_energy(edges, beta, lam):
    G = yamaguchi_form_energy(edges, beta)
    return -lam * np.outer(G, G)


def yukawa_wp_energy(edges, l: int, mu: float, n_gauss: int = 32):
    """Unit-strength Yukawa WP matrix for energy weights: n x n Gauss per bin pair in t = sqrt(p)
    (p = t^2, dp = 2 t dt, so sqrt(p) dp = 2 t^2 dt and the integrand stays smooth at p = 0)."""
    x, w = np.polynomial.legendre.leggauss(n_gauss)
    a, b = np.sqrt(edges[:-1]), np.sqrt(edges[1:])
    h = 0.5 * (b - a)
    m = 0.5 * (b + a)
    T = m[:, None] + h[:, None] * x[None, :]
    W = h[:, None] * w[None, :] * 2.0 * T * T
    P = T * T
    M = len(a)
    pp = P.reshape(M, 1, -1, 1)
    pq = P.reshape(1, M, 1, -1)
    z = (pp ** 2 + pq ** 2 + mu ** 2) / (2.0 * pp * pq)
    f = legendre_q(l, z.reshape(-1)).reshape(z.shape) / np.pi
    I = np.einsum("ijab,ia,jb->ij", f, W, W)
    d2 = edges[1:] ** 2 - edges[:-1] ** 2
    return 2.0 * I / np.sqrt(np.outer(d2, d2))


def h0_of(edges, h2m=H2M, weights="unit"):
    from .lattice import h0_diagonal_energy
    return h0_diagonal(edges, h2m) if weights == "unit" else h0_diagonal_energy(edges, h2m)


def ground_state(edges, v, h2m=H2M, weights="unit"):
    return np.linalg.eigvalsh(np.diag(h0_of(edges, h2m, weights)) + v)[0]


def tune_yamaguchi(edges, beta, target_BE, h2m=H2M, weights="unit"):
    """lam such that the lowest eigenvalue of h0 + v equals -target_BE (bisection)."""
    G = yamaguchi_form(edges)(beta) if weights == "unit" else yamaguchi_form_energy(edges, beta)
    f = lambda lam: ground_state(edges, -lam * np.outer(G, G), h2m, weights) + target_BE
    return brentq(f, 1.0, 2000.0, xtol=1e-14, rtol=1e-15, maxiter=500)


def mt_parts(edges, l, mu_R, mu_A, weights="unit"):
    """(Yuk(mu_R), Yuk(mu_A)) unit matrices for orbital l (closed form for l = 0, unit weights)."""
    if weights == "energy":
        return yukawa_wp_energy(edges, l, mu_R), yukawa_wp_energy(edges, l, mu_A)
    if l == 0:
        return yukawa_wp_swave_closed(edges, mu_R), yukawa_wp_swave_closed(edges, mu_A)
    return yukawa_wp(edges, l, mu_R), yukawa_wp(edges, l, mu_A)


def tune_mt(edges, V_R, mu_R, mu_A, target_BE, h2m=H2M, weights="unit"):
    """V_A such that the 3S1 (l = 0) lowest eigenvalue equals -target_BE."""
    YR, YA = mt_parts(edges, 0, mu_R, mu_A, weights)
    f = lambda VA: ground_state(edges, V_R * YR - VA * YA, h2m, weights) + target_BE
    return brentq(f, 10.0, 5000.0, xtol=1e-13, rtol=1e-15, maxiter=500)
