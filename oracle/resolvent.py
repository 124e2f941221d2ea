"""Diagonal channel resolvent G1(E) in the three-body SWP basis (Sec. III.B, eqs. dg1, dg1a, dg1b).

Oracle: test-only. Unit momentum weights (the same weights as the P0 Appendix and the
amplitude formula; the paper's closed formulas quoted in a footnote are for energy weights):

  bound-continuum  G_0j = (1/dq_j) int_{Dq_j} dq / (E + i0 - eps0 - b3 q^2),
  continuum        G_kj = (1/(d*_k dq_j)) int_{Delta_k} dp int_{Dq_j} dq / (E + i0 - h p^2 - b3 q^2),

h = H2M, b3 = (3/4) H2M.

G_0j: with E - eps0 = b3 q0^2 the q integral is elementary,
  PV -> (1/(2 b3 q0)) [ln|(q0 + q)/(q0 - q)|],  imaginary part -i pi / (2 b3 q0) if q0 in bin j.
G_kj: the p integral is done in closed form for fixed q (log or arctangent), the q integral by
adaptive quadrature with breakpoints at the singular points; for E > 0 the imaginary part is
-(pi / (d*_k dq_j)) (1 / (2 sqrt(h b3))) times the polar angle of the energy ellipse inside the
rectangle (p = sqrt(E/h) cos t, q = sqrt(E/b3) sin t).
Where the energy shell crosses the box or passes within one bin width of it, the q integrand
has endpoint singularities (an inverse square root where E - b3 q^2 changes sign, logarithms
where the pole of the p integrand meets a p-bin edge) that limit double-precision adaptive
quadrature to about 1e-10; those elements are integrated in 30-digit arithmetic (mpmath
tanh-sinh, the same formula and breakpoints). Every other element has a smooth integrand and
is done in double precision.
"""
from __future__ import annotations

import mpmath
import numpy as np
from scipy import integrate

from .lattice import H2M


def bound_continuum(q_edges, E, eps0, h2m=H2M):
    b3 = 0.75 * h2m
    q0 = np.sqrt((E - eps0) / b3)
    qa, qb = q_edges[:-1], q_edges[1:]
    f = lambda q: np.log(np.abs((q0 + q) / (q0 - q)))
    re = (f(qb) - f(qa)) / (2.0 * b3 * q0)
    im = np.where((q0 > qa) & (q0 <= qb), -np.pi / (2.0 * b3 * q0), 0.0)
    d = qb - qa
    return (re + 1j * im) / d


def _inner_p(q, pa, pb, E, h, b3):
    """PV int_{pa}^{pb} dp / (E - b3 q^2 - h p^2)."""
    c2 = E - b3 * q * q
    sh = np.sqrt(h)
    if c2 > 0.0:
        c = np.sqrt(c2)
        g = lambda p: np.log(abs((c + sh * p) / (c - sh * p))) if p != c / sh else np.inf
        return (g(pb) - g(pa)) / (2.0 * c * sh)
    if c2 < 0.0:
        k = np.sqrt(-c2)
        return -(np.arctan(sh * pb / k) - np.arctan(sh * pa / k)) / (sh * k)
    return 1.0 / (h * pb) - (1.0 / (h * pa) if pa > 0 else np.inf)


def _arc_inside(pa, pb, qa, qb, E, h, b3):
    """Polar angle t in [0, pi/2] with (sqrt(E/h) cos t, sqrt(E/b3) sin t) inside the box."""
    if E <= 0.0:
        return 0.0
    P, Q = np.sqrt(E / h), np.sqrt(E / b3)
    # p in [pa, pb] <=> cos t in [pa/P, pb/P]; q in [qa, qb] <=> sin t in [qa/Q, qb/Q]
    lo_p = np.arccos(min(1.0, pb / P))
    hi_p = np.arccos(min(1.0, pa / P))
    lo_q = np.arcsin(min(1.0, qa / Q))
    hi_q = np.arcsin(min(1.0, qb / Q))
    return max(0.0, min(hi_p, hi_q) - max(lo_p, lo_q))


def _inner_p_mp(q, pa, pb, E, h, b3):
    """_inner_p in mpmath arithmetic."""
    c2 = E - b3 * q * q
    sh = mpmath.sqrt(h)
    if c2 > 0:
        c = mpmath.sqrt(c2)
        g = lambda p: mpmath.log(abs((c + sh * p) / (c - sh * p)))
        return (g(pb) - g(pa)) / (2 * c * sh)
    if c2 < 0:
        k = mpmath.sqrt(-c2)
        return -(mpmath.atan(sh * pb / k) - mpmath.atan(sh * pa / k)) / (sh * k)
    return 1 / (h * pb) - 1 / (h * pa)


def _near_shell(pa, pb, qa, qb, E, h, b3):
    """True if the q set where the p bin holds the pole (h pa^2 <= E - b3 q^2 <= h pb^2) lies within
    one bin width of [qa, qb]."""
    hi2 = (E - h * pa * pa) / b3
    if E <= 0.0 or hi2 <= 0.0:
        return False
    lo = np.sqrt(max((E - h * pb * pb) / b3, 0.0))
    w = qb - qa
    return lo <= qb + w and np.sqrt(hi2) >= qa - w


def _real_part_mp(pa, pb, qa, qb, E, h2m):
    mp = mpmath.mpf
    with mpmath.workdps(30):
        h = mp(h2m)
        b3 = mp(3) / 4 * h
        pa_, pb_, qa_, qb_, E_ = mp(pa), mp(pb), mp(qa), mp(qb), mp(E)
        pts = [qa_, qb_]
        for c2 in (E_, E_ - h * pa_ * pa_, E_ - h * pb_ * pb_):
            if c2 > 0:
                qs = mpmath.sqrt(c2 / b3)
                if qa_ < qs < qb_:
                    pts.append(qs)
        re = mpmath.quad(lambda q: _inner_p_mp(q, pa_, pb_, E_, h, b3), sorted(set(pts)))
        return float(re)


def continuum_element(pa, pb, qa, qb, E, h2m=H2M, epsabs=1e-15, epsrel=1e-13):
    h = h2m
    b3 = 0.75 * h2m
    if _near_shell(pa, pb, qa, qb, E, h, b3):
        re = _real_part_mp(pa, pb, qa, qb, E, h2m)
        im = -np.pi / (2.0 * np.sqrt(h * b3)) * _arc_inside(pa, pb, qa, qb, E, h, b3)
        return (re + 1j * im) / ((pb - pa) * (qb - qa))
    pts = []
    for c2 in (E, E - h * pa * pa, E - h * pb * pb):
        if c2 > 0:
            qs = np.sqrt(c2 / b3)
            if qa < qs < qb:
                pts.append(qs)
    f = lambda q: _inner_p(q, pa, pb, E, h, b3)
    re, _ = integrate.quad(f, qa, qb, points=sorted(pts) or None, epsabs=epsabs, epsrel=epsrel, limit=400)
    im = -np.pi / (2.0 * np.sqrt(h * b3)) * _arc_inside(pa, pb, qa, qb, E, h, b3)
    return (re + 1j * im) / ((pb - pa) * (qb - qa))


def channel_diagonal(q_edges, E, eps_bound, cont_bins, h2m=H2M):
    """G1 over (k, j) for one pair channel: bound rows first (if any), then continuum bins.

    eps_bound: list of bound-state energies of this pair channel (the deuteron in 3S1).
    cont_bins: momentum edges of the continuum pseudostate bins.
    Returns complex array (K, N).
    """
    N = len(q_edges) - 1
    rows = []
    for eb in eps_bound:
        rows.append(bound_continuum(q_edges, E, eb, h2m))
    for k in range(len(cont_bins) - 1):
        pa, pb = cont_bins[k], cont_bins[k + 1]
        rows.append(np.array([continuum_element(pa, pb, q_edges[j], q_edges[j + 1], E, h2m)
                              for j in range(N)]))
    return np.array(rows)


# --------------------------------------------------------------------------- energy weights
#
# With the weights w(p) ~ sqrt(p), f(q) ~ sqrt(q) of the footnote in Sec. III.B (|w|^2 dp = d eps,
# |f|^2 dq = d eps_q), eqs. dg1a and dg1b are integrals over energy intervals and come out in
# closed form:
#
#   G_0j = (1/B_j) int_{y1}^{y2} dy / (E + i0 - eps_n - y) = (1/B_j) [ln(z1) - ln(z2)],
#          z_b = E - eps_n - y_b;
#   G_kj = (1/(C_k B_j)) int_{x1}^{x2} dx int_{y1}^{y2} dy / (E + i0 - x - y)
#        = (1/(C_k B_j)) [phi(z11) - phi(z21) - phi(z12) + phi(z22)],
#          z_ab = E - x_a - y_b, phi(z) = z ln(z + i0) (phi(0) = 0),
#
# with x = H2M p^2 over the pseudostate's energy bin (width C_k), y = (3/4) H2M q^2 over the q bin
# (width B_j) and ln(z + i0) = ln|z| + i pi for z < 0. The four-term difference cancels heavily
# when the bins are small next to |z|, so it is evaluated in 40-digit arithmetic here.

def _log_i0(z):
    return mpmath.log(abs(z)) + (1j * mpmath.pi if z < 0 else 0)


def _phi_re(z):
    """Real part of phi(z) = z ln(z + i0)."""
    return mpmath.mpf(0) if z == 0 else z * mpmath.log(abs(z))


def bound_continuum_energy(q_edges, E, eps0, h2m=H2M):
    out = np.empty(len(q_edges) - 1, dtype=complex)
    with mpmath.workdps(40):
        b3 = mpmath.mpf(3) / 4 * mpmath.mpf(h2m)
        for j in range(len(q_edges) - 1):
            y1 = b3 * mpmath.mpf(q_edges[j]) ** 2
            y2 = b3 * mpmath.mpf(q_edges[j + 1]) ** 2
            z1 = mpmath.mpf(E) - mpmath.mpf(eps0) - y1
            z2 = mpmath.mpf(E) - mpmath.mpf(eps0) - y2
            out[j] = complex((_log_i0(z1) - _log_i0(z2)) / (y2 - y1))
    return out


def continuum_element_energy(pa, pb, qa, qb, E, h2m=H2M):
    with mpmath.workdps(40):
        h = mpmath.mpf(h2m)
        b3 = mpmath.mpf(3) / 4 * h
        x1, x2 = h * mpmath.mpf(pa) ** 2, h * mpmath.mpf(pb) ** 2
        y1, y2 = b3 * mpmath.mpf(qa) ** 2, b3 * mpmath.mpf(qb) ** 2
        E_ = mpmath.mpf(E)
        re = (_phi_re(E_ - x1 - y1) - _phi_re(E_ - x2 - y1) - _phi_re(E_ - x1 - y2) + _phi_re(E_ - x2 - y2))
        # the imaginary parts pi z [z < 0] of the four terms add up to -pi times the length of the
        # segment x + y = E inside the box (exactly 0 off the shell)
        C, B, s0 = x2 - x1, y2 - y1, x1 + y1
        ell = max(mpmath.mpf(0), min(E_ - s0, C, B, s0 + C + B - E_))
        return complex(re / (C * B), -mpmath.pi * ell / (C * B))


def channel_diagonal_energy(q_edges, E, eps_bound, cont_bins, h2m=H2M):
    """channel_diagonal for energy-weight packets (cont_bins: momentum edges of the energy bins)."""
    N = len(q_edges) - 1
    rows = [bound_continuum_energy(q_edges, E, eb, h2m) for eb in eps_bound]
    for k in range(len(cont_bins) - 1):
        rows.append(np.array([continuum_element_energy(cont_bins[k], cont_bins[k + 1], q_edges[j], q_edges[j + 1],
                                                       E, h2m) for j in range(N)]))
    return np.array(rows)
