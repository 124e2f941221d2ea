"""Independent m-scheme evaluation of the angular-spin-isospin function G (pin for eq. gal).

Oracle: test-only. Nothing here uses 6j or 9j symbols: the channel states are built from
Clebsch-Gordan coefficients, spherical harmonics and explicit 8-dimensional spin and isospin
spaces of three nucleons, and the cyclic permutations act as explicit permutation matrices.

Conventions (Appendix, eq. P_kern):
  * set-1 Jacobi momenta: q = k1, p = k2 + k1/2 (so k2 = p - q/2, k3 = -p - q/2);
  * C = P12 P23 sends (particle 1, 2, 3) <- (k3, k1, k2) and the same for spins and isospins;
    in set-1 momenta <p q | C | p' q'> = delta(p - q/2 - q') delta(p' + q + q'/2);
  * C^-1 = P13 P23 = C^T gives delta(p + q/2 + q') delta(p' - q - q'/2);
  * P = C + C^-1.
Integrating the two deltas over the directions of p and p' leaves
delta(p - pi2)/p^2 * delta(p' - pi1)/p'^2 times an integral over q-hat, q'-hat that reduces to
8 pi^2 int dx of the M-averaged overlap at a fixed orientation. Comparing with eq. P_kern:

    G(q, q', x) = 8 pi^2 p^l p'^l' (1/(2J+1)) sum_M [Phi_gM(p-hat, q-hat)^+ C Phi_g'M(p'-hat, q'-hat)
                                                  + same for C^-1].
"""
from __future__ import annotations

from functools import lru_cache
from itertools import product

import numpy as np
from scipy.special import sph_harm_y
from sympy import Rational
from sympy.physics.wigner import clebsch_gordan

HALF = Rational(1, 2)


@lru_cache(maxsize=None)
def _cg(j1, m1, j2, m2, j3, m3) -> float:
    return float(clebsch_gordan(j1, j2, j3, m1, m2, m3))


def _idx(b1, b2, b3):
    return b1 * 4 + b2 * 2 + b3


def _m(b):  # bit -> projection
    return HALF - b


def _cyclic_matrix():
    """8x8 matrix of C on three spin-1/2 (or isospin-1/2) labels: (s1,s2,s3) -> (s3,s1,s2)."""
    c = np.zeros((8, 8))
    for b1, b2, b3 in product((0, 1), repeat=3):
        c[_idx(b3, b1, b2), _idx(b1, b2, b3)] = 1.0
    return c


def _pair_times_third(s, ms, sig1):
    """|s ms>_{23} |sig1>_1 in the 8-dim product space."""
    v = np.zeros(8)
    for b2, b3 in product((0, 1), repeat=2):
        if _m(b2) + _m(b3) != ms:
            continue
        b1 = 0 if sig1 == HALF else 1
        v[_idx(b1, b2, b3)] += _cg(HALF, _m(b2), HALF, _m(b3), s, ms)
    return v


def _iso_vec(t, two_T=1, two_MT=1):
    T = Rational(two_T, 2)
    MT = Rational(two_MT, 2)
    v = np.zeros(8)
    for mt in range(-t, t + 1):
        tau1 = MT - mt
        if abs(tau1) != HALF:
            continue
        v += _cg(t, mt, HALF, tau1, T, MT) * _pair_times_third(t, mt, tau1)
    return v


def _ylm(l, m, vec):
    r = np.linalg.norm(vec)
    th = np.arccos(np.clip(vec[2] / r, -1.0, 1.0))
    ph = np.arctan2(vec[1], vec[0])
    return complex(sph_harm_y(l, int(m), th, ph))


def _state(ch, two_J, two_M, phat, qhat):
    """Phi_{gamma M}(p-hat, q-hat) as a 64-vector (spin (x) isospin), T = M_T = 1/2."""
    l, s, j, lam, two_I, t = ch
    J = Rational(two_J, 2)
    M = Rational(two_M, 2)
    I = Rational(two_I, 2)
    spin = np.zeros(8, dtype=complex)
    for mj in range(-j, j + 1):
        mI = M - mj
        if abs(mI) > I:
            continue
        c1 = _cg(j, mj, I, mI, J, M)
        if c1 == 0.0:
            continue
        for ml in range(-l, l + 1):
            ms = mj - ml
            if abs(ms) > s:
                continue
            c2 = _cg(l, ml, s, ms, j, mj)
            if c2 == 0.0:
                continue
            yl = _ylm(l, ml, phat)
            for sig1 in (HALF, -HALF):
                mlam = mI - sig1
                if abs(mlam) > lam:
                    continue
                c3 = _cg(lam, mlam, HALF, sig1, I, mI)
                if c3 == 0.0:
                    continue
                spin += c1 * c2 * c3 * yl * _ylm(lam, mlam, qhat) * _pair_times_third(s, ms, sig1)
    return np.kron(spin, _iso_vec(t))


def G_mscheme(ch, chp, two_J, q, qp, x):
    """G_{gamma gamma'}(q, q', x) from explicit permutations (see module docstring)."""
    C8 = _cyclic_matrix()
    C = np.kron(C8, C8)
    Ci = C.T
    sth = np.sqrt(1.0 - x * x)
    qv = np.array([0.0, 0.0, q])
    qpv = qp * np.array([sth, 0.0, x])
    l, lp = ch[0], chp[0]
    tot = 0.0
    for op, pv, ppv in ((C, qv / 2 + qpv, -(qv + qpv / 2)),
                        (Ci, -(qv / 2 + qpv), qv + qpv / 2)):
        p = np.linalg.norm(pv)
        pp = np.linalg.norm(ppv)
        acc = 0.0
        for two_M in range(-two_J, two_J + 1, 2):
            bra = _state(ch, two_J, two_M, pv, qv)
            ket = _state(chp, two_J, two_M, ppv, qpv)
            acc += np.vdot(bra, op @ ket)
        tot += p ** l * pp ** lp * acc / (two_J + 1)
    val = 8.0 * np.pi ** 2 * tot
    return val.real, val.imag


def G_polynomial(ch, chp, two_J, n_x=16, check=4, seed=0):
    """G_{gamma gamma'}(q, q', x) as an exact polynomial rebuilt from m-scheme samples.

    G is homogeneous of degree L = l + l' in (q, q') (the factors p^l p'^l' turn the spherical
    harmonics of p-hat and p'-hat into solid harmonics) and a polynomial in x, so
    G = sum_{a=0..L} q^a q'^(L-a) h_a(x). The h_a are recovered from G_mscheme on L + 1 ratios
    q/q' times n_x Chebyshev nodes in x; the structure is then checked against G_mscheme itself
    at ``check`` random points (a failure raises). Nothing from eq. gal is used.

    Returns a vectorised callable G(q, q', x).
    """
    from numpy.polynomial import chebyshev as _ch
    L = ch[0] + chp[0]
    r = np.linspace(0.45, 2.2, L + 1)
    xs = np.cos(np.pi * (np.arange(n_x) + 0.5) / n_x)
    S = np.array([[G_mscheme(ch, chp, two_J, rr, 1.0, xx)[0] for xx in xs] for rr in r])
    V = np.vander(r, L + 1, increasing=True)
    H = np.linalg.solve(V, S)                      # H[a, m] = h_a(x_m)
    coef = [_ch.chebfit(xs, H[a], n_x - 1) for a in range(L + 1)]

    def G(q, qp, x):
        q, qp, x = np.broadcast_arrays(np.asarray(q, float), np.asarray(qp, float), np.asarray(x, float))
        out = np.zeros(q.shape)
        for a in range(L + 1):
            out = out + q ** a * qp ** (L - a) * _ch.chebval(x, coef[a])
        return out

    rng = np.random.default_rng(seed)
    scale = max(np.abs(S).max(), 1.0)
    for _ in range(check):
        q, qp, x = rng.uniform(0.2, 3.0), rng.uniform(0.2, 3.0), rng.uniform(-1.0, 1.0)
        ref = G_mscheme(ch, chp, two_J, q, qp, x)[0]
        got = float(G(q, qp, x))
        tol = 1e-10 * scale * max(q, qp, 1.0) ** L
        if abs(got - ref) > tol:
            raise AssertionError(f"G is not the assumed polynomial for {ch}, {chp}: {got} vs {ref}")
    return G
