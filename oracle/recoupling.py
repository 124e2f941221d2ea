"""Spin-isospin-angular coefficients of the permutation kernel (Appendix, eqs. ggaga and gal).

Oracle: test-only. Exact Wigner symbols from SymPy, converted to float at the end.

The kernel of P = P12 P23 + P13 P23 between partial-wave states is (Appendix, eq. P_kern)

    <p q gamma | P | p' q' gamma'> = int dx delta(p' - pi1) delta(p - pi2) / (p'^(l'+2) p^(l+2))
                                      * G_{gamma gamma'}(q, q', x),

    pi1 = |q + q'/2|,  pi2 = |q/2 + q'|,

with G a sum of terms q^a q'^b P_k(x) g^{l1 l1' k}_{gamma gamma'} (eq. ggaga), l1 + l2 = l,
l1' + l2' = l'. This module evaluates g exactly as printed in eq. gal.

Reading of the exponents (the paper's eq. ggaga and the final Appendix formula attach
q^(l2+l2') q'^(l1+l1'), while eq. gal couples l1 and l1' with the orbital momentum lam of q):
the exponent pair is returned by ``exponents()`` and the choice is fixed by the m-scheme pin in
``mscheme`` (tests/test_oracle_recoupling.py), not by assumption.
"""
from __future__ import annotations

from functools import lru_cache
from math import factorial, sqrt

from sympy import Rational, S as _S
from sympy.physics.wigner import clebsch_gordan, wigner_6j, wigner_9j

HALF = Rational(1, 2)


def _hat(x) -> float:
    return float(2 * x + 1)


@lru_cache(maxsize=None)
def _w6(a, b, c, d, e, f) -> float:
    return float(wigner_6j(a, b, c, d, e, f))


@lru_cache(maxsize=None)
def _w9(a, b, c, d, e, f, g, h, i) -> float:
    return float(wigner_9j(a, b, c, d, e, f, g, h, i, prec=None))


@lru_cache(maxsize=None)
def _cg0(a, b, c) -> float:
    """<a 0 b 0 | c 0>."""
    return float(clebsch_gordan(a, b, c, 0, 0, 0))


def _tri(a, b, c) -> bool:
    return abs(a - b) <= c <= a + b


def g_table(ch, chp, two_J: int, two_T: int = 1):
    """Dict {(l1, l1p, k): g} for channels ch = (l, s, j, lam, 2I, t) and chp (primed), eq. gal.

    Zero entries are dropped. J = two_J / 2, T = two_T / 2.
    """
    l, s, j, lam, two_I, t = ch
    lp, sp, jp, lamp, two_Ip, tp = chp
    I = Rational(two_I, 2)
    Ip = Rational(two_Ip, 2)
    J = Rational(two_J, 2)
    T = Rational(two_T, 2)
    pref = -sqrt(_hat(l) * _hat(s) * _hat(j) * _hat(t) * _hat(lam) * _hat(I)
                 * _hat(lp) * _hat(sp) * _hat(jp) * _hat(tp) * _hat(lamp) * _hat(Ip))
    pref *= _w6(HALF, HALF, tp, HALF, T, t)
    if pref == 0.0:
        return {}
    out = {}
    for L in range(0, max(l + lam, lp + lamp) + 1):
        if not (_tri(l, lam, L) and _tri(lp, lamp, L)):
            continue
        for two_S in (1, 3):
            Sv = Rational(two_S, 2)
            a = _hat(L) * _hat(Sv) * _w6(HALF, HALF, sp, HALF, Sv, s)
            if a == 0.0:
                continue
            a *= _w9(l, s, j, lam, HALF, I, L, Sv, J) * _w9(lp, sp, jp, lamp, HALF, Ip, L, Sv, J)
            if a == 0.0:
                continue
            for l1 in range(0, l + 1):
                l2 = l - l1
                for l1p in range(0, lp + 1):
                    l2p = lp - l1p
                    c = (0.5 ** (l2p + l1)
                         * sqrt(factorial(2 * l + 1) / (factorial(2 * l1) * factorial(2 * l2)))
                         * sqrt(factorial(2 * lp + 1) / (factorial(2 * l1p) * factorial(2 * l2p))))
                    kmax = l1p + l2 + lam + lamp + L + 2
                    for k in range(0, kmax + 1):
                        acc = 0.0
                        for f in range(abs(l1 - lam), l1 + lam + 1):
                            cf = _cg0(l1, lam, f)
                            if cf == 0.0:
                                continue
                            if not _tri(k, l1p, f):
                                continue
                            ck = _cg0(k, l1p, f)
                            if ck == 0.0:
                                continue
                            w6b = _w6(l2, l1, l, lam, L, f)
                            if w6b == 0.0:
                                continue
                            for fp in range(abs(l2p - lamp), l2p + lamp + 1):
                                cfp = _cg0(l2p, lamp, fp)
                                if cfp == 0.0:
                                    continue
                                if not _tri(k, l2, fp):
                                    continue
                                ck2 = _cg0(k, l2, fp)
                                if ck2 == 0.0:
                                    continue
                                acc += (_w6(l1p, l2p, lp, lamp, L, fp) * w6b * cfp * cf
                                        * _w6(fp, l1p, L, f, l2, k) * ck * ck2)
                        if acc != 0.0:
                            key = (l1, l1p, k)
                            out[key] = out.get(key, 0.0) + pref * a * _hat(k) * c * acc
    return {key: v for key, v in out.items() if abs(v) > 1e-15}


def exponents(ch, chp, l1: int, l1p: int):
    """(a, b): powers of q and q' multiplying g^{l1 l1' k} in G (reading pinned by mscheme).

    The m-scheme pin shows that the orbital momenta l1, l1' (those coupled with lam in eq. gal
    and carrying the factor 1/2 from p = |q/2 + q'| and p' = |q + q'/2|) go with q, so
    a = l1 + l1' and b = l2 + l2'.
    """
    l, lp = ch[0], chp[0]
    return l1 + l1p, (l - l1) + (lp - l1p)


def G_from_table(table, ch, chp, q, qp, x):
    """G_{gamma gamma'}(q, q', x) = sum q^a q'^b P_k(x) g (eq. ggaga with the pinned exponents)."""
    from numpy.polynomial import legendre as _leg
    tot = 0.0
    for (l1, l1p, k), gv in table.items():
        a, b = exponents(ch, chp, l1, l1p)
        coef = [0.0] * k + [1.0]
        tot += gv * q ** a * qp ** b * _leg.legval(x, coef)
    return tot
