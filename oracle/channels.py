"""Three-body channel enumeration in jj coupling (Sec. II.B.1, eq. qnum). Oracle: test-only.

A channel is gamma = (l, s, j, lam, 2I, t) for fixed Gamma = (J, pi, T = 1/2):
  * NN pair: orbital l, spin s, total j = l + s, isospin t with l + s + t odd (pair
    antisymmetry);
  * third nucleon: orbital lam, I = lam + 1/2;
  * J = j + I, parity pi = (-1)^(l + lam), total isospin T = 1/2.
Canonical order: sorted by (j, l, s, lam, 2I).
"""
from __future__ import annotations


def pair_isospin(l: int, s: int) -> int:
    """t such that l + s + t is odd."""
    return (l + s + 1) % 2


def enumerate_channels(two_J: int, parity: int, j_max: int, l_max: int | None = None):
    """All (l, s, j, lam, two_I, t) with J = two_J/2, (-1)^(l+lam) = parity, j <= j_max."""
    out = []
    for j in range(0, j_max + 1):
        for s in (0, 1):
            for l in range(abs(j - s), j + s + 1):
                if l_max is not None and l > l_max:
                    continue
                t = pair_isospin(l, s)
                # I = lam +- 1/2 with |j - I| <= J <= j + I
                for two_I in range(1, 2 * j + two_J + 2, 2):
                    if not (abs(2 * j - two_I) <= two_J <= 2 * j + two_I):
                        continue
                    for lam in ((two_I - 1) // 2, (two_I + 1) // 2):
                        if (-1) ** (l + lam) != parity:
                            continue
                        out.append((l, s, j, lam, two_I, t))
    out = sorted(set(out), key=lambda c: (c[2], c[0], c[1], c[3], c[4]))
    return out


def swave_quartet():
    """J = 3/2+, s-wave: the single channel 3S1 (x) (lam = 0, I = 1/2)."""
    return [c for c in enumerate_channels(3, +1, 1) if c[0] == 0 and c[3] == 0]


def swave_doublet():
    """J = 1/2+, s-wave: 1S0 and 3S1, both with (lam = 0, I = 1/2)."""
    return [c for c in enumerate_channels(1, +1, 1) if c[0] == 0 and c[3] == 0]
