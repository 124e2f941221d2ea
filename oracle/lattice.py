"""Free wave-packet lattice and nd kinematics. Oracle: test-only.

Paper: Sec. II.B.1 (eq. pq: WPs as integrals of plane waves over bins; the lattice cells
D_ij = D_i x D_j) and the Appendix (projection of plane waves onto unit-weight WPs:
<p, q | p_i q_j> = theta(p in D_i) theta(q in D_j) / (p q sqrt(d_i d_j))).

Units: momenta in fm^-1, energies in MeV, hbar^2/m = H2M MeV fm^2 (the paper keeps hbar = 1
and a nucleon mass m without numbers). The two-body kinetic energy is H2M p^2, the
third-nucleon one (3/4) H2M q^2.
"""
from __future__ import annotations

import numpy as np

H2M = 41.471  # hbar^2 / m_N  [MeV fm^2]


def tangent_edges(n: int, alpha: float = 1.0, p_max: float = 10.0) -> np.ndarray:
    """Edges p_0 = 0 < p_1 < ... < p_n = p_max, p_i = alpha tan(i theta_max / n).

    The paper leaves the partition free; this tangent map (dense near 0, sparse near p_max) is
    the lattice used throughout.
    """
    th = np.arctan(p_max / alpha)
    e = alpha * np.tan(np.arange(n + 1) * th / n)
    e[0] = 0.0
    e[-1] = p_max
    return e


def widths(edges: np.ndarray) -> np.ndarray:
    return np.diff(edges)


def h0_diagonal(edges: np.ndarray, h2m: float = H2M) -> np.ndarray:
    """<p_i | H2M p^2 | p_i> for unit-weight packets: (H2M / d_i) int_{D_i} p^2 dp."""
    a, b = edges[:-1], edges[1:]
    return h2m * (b ** 3 - a ** 3) / (3.0 * (b - a))


# ---- energy weights (Sec. III.B, the footnote to eqs. dg1a, dg1b) ----
#
# A packet with weight w(p) ~ sqrt(p) is |p_i> = C_i^(-1/2) int_{D_i} w(p) |p> dp with
# |w(p)|^2 = d eps / dp: the weight is flat in the energy eps = H2M p^2, and C_i is the energy
# width H2M (p_i^2 - p_{i-1}^2). For the third nucleon, |f(q)|^2 = d eps_q / dq with
# eps_q = (3/4) H2M q^2 and B_j = (3/4) H2M (q_j^2 - q_{j-1}^2).

def energy_widths(edges: np.ndarray, scale: float) -> np.ndarray:
    """scale * (p_i^2 - p_{i-1}^2): C_i with scale = H2M, B_j with scale = (3/4) H2M."""
    return scale * (edges[1:] ** 2 - edges[:-1] ** 2)


def h0_diagonal_energy(edges: np.ndarray, h2m: float = H2M) -> np.ndarray:
    """<p_i | H2M p^2 | p_i> for energy-weight packets: (1/C_i) int eps d eps, the bin's mean energy."""
    a, b = edges[:-1], edges[1:]
    return 0.5 * h2m * (a * a + b * b)


# ---- kinematics (nd elastic: deuteron at rest, neutron with lab energy E_lab) ----

def e_cm(E_lab: float) -> float:
    """Centre-of-mass energy of n + d with equal nucleon masses: (2/3) E_lab."""
    return 2.0 * E_lab / 3.0


def q_onshell(E_lab: float, h2m: float = H2M) -> float:
    """q0 with (3/4) H2M q0^2 = E_cm."""
    return np.sqrt(4.0 * e_cm(E_lab) / (3.0 * h2m))


def total_energy(E_lab: float, eps0: float) -> float:
    return eps0 + e_cm(E_lab)


def onshell_bin(q_edges: np.ndarray, q0: float) -> int:
    """Index j0 of the bin (q_{j-1}, q_j] containing q0 (half-open on the left)."""
    j = int(np.searchsorted(q_edges, q0, side="left")) - 1
    if j < 0 or j >= len(q_edges) - 1:
        raise ValueError("on-shell momentum outside the q lattice")
    return j
