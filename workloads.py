"""Seeded synthetic workloads shared by the tests, the bench and the oracle-based checks.

This module only holds sizes, physical constants of the synthetic inputs and seeded random
draws. It contains none of the method's arithmetic, so both the product path and the oracle
may read it.

Workloads (stand-ins for the paper's MT I-III s-wave runs and its 18-channel J = 1/2+ run;
the paper's Nijmegen potential and data are not available):

* ``quartet_yamaguchi_40``: s-wave spin-quartet nd (one channel, J = 3/2+), separable
  Yamaguchi potential beta = 1.394 fm^-1 with the strength tuned to a 2.2246 MeV deuteron,
  M = N = 40 tangent-mapped bins up to 10 fm^-1, 8 x 8 (x, phi) Gauss nodes per cell pair,
  E_lab = 10 MeV.
* ``swave_mt_100``: s-wave doublet (1S0 + 3S1, J = 1/2+) and quartet (J = 3/2+) with the
  Malfliet-Tjon form V_R e^{-mu_R r}/r - V_A e^{-mu_A r}/r, mu_R = 3.11, mu_A = 1.55 fm^-1,
  V_R drawn from U[1200, 1600] MeV fm (seed 0), V_A tuned to the deuteron, singlet strength
  0.82 V_A, M = N = 100, E_lab = 14.1 MeV.
* ``pw_mt_150``: the same potential in all partial waves with j <= 2 (18 channels for
  J = 1/2+), M = N = 150, E_lab = 3 and 22.7 MeV.
* ``batched_energies``: 64 lab energies U[1, 50] MeV (seed 1234) on the doublet lattice.
* ``serving``: Poisson arrivals (200 requests/s, seed 2026) over several resident lattices.
"""
from __future__ import annotations

import numpy as np

HBAR2_OVER_M = 41.471      # MeV fm^2
DEUTERON_BE = 2.2246       # MeV
ALPHA = 1.0                # fm^-1, tangent-map scale
P_MAX = 10.0               # fm^-1
Q_MAX = 10.0               # fm^-1
YAMAGUCHI_BETA = 1.394     # fm^-1
MT_MU_R = 3.11             # fm^-1
MT_MU_A = 1.55             # fm^-1
SINGLET_RATIO = 0.82


def mt_repulsion(seed: int) -> float:
    """V_R in MeV fm drawn uniformly from [1200, 1600]."""
    return float(np.random.default_rng(seed).uniform(1200.0, 1600.0))


def batched_energies(n: int = 64, seed: int = 1234, lo: float = 1.0, hi: float = 50.0):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def poisson_arrivals(rate: float, duration: float, seed: int = 2026):
    """Arrival times (s) of a Poisson stream with the given mean rate."""
    rng = np.random.default_rng(seed)
    t, out = 0.0, []
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            return np.array(out)
        out.append(t)


def serving_requests(n_lattices: int, rate: float = 200.0, duration: float = 2.0, seed: int = 2026):
    """(arrival time, lattice index, E_lab) triples of a Poisson request stream."""
    arr = poisson_arrivals(rate, duration, seed)
    rng = np.random.default_rng(seed + 1)
    lat = rng.integers(0, n_lattices, len(arr))
    E = rng.uniform(1.0, 50.0, len(arr))
    return list(zip(arr.tolist(), lat.tolist(), E.tolist()))


# name -> dict of lattice / potential parameters (two_J: 1 = doublet J=1/2, 3 = quartet J=3/2)
WORKLOADS = {
    "quartet_yamaguchi_40": dict(M=40, N=40, pot="yamaguchi", systems=[dict(two_J=3, j_max=1, swave=True)],
                                 E_lab=[10.0], n_x=8, n_phi=8),
    "swave_mt_100": dict(M=100, N=100, pot="mt", V_R_seed=0,
                         systems=[dict(two_J=1, j_max=1, swave=True), dict(two_J=3, j_max=1, swave=True)],
                         E_lab=[14.1], n_x=8, n_phi=8),
    "pw_mt_150": dict(M=150, N=150, pot="mt", V_R_seed=0, systems=[dict(two_J=1, j_max=2, swave=False)],
                      E_lab=[3.0, 22.7], n_x=8, n_phi=8),
}
