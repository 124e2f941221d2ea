"""Shared checks of the FP64 solve against the oracle (used by the GPU parity tests).

Series terms: a_n = e^T O K^n b is the n-th application of the kernel K. Both sides build K from
their own FP64 two-body eigensolutions, whose eigenvectors agree only to rounding over the level
spacing (1e-12 relative on the 20 x 20 doublet lattice, more with 150 pseudostates per wave), and
a relative difference delta of K moves K^n b by about n delta (measured: the mismatch grows
linearly in n, ~2e-12 per term). The tolerance is the FP64 target 1e-10 for the first ten
applications and grows linearly after them:

    |a_n[f] - a_n^ref[f]| <= 1e-10 max(1, (n + 1) / 10) max_{m <= n, f'} |a_m^ref[f']|,

relative to the largest term of the column so far (single terms of an oscillating series can
pass through zero, and a final channel's first terms can vanish).

Amplitudes: the Neumann series of the nd kernel converges below some energies and diverges
above others (its terms then grow by 1e12 to 1e22 over the 50 to 80 terms Pade needs). Pade
summation of a convergent series is well conditioned: both sides' amplitudes agree to 1e-10
relative. Summing a divergent series, the Wynn table amplifies term perturbations of ~1e-11 and
its own rounding: the oracle's Pade value differs from the exact solution of the same discrete
system (dense LU) by up to 1.2e-9 relative on the 20 x 20 doublet lattice (64 energies, measured)
while its error estimate says 3e-10 or less. For divergent series the amplitude is therefore held
to 1e-8 relative against the dense LU solution (small lattices) or the oracle's amplitude.
"""
import numpy as np

SERIES_TOL = 1e-10
CONVERGENT_TOL = 1e-10
DIVERGENT_TOL = 1e-8


def series_mismatch(got, ref, grow=True):
    """Largest |a_n[f] - a_n^ref[f]| / (max(1, (n + 1) / 10) max_{m <= n, f'} |a_m^ref[f']|) over the
    common terms; to be compared with SERIES_TOL. grow=False drops the factor that grows with n
    (two library solves built from the same pseudostates)."""
    n = min(len(got), len(ref))
    assert n >= 8, (len(got), len(ref))
    scale = np.maximum.accumulate(np.max(np.abs(ref[:n]), axis=1))
    if grow:
        scale *= np.maximum(1.0, (np.arange(n) + 1) / 10.0)
    return float(np.max(np.abs(got[:n] - ref[:n]) / scale[:, None]))


def divergent(terms):
    """True if the series terms grow (the last term is larger than the first)."""
    return float(np.max(np.abs(terms[-1]))) > float(np.max(np.abs(terms[0])))


def amplitude_tolerance(series_list):
    """Relative amplitude tolerance for an energy whose columns have these oracle series."""
    return DIVERGENT_TOL if any(divergent(t) for t in series_list) else CONVERGENT_TOL
