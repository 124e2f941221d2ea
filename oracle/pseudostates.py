"""Two-body pseudostates: h1 = h0 + v1 diagonalised in the free WP basis (eq. exp_z).

Oracle: test-only.

  * eigenpairs of diag(e) + v (numpy.linalg.eigh), ascending energies eps_k;
  * O has the eigenvectors as ROWS: |z_k> ~ sum_i O_ki |p_i>;
  * negative energies are bound states; continuum pseudostates carry the momenta
    p*_k = sqrt(eps_k / H2M).

Scattering-WP bins Delta_k (the paper never states how they are built): momentum bins with
edges p^_0 = 0, p^_k = (p*_k + p*_{k+1})/2 between neighbours and p^_K = 2 p*_K - p^_{K-1} at
the top, widths d*_k. The amplitude is independent of the partition as the basis grows
(Sec. III.B, after eq. dg1b).
"""
from __future__ import annotations

import numpy as np

from .lattice import H2M, h0_diagonal


def diagonalize(edges, v, h2m=H2M, h0=None):
    """Eigenpairs of h1 = h0 + v1. Each eigenvector is fixed up to its sign by the eigensolver;
    the convention here makes its component of largest magnitude positive, so that projections
    onto single pseudostates (the breakup elements) are defined. h0: the free diagonal (default:
    unit-weight packets)."""
    if h0 is None:
        h0 = h0_diagonal(edges, h2m)
    eps, vec = np.linalg.eigh(np.diag(h0) + v)
    O = vec.T.copy()
    for k in range(O.shape[0]):
        if O[k, np.argmax(np.abs(O[k]))] < 0.0:
            O[k] = -O[k]
    return eps, O


def scattering_bins(eps_cont, h2m=H2M):
    """Edges of the momentum bins around the continuum pseudostates (ascending eps > 0)."""
    if np.any(eps_cont <= 0):
        raise ValueError("continuum pseudostate with non-positive energy")
    ps = np.sqrt(eps_cont / h2m)
    K = len(ps)
    e = np.empty(K + 1)
    e[0] = 0.0
    e[1:K] = 0.5 * (ps[:-1] + ps[1:])
    e[K] = 2.0 * ps[-1] - e[K - 1]
    return e


def scattering_bins_energy(eps_cont, h2m=H2M):
    """Energy-weight reading of the scattering-WP bins: the bins are energy intervals with edges
    e_0 = 0, e_k = (eps_k + eps_{k+1})/2 between neighbours and e_K = 2 eps_K - e_{K-1} at the
    top (the weight is flat in energy, so the bins are cut there). Returned as the momentum edges
    sqrt(e / H2M), the form the unit-weight bins take."""
    if np.any(eps_cont <= 0):
        raise ValueError("continuum pseudostate with non-positive energy")
    K = len(eps_cont)
    e = np.empty(K + 1)
    e[0] = 0.0
    e[1:K] = 0.5 * (eps_cont[:-1] + eps_cont[1:])
    e[K] = 2.0 * eps_cont[-1] - e[K - 1]
    return np.sqrt(e / h2m)
