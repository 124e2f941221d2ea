"""Many J^pi blocks solved on one lattice size and summed into elastic nd observables (Sec. IV).

Every block (J, pi) is its own lattice (channels of that J^pi, its own P0) solved at the same
energies; the elastic S matrices of all blocks at one energy go to nd_elastic_observables (host
C++). This module only orders the calls: each build and solve runs in the library's kernels.
"""
from __future__ import annotations

import numpy as np

from . import H2M, Lattice, nd_elastic_observables, open_channels


class JBlocks:
    """Lattices for the blocks blocks = [(two_J, parity)], all M x N bins, pair waves j <= j_max."""

    def __init__(self, blocks, M, N, j_max=1, n_x=8, n_phi=8, precision="fp64", weights="unit", **pot):
        self.lats = []
        for two_J, parity in blocks:
            L = Lattice(M, N, two_J=two_J, parity=parity, j_max=j_max, swave_only=False, n_x=n_x, n_phi=n_phi,
                        weights=weights)
            L.pseudostates(**pot)
            L.build_perm(precision)
            self.lats.append(((two_J, parity), L))

    def solve(self, E_lab, mode="fp64", hbar2_over_m=H2M, **kw):
        """S matrices per energy: out[e] = [(two_J, chans, S)], plus the nd relative momenta q0[e]
        ((3/4) (hbar^2/m) q0^2 = E_cm = (2/3) E_lab, the on-shell momentum of the solves)."""
        Es = list(E_lab)
        per_E = [[] for _ in Es]
        for (two_J, _), L in self.lats:
            sol = L.solve(Es, mode, **kw)
            chans = open_channels(L.channels)
            for e in range(len(Es)):
                per_E[e].append((two_J, chans, sol.amplitude(e)["S"]))
        q0 = [float(np.sqrt(8.0 * E / (9.0 * hbar2_over_m))) for E in Es]
        return per_E, q0

    @staticmethod
    def observables(blocks, k, thetas):
        return nd_elastic_observables(blocks, k, thetas)
