"""On-shell elastic nd amplitude in the WP representation (Sec. II.B.4). Oracle: test-only.

A_el = (2m / (3 q0)) <Z_{0 j0} | U | Z_{0 j0}> / dq_{j0}, with m -> 1/H2M in MeV fm units
(hbar = 1). S = 1 - 2 pi i A (reading: this sign and factor make S exactly unitary below
breakup for the discrete system, since there G1 has a single imaginary entry
-i pi / (2 b3 q0 dq_j0)); delta = arg(S)/2, eta = |S| for one open channel.
"""
from __future__ import annotations

import numpy as np


def amplitude_matrix(U, q0, dq0, h2m):
    return (2.0 / (3.0 * h2m * q0)) * np.asarray(U) / dq0


def amplitude_matrix_energy(U, B0):
    """Energy-weight packets: A = U / B_j0 with B_j0 the energy width of the on-shell q bin. The
    on-shell factor |f(q0)|^2 / B_j0 replaces 1/dq_j0 and |f(q0)|^2 = (3/2) H2M q0 cancels the
    prefactor 2 / (3 H2M q0); G1 has the single imaginary entry -i pi / B_j0 below breakup, so the
    same S = 1 - 2 pi i A is exactly unitary there."""
    return np.asarray(U) / B0


def s_matrix(A):
    A = np.atleast_2d(A)
    return np.eye(A.shape[0]) - 2j * np.pi * A


def phase_deg(S):
    """Half the argument of each diagonal S element, degrees."""
    return np.degrees(0.5 * np.angle(np.diag(np.atleast_2d(S))))


def inelasticity(S):
    return np.abs(np.diag(np.atleast_2d(S)))
