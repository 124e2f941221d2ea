"""Elastic nd observables from the S matrices of several J^pi blocks (Sec. IV). Oracle: test-only.

The open channels of a block are (lam, I) with the deuteron (l = 0, s = 1, j = 1) as pair state;
a channel state couples J = j (x) I with I = lam (x) 1/2 (the order of the channel basis, eq. qnum).

* Sigma representation (Sec. IV, the transformation printed there):
    S^Sigma = T S^I T^T,  T[(lam, Sigma), (lam, I)] = sqrt((2I+1)(2Sigma+1)) (-1)^(J-I) {lam 1/2 I; j J Sigma},
  which is the overlap <(j 1/2) Sigma, lam; J | j, (lam 1/2) I; J> for the channel-spin states
  |Sigma nu, lam m; J M> = sum <Sigma nu lam m | J M> <j m_d 1/2 sigma | Sigma nu> (pinned by the
  m-scheme overlap in the tests; the other three coupling orders disagree in sign somewhere).
* Eigenphases (below breakup S is symmetric and unitary): S = O diag(exp(2 i delta)) O^T with O
  real orthogonal, found from the real symmetric matrix Re S + a Im S (a generic a), which O
  diagonalises.
* Amplitude matrix for a beam along z and the outgoing direction (theta, phi = 0), channel-spin
  basis (the partial-wave expansion of the scattering amplitude with Y*_lam,m(z) = delta_m0
  sqrt((2 lam + 1)/(4 pi))):
    M[(Sigma' nu'), (Sigma nu)] = (sqrt(pi) / (i k)) sum_{J pi, lam, lam'} sqrt(2 lam + 1)
        <Sigma nu lam 0 | J nu> <Sigma' nu' lam' nu - nu' | J nu> (S - 1)^J[(lam' Sigma'), (lam Sigma)]
        Y_lam'^(nu - nu')(theta, 0),
  k the nd relative momentum (q0). dsigma/dOmega = Tr(M M^+) / 6; the neutron analysing power
  A_y = Tr(M sigma_y M^+) / Tr(M M^+), sigma_y acting on the incoming neutron's spin, y along
  k_in x k_out.
* An independent route builds the same M in the product basis (m_d, sigma) from the jj channels
  directly (``amplitude_product_basis``), never passing through Sigma.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np
from scipy.special import sph_harm_y
from sympy import Rational
from sympy.physics.wigner import clebsch_gordan, wigner_6j

HALF = Rational(1, 2)


@lru_cache(maxsize=None)
def _cg(j1, m1, j2, m2, j3, m3) -> float:
    return float(clebsch_gordan(j1, j2, j3, m1, m2, m3))


def _R(two_x):
    return Rational(two_x, 2)


def sigma_channels(two_J, chans):
    """(lam, 2 Sigma) of the channel-spin basis spanning the same open channels: for every lam the
    Sigma in {1/2, 3/2} with |lam - Sigma| <= J <= lam + Sigma."""
    lams = sorted({c[0] for c in chans})
    out = []
    for lam in lams:
        for two_S in (1, 3):
            if abs(2 * lam - two_S) <= two_J <= 2 * lam + two_S:
                out.append((lam, two_S))
    return out


def sigma_transform(two_J, chans, j=1):
    """T over (lam, 2I) -> (lam, 2 Sigma) (the printed transformation)."""
    sig = sigma_channels(two_J, chans)
    T = np.zeros((len(sig), len(chans)))
    J = _R(two_J)
    for a, (lam, two_S) in enumerate(sig):
        for b, (lamb, two_I) in enumerate(chans):
            if lam != lamb:
                continue
            I, Sg = _R(two_I), _R(two_S)
            T[a, b] = (np.sqrt(float((2 * I + 1) * (2 * Sg + 1))) * float((-1) ** (J - I))
                       * float(wigner_6j(lam, HALF, I, j, J, Sg)))
    return sig, T


def to_sigma(two_J, chans, S):
    sig, T = sigma_transform(two_J, chans)
    return sig, T @ S @ T.T


def eigenphases(S, a=0.6180339887498949):
    """delta (radians, in (-pi/2, pi/2]) and real orthogonal O with S = O diag(exp(2 i delta)) O^T."""
    S = np.asarray(S, dtype=complex)
    w, O = np.linalg.eigh(S.real + a * S.imag)
    D = O.T @ S @ O
    return np.angle(np.diag(D)) / 2.0, O


def _ylm(l, m, theta):
    return sph_harm_y(l, m, theta, 0.0)


def amplitude_sigma(blocks, k, theta):
    """M[(Sigma' nu'), (Sigma nu)] at one angle from blocks = [(two_J, sig_channels, S_sigma)].
    Rows/columns: (2 Sigma, 2 nu) over Sigma = 1/2 (nu = -1/2, 1/2) then 3/2 (nu = -3/2 .. 3/2)."""
    states = [(1, -1), (1, 1), (3, -3), (3, -1), (3, 1), (3, 3)]
    idx = {s: n for n, s in enumerate(states)}
    M = np.zeros((6, 6), dtype=complex)
    pref = np.sqrt(np.pi) / (1j * k)
    for two_J, sig, S in blocks:
        J = _R(two_J)
        D = np.asarray(S, dtype=complex) - np.eye(len(sig))
        for b, (lam, two_S) in enumerate(sig):
            Sg = _R(two_S)
            for two_nu in range(-two_S, two_S + 1, 2):
                nu = _R(two_nu)
                c1 = _cg(Sg, nu, lam, 0, J, nu)
                if c1 == 0.0:
                    continue
                for a, (lamp, two_Sp) in enumerate(sig):
                    if D[a, b] == 0.0:
                        continue
                    Sp = _R(two_Sp)
                    for two_nup in range(-two_Sp, two_Sp + 1, 2):
                        nup = _R(two_nup)
                        m = nu - nup
                        if abs(m) > lamp:
                            continue
                        c2 = _cg(Sp, nup, lamp, m, J, nu)
                        if c2 == 0.0:
                            continue
                        M[idx[(two_Sp, two_nup)], idx[(two_S, two_nu)]] += (
                            pref * np.sqrt(2 * lam + 1) * c1 * c2 * D[a, b] * _ylm(lamp, int(m), theta))
    return M


def sigma_y_channel_spin():
    """The neutron's sigma_y in the channel-spin basis (2 Sigma, 2 nu) of amplitude_sigma:
    <Sigma nu | sigma_y(n) | Sigma~ nu~> = sum <1 m_d 1/2 s | Sigma nu> (sigma_y)_{s s~} <1 m_d 1/2 s~ | Sigma~ nu~>."""
    states = [(1, -1), (1, 1), (3, -3), (3, -1), (3, 1), (3, 3)]
    sy = {(HALF, HALF): 0.0, (HALF, -HALF): -1j, (-HALF, HALF): 1j, (-HALF, -HALF): 0.0}
    out = np.zeros((6, 6), dtype=complex)
    for a, (two_S, two_nu) in enumerate(states):
        for b, (two_T, two_mu) in enumerate(states):
            v = 0.0
            for md in (-1, 0, 1):
                for s1 in (HALF, -HALF):
                    for s2 in (HALF, -HALF):
                        if sy[(s1, s2)] == 0.0 or md + s1 != _R(two_nu) or md + s2 != _R(two_mu):
                            continue
                        v += (_cg(1, md, HALF, s1, _R(two_S), _R(two_nu)) * sy[(s1, s2)]
                              * _cg(1, md, HALF, s2, _R(two_T), _R(two_mu)))
            out[a, b] = v
    return out


def observables(blocks_jj, k, thetas):
    """dsigma/dOmega (fm^2 / sr) and A_y at each angle; blocks_jj = [(two_J, chans_open, S)] with
    chans_open the (lam, 2I) of the open channels in the order of S."""
    blocks = []
    for two_J, chans, S in blocks_jj:
        sig, Ss = to_sigma(two_J, chans, S)
        blocks.append((two_J, sig, Ss))
    sy = sigma_y_channel_spin()
    ds, ay = [], []
    for th in thetas:
        M = amplitude_sigma(blocks, k, th)
        den = np.trace(M @ M.conj().T).real
        ds.append(den / 6.0)
        ay.append((np.trace(M @ sy @ M.conj().T) / den).real)
    return np.array(ds), np.array(ay)


def amplitude_product_basis(blocks_jj, k, theta):
    """The same amplitude in the product basis (m_d, 2 sigma) from the jj channels (J = j (x) I,
    I = lam (x) 1/2), with no channel-spin step: rows/columns (m_d, 2 sigma) for m_d = -1, 0, 1 and
    sigma = -1/2, 1/2."""
    states = [(md, ts) for md in (-1, 0, 1) for ts in (-1, 1)]
    idx = {s: n for n, s in enumerate(states)}
    M = np.zeros((6, 6), dtype=complex)
    pref = np.sqrt(np.pi) / (1j * k)
    for two_J, chans, S in blocks_jj:
        J = _R(two_J)
        D = np.asarray(S, dtype=complex) - np.eye(len(chans))
        for b, (lam, two_I) in enumerate(chans):
            I = _R(two_I)
            for (md, ts) in states:
                sg = _R(ts)
                nu = md + sg                      # M of the initial state (m_lam = 0)
                if abs(nu) > J or abs(sg) > I:
                    continue
                c_in = _cg(1, md, I, sg, J, nu) * _cg(lam, 0, HALF, sg, I, sg)
                if c_in == 0.0:
                    continue
                for a, (lamp, two_Ip) in enumerate(chans):
                    if D[a, b] == 0.0:
                        continue
                    Ip = _R(two_Ip)
                    for (mdp, tsp) in states:
                        sgp = _R(tsp)
                        mIp = nu - mdp
                        m = mIp - sgp
                        if abs(mIp) > Ip or abs(m) > lamp:
                            continue
                        c_out = _cg(1, mdp, Ip, mIp, J, nu) * _cg(lamp, m, HALF, sgp, Ip, mIp)
                        if c_out == 0.0:
                            continue
                        M[idx[(mdp, tsp)], idx[(md, ts)]] += (
                            pref * np.sqrt(2 * lam + 1) * c_in * c_out * D[a, b] * _ylm(lamp, int(m), theta))
    return M


def sigma_y_product_basis():
    states = [(md, ts) for md in (-1, 0, 1) for ts in (-1, 1)]
    out = np.zeros((6, 6), dtype=complex)
    for a, (md, ts) in enumerate(states):
        for b, (md2, ts2) in enumerate(states):
            if md != md2:
                continue
            if ts == 1 and ts2 == -1:
                out[a, b] = -1j
            elif ts == -1 and ts2 == 1:
                out[a, b] = 1j
    return out


def elastic_cross_section_partial_waves(blocks_jj, k):
    """sigma_el = (pi / k^2) sum_J (2J + 1) / 6 sum_ab |S_ab - delta_ab|^2 (fm^2)."""
    tot = 0.0
    for two_J, chans, S in blocks_jj:
        D = np.asarray(S) - np.eye(len(chans))
        tot += (two_J + 1) / 6.0 * float(np.sum(np.abs(D) ** 2))
    return np.pi / k ** 2 * tot
