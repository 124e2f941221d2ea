"""Permutation matrix P0 in the free-WP lattice basis (Appendix; Sec. II.B.3, eq. perm).

Oracle: test-only.

(i) THE RULE (what the product library must reproduce). The Appendix reduces eq. perm, after
the p and p' integrations against the delta functions and the polar substitution
q = Q cos(phi), q' = Q sin(phi) with the analytic Q integration, to

  [P0]^{gg'}_{ij,i'j'} = sum_{l1,l1',k} g^{l1 l1' k}_{gg'} / sqrt(d_i dq_j d_i' dq_j')
        * int_{-1}^{1} dx P_k(x) int_{phi1}^{phi2} dphi F(phi, x)
          cos(phi)^(a+1) sin(phi)^(b+1) / (zeta1^(l'+1) zeta2^(l+1)),

  zeta1 = sqrt(cos^2 + sin^2/4 + x cos sin),  zeta2 = sqrt(cos^2/4 + sin^2 + x cos sin),
  phi1 = atan(q'_{j'-1} / q_j),  phi2 = atan(q'_{j'} / q_{j-1}),
  F = 1/2 U^2 - 1/2 L^2 with U = min(q_j/cos, q'_{j'}/sin, p'_{i'}/zeta1, p_i/zeta2),
                          L = max(q_{j-1}/cos, q'_{j'-1}/sin, p'_{i'-1}/zeta1, p_{i-1}/zeta2),

evaluated with an n_x-point Gauss-Legendre rule in x on [-1, 1] and an n_phi-point rule on
[phi1, phi2]. Readings: F is taken as 0 where U <= L (the printed difference would be negative
on an empty Q range) and written 0.5 (U - L)(U + L); (a, b) = (l1 + l1', l2 + l2') (pinned by
the m-scheme evaluation of G in ``mscheme``); atan of x/0 is pi/2.

(ii) SEMI-ANALYTIC: the 3D (q, q', x) form before the polar substitution with x traded for pi1
(dx = 2 pi1 dpi1 / (q q'), pi2^2 = pi1^2 + 3/4 (q'^2 - q^2)). For s-wave the inner integral is
2 ln(pi1 + pi2) on one exact pi1 interval and the (q, q') box is done adaptively
(``element_semianalytic_s``). For any channel pair the inner integral of G / (pi1^l' pi2^l) is a
smooth integral in w = ln(pi1 + pi2) on the same exact interval, with G supplied by the caller
(the tests pass the m-scheme G, which shares nothing with the moment decomposition of the rule)
and the box done by a composite Gauss rule (``element_semianalytic``).

(iii) BRUTE FORCE: midpoint sums of the 3D theta form on tiny lattices (``element_bruteforce_s``,
``element_bruteforce``).

(iv) ENERGY WEIGHTS (Sec. III.B, footnote: packets with w(p) ~ sqrt(p), f(q) ~ sqrt(q)). The
plane-wave projection gains the factor w(p) f(q) / sqrt(C_i B_j) in place of 1/sqrt(d_i dq_j),
with |w|^2 = 2 H2M p, |f|^2 = (3/2) H2M q, C_i = H2M (p_i^2 - p_{i-1}^2) and
B_j = (3/4) H2M (q_j^2 - q_{j-1}^2). In the integrand of the Appendix this multiplies by
w(pi2) w(pi1) f(q) f(q') = 3 H2M^2 sqrt(pi1 pi2 q q') = 3 H2M^2 Q^2 sqrt(cos sin zeta1 zeta2),
so the Q integral becomes int Q^3 dQ = (U^4 - L^4)/4, and with the constants

  [P0]^{gg'}_{ij,i'j'} = sum g / sqrt(dp2_i dq2_j dp2_i' dq2_j')
        * int dx P_k(x) int dphi (U^4 - L^4) sqrt(cos sin zeta1 zeta2)
          cos^(a+1) sin^(b+1) / (zeta1^(l'+1) zeta2^(l+1)),

dp2_i = p_i^2 - p_{i-1}^2, dq2_j = q_j^2 - q_{j-1}^2: the same rule with F = U^4 - L^4 (written
(U - L)(U + L)(U^2 + L^2)), one more node factor and another norm. The brute force
(``element_bruteforce`` with weights="energy") applies the weights and widths as defined, in
MeV units, so the reduction of the constants is checked too.

Layout used by the oracle: a lattice row/column index is (j, i) -> j * M + i.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as _leg
from scipy import integrate

from .recoupling import exponents


# --------------------------------------------------------------------------- nodes per box

def box_nodes(q_edges, j, jp, n_x, n_phi):
    """Quadrature nodes of the (x, phi) rule for the q-box (j, j'), 0-based bins."""
    qa, qb = q_edges[j], q_edges[j + 1]        # q_{j-1}, q_j
    qpa, qpb = q_edges[jp], q_edges[jp + 1]    # q'_{j'-1}, q'_{j'}
    phi1 = np.arctan2(qpa, qb)
    phi2 = np.arctan2(qpb, qa)
    xg, xw = _leg.leggauss(n_x)
    tg, tw = _leg.leggauss(n_phi)
    phi = 0.5 * (phi1 + phi2) + 0.5 * (phi2 - phi1) * tg
    wphi = 0.5 * (phi2 - phi1) * tw
    X = np.repeat(xg, n_phi)
    PHI = np.tile(phi, n_x)
    W = np.repeat(xw, n_phi) * np.tile(wphi, n_x)
    c, s = np.cos(PHI), np.sin(PHI)
    z1 = np.sqrt(c * c + 0.25 * s * s + X * c * s)
    z2 = np.sqrt(0.25 * c * c + s * s + X * c * s)
    Q1 = np.maximum(qa / c, qpa / s)
    Q2 = np.minimum(qb / c, qpb / s)
    return dict(x=X, c=c, s=s, z1=z1, z2=z2, Q1=Q1, Q2=Q2, w=W, ew=np.sqrt(c * s * z1 * z2))


def moment_weight(nodes, key, weights="unit"):
    """Node weight of moment key = (k, a, b, l, l'): w P_k(x) c^(a+1) s^(b+1) / (z1^(l'+1) z2^(l+1)),
    times sqrt(c s z1 z2) for energy weights."""
    k, a, b, l, lp = key
    Pk = _leg.legval(nodes["x"], [0.0] * k + [1.0])
    wt = (nodes["w"] * Pk * nodes["c"] ** (a + 1) * nodes["s"] ** (b + 1)
          / (nodes["z1"] ** (lp + 1) * nodes["z2"] ** (l + 1)))
    return wt * nodes["ew"] if weights == "energy" else wt


def pair_norm(p_edges, q_edges, ii, j, iip, jp, weights="unit"):
    """1/sqrt(d_i dq_j d_i' dq_j') (unit) or 1/sqrt(dp2_i dq2_j dp2_i' dq2_j') (energy weights)."""
    if weights == "energy":
        dp = p_edges[1:] ** 2 - p_edges[:-1] ** 2
        dq = q_edges[1:] ** 2 - q_edges[:-1] ** 2
    else:
        dp = np.diff(p_edges)
        dq = np.diff(q_edges)
    return 1.0 / np.sqrt(dp[ii] * dq[j] * dp[iip] * dq[jp])


def F_values(p_edges, nodes, ii, iip, weights="unit"):
    """F at every node for the cell pairs (i, i') given as index arrays -> (npairs, nnodes):
    (U^2 - L^2)/2 for unit weights, U^4 - L^4 for energy weights, 0 where U <= L."""
    z1 = nodes["z1"][None, :]
    z2 = nodes["z2"][None, :]
    U = np.minimum(np.minimum(nodes["Q2"][None, :], p_edges[iip + 1][:, None] / z1),
                   p_edges[ii + 1][:, None] / z2)
    L = np.maximum(np.maximum(nodes["Q1"][None, :], p_edges[iip][:, None] / z1),
                   p_edges[ii][:, None] / z2)
    if weights == "energy":
        return np.where(U > L, (U - L) * (U + L) * (U * U + L * L), 0.0)
    return np.where(U > L, 0.5 * (U - L) * (U + L), 0.0)


def candidate_pairs(p_edges, nodes):
    """All (i, i') for which some node has F > 0 (widened by one bin each side).

    For one node and row i, F > 0 needs A < B with A = max(Q1, p_{i-1}/z2), B = min(Q2, p_i/z2)
    and p'_{i'-1} < B z1, p'_{i'} > A z1: a contiguous i' range. The union over nodes is
    covered by its hull.
    """
    M = len(p_edges) - 1
    pa, pb = p_edges[:-1], p_edges[1:]
    A = np.maximum(nodes["Q1"][None, :], pa[:, None] / nodes["z2"][None, :])
    B = np.minimum(nodes["Q2"][None, :], pb[:, None] / nodes["z2"][None, :])
    ok = A < B
    lo = np.searchsorted(p_edges, (A * nodes["z1"][None, :]).ravel(), side="right").reshape(A.shape) - 1
    hi = np.searchsorted(p_edges, (B * nodes["z1"][None, :]).ravel(), side="left").reshape(B.shape) - 1
    lo = np.where(ok, lo, M + 10)
    hi = np.where(ok, hi, -10)
    lo_i = np.clip(lo.min(axis=1) - 1, 0, M - 1)
    hi_i = np.clip(hi.max(axis=1) + 1, 0, M - 1)
    ii, iip = [], []
    for i in range(M):
        if hi.max(axis=1)[i] < 0:
            continue
        r = np.arange(lo_i[i], hi_i[i] + 1)
        ii.append(np.full(len(r), i))
        iip.append(r)
    if not ii:
        return np.zeros(0, int), np.zeros(0, int)
    return np.concatenate(ii), np.concatenate(iip)


# --------------------------------------------------------------------------- channel terms

def channel_terms(chans, gtabs):
    """Distinct moment keys and the coefficient array C[g, g', m] (g summed over terms)."""
    keys = []
    index = {}
    n = len(chans)
    entries = []
    for a, ca in enumerate(chans):
        for b, cb in enumerate(chans):
            for (l1, l1p, k), gv in gtabs[(a, b)].items():
                ea, eb = exponents(ca, cb, l1, l1p)
                key = (k, ea, eb, ca[0], cb[0])
                if key not in index:
                    index[key] = len(keys)
                    keys.append(key)
                entries.append((a, b, index[key], gv))
    C = np.zeros((n, n, len(keys)))
    for a, b, m, gv in entries:
        C[a, b, m] += gv
    return keys, C


# --------------------------------------------------------------------------- P0 build

class P0Lattice:
    """Geometric P0 data: for every q-box, the stored cell pairs and their moment integrals."""

    def __init__(self, p_edges, q_edges, keys, n_x=8, n_phi=8, exhaustive=False, weights="unit"):
        self.p_edges = np.asarray(p_edges, float)
        self.q_edges = np.asarray(q_edges, float)
        self.M = len(p_edges) - 1
        self.N = len(q_edges) - 1
        self.keys = list(keys)
        self.n_x, self.n_phi = n_x, n_phi
        self.weights = weights
        rows, cols, moms = [], [], []
        M, N = self.M, self.N
        for j in range(N):
            for jp in range(N):
                nodes = box_nodes(self.q_edges, j, jp, n_x, n_phi)
                if exhaustive:
                    ii, iip = np.meshgrid(np.arange(M), np.arange(M), indexing="ij")
                    ii, iip = ii.ravel(), iip.ravel()
                else:
                    ii, iip = candidate_pairs(self.p_edges, nodes)
                if len(ii) == 0:
                    continue
                F = F_values(self.p_edges, nodes, ii, iip, weights)
                Wm = np.stack([moment_weight(nodes, key, weights) for key in self.keys], axis=1)
                mom = F @ Wm
                norm = pair_norm(self.p_edges, self.q_edges, ii, j, iip, jp, weights)
                mom *= norm[:, None]
                keep = np.any(mom != 0.0, axis=1)
                rows.append(j * M + ii[keep])
                cols.append(jp * M + iip[keep])
                moms.append(mom[keep])
        self.rows = np.concatenate(rows) if rows else np.zeros(0, int)
        self.cols = np.concatenate(cols) if cols else np.zeros(0, int)
        self.moms = np.concatenate(moms) if moms else np.zeros((0, len(keys)))
        order = np.lexsort((self.cols, self.rows))
        self.rows, self.cols, self.moms = self.rows[order], self.cols[order], self.moms[order]

    @property
    def geo_nnz(self):
        return len(self.rows)

    def channel_block(self, C, a, b):
        """Sparse (M N x M N) block P0^{ab} = sum_m C[a, b, m] moment_m, exact zeros dropped."""
        v = self.moms @ C[a, b]
        keep = v != 0.0
        D = self.M * self.N
        return sp.csr_matrix((v[keep], (self.rows[keep], self.cols[keep])), shape=(D, D))

    def full(self, C):
        """Full P0 in the channel-major layout (g, j, i) -> (g N + j) M + i."""
        n = C.shape[0]
        blocks = [[self.channel_block(C, a, b) for b in range(n)] for a in range(n)]
        return sp.bmat(blocks, format="csr")


def element_rule(p_edges, q_edges, i, j, ip, jp, key, n_x, n_phi, weights="unit"):
    """One moment integral of one cell pair by the rule (for sampled checks at full size)."""
    p_edges, q_edges = np.asarray(p_edges, float), np.asarray(q_edges, float)
    nodes = box_nodes(q_edges, j, jp, n_x, n_phi)
    F = F_values(p_edges, nodes, np.array([i]), np.array([ip]), weights)[0]
    return float(F @ moment_weight(nodes, key, weights)) * float(pair_norm(p_edges, q_edges, i, j, ip, jp, weights))


# --------------------------------------------------------------------------- pins (s-wave)

def element_semianalytic_s(p_edges, q_edges, i, j, ip, jp, epsabs=1e-13, epsrel=1e-11):
    """Exact s-wave moment (l = l' = k = 0) of one cell pair, adaptive 2D integration.

    int_{Dq_j} dq int_{Dq_j'} dq' int dx q q' / (pi1 pi2) theta(pi1 in D_i') theta(pi2 in D_i)
    with x -> pi1: inner = 2 [ln(pi1 + pi2)] over
    [|q - q'/2|, q + q'/2] cap [p'_{i'-1}, p'_{i'}] cap {pi1^2 in [p_{i-1}^2 - c, p_i^2 - c]},
    c = 3/4 (q'^2 - q^2).
    """
    pa, pb = p_edges[i], p_edges[i + 1]
    ppa, ppb = p_edges[ip], p_edges[ip + 1]

    def inner(qp, q):
        c = 0.75 * (qp * qp - q * q)
        lo = max(abs(q - 0.5 * qp), ppa, np.sqrt(max(0.0, pa * pa - c)))
        if pb * pb - c <= 0.0:
            return 0.0
        hi = min(q + 0.5 * qp, ppb, np.sqrt(pb * pb - c))
        if hi <= lo:
            return 0.0
        f = lambda r: np.log(r + np.sqrt(max(0.0, r * r + c)))
        return 2.0 * (f(hi) - f(lo))

    qa, qb = q_edges[j], q_edges[j + 1]
    qpa, qpb = q_edges[jp], q_edges[jp + 1]
    val, _ = integrate.dblquad(inner, qa, qb, qpa, qpb, epsabs=epsabs, epsrel=epsrel)
    dp = np.diff(p_edges)
    dq = np.diff(q_edges)
    return val / np.sqrt(dp[i] * dq[j] * dp[ip] * dq[jp])


def element_bruteforce_s(p_edges, q_edges, i, j, ip, jp, n):
    """Midpoint sum with n^3 points of the 3D (q, q', x) theta form, s-wave."""
    qa, qb = q_edges[j], q_edges[j + 1]
    qpa, qpb = q_edges[jp], q_edges[jp + 1]
    t = (np.arange(n) + 0.5) / n
    q = qa + (qb - qa) * t
    qp = qpa + (qpb - qpa) * t
    x = -1.0 + 2.0 * t
    Q, QP, X = np.meshgrid(q, qp, x, indexing="ij")
    pi1 = np.sqrt(Q * Q + 0.25 * QP * QP + Q * QP * X)
    pi2 = np.sqrt(0.25 * Q * Q + QP * QP + Q * QP * X)
    th = ((pi1 > p_edges[ip]) & (pi1 <= p_edges[ip + 1]) & (pi2 > p_edges[i]) & (pi2 <= p_edges[i + 1]))
    f = np.where(th, Q * QP / (pi1 * pi2), 0.0)
    vol = (qb - qa) * (qpb - qpa) * 2.0 / n ** 3
    dp = np.diff(p_edges)
    dq = np.diff(q_edges)
    return f.sum() * vol / np.sqrt(dp[i] * dq[j] * dp[ip] * dq[jp])


# --------------------------------------------------------------------------- pins (any channel pair)

def element_rule_channel(p_edges, q_edges, i, j, ip, jp, keys, Cab, n_x, n_phi, weights="unit"):
    """Channel-pair element sum_m C[g, g', m] * moment_m of one cell pair by the rule."""
    return float(sum(c * element_rule(p_edges, q_edges, i, j, ip, jp, key, n_x, n_phi, weights)
                     for key, c in zip(keys, Cab) if c != 0.0))


def element_semianalytic(p_edges, q_edges, i, j, ip, jp, G, l, lp, n_w=24, n_sub=96, n_g=6, weights="unit",
                         h2m=41.471):
    """Channel-pair element of P0 from the 3D kernel, for any l, l' (eq. P_kern before the polar step).

    With the kernel delta(p' - pi1) delta(p - pi2) G(q, q', x) / (p'^(l'+2) p^(l+2)) and the unit
    momentum weights, the element is

        (d_i dq_j d_i' dq_j')^(-1/2) int dq int dq' int dx q q' G / (pi1^(l'+1) pi2^(l+1))
                                          * theta(pi1 in D_i') theta(pi2 in D_i).

    x -> pi1 (dx = 2 pi1 dpi1 / (q q')) and then w = ln(pi1 + pi2) (dpi1 / pi2 = dw, which
    removes the 1/pi2 end singularity) turn the x integral into

        2 int dw G(q, q', x(w)) / (pi1^l' pi2^l),  pi1 = (e^w - c e^-w)/2, pi2 = (e^w + c e^-w)/2,

    c = 3/4 (q'^2 - q^2), over the exact pi1 interval [|q - q'/2|, q + q'/2] cap D_i' cap
    {pi2 in D_i}. That smooth integral takes an n_w-point Gauss rule. The result is a continuous
    function of (q, q') with kinks where the interval ends switch, integrated over the box by a
    composite Gauss rule (n_sub panels of n_g points per axis; error O(n_sub^-2) at the kinks).
    G is any vectorised callable (for the pin: the m-scheme polynomial).

    weights="energy": the integrand gains w(pi2) w(pi1) f(q) f(q') (|w|^2 = 2 h2m p, |f|^2 =
    (3/2) h2m q) and the widths are the energy widths C_i, B_j (MeV), as defined.
    """
    pa, pb = p_edges[i], p_edges[i + 1]
    ppa, ppb = p_edges[ip], p_edges[ip + 1]
    tg, tw = _leg.leggauss(n_w)
    gg, gw = _leg.leggauss(n_g)

    def composite(a, b):
        h = (b - a) / n_sub
        mids = a + h * (np.arange(n_sub) + 0.5)
        return (mids[:, None] + 0.5 * h * gg[None, :]).ravel(), np.tile(0.5 * h * gw, n_sub)

    q, wq = composite(q_edges[j], q_edges[j + 1])
    qp, wqp = composite(q_edges[jp], q_edges[jp + 1])
    Q, QP = np.meshgrid(q, qp, indexing="ij")
    W2 = np.outer(wq, wqp)
    Q, QP, W2 = Q.ravel(), QP.ravel(), W2.ravel()
    c = 0.75 * (QP * QP - Q * Q)
    lo = np.maximum(np.maximum(np.abs(Q - 0.5 * QP), ppa), np.sqrt(np.maximum(0.0, pa * pa - c)))
    hi = np.minimum(np.minimum(Q + 0.5 * QP, ppb), np.sqrt(np.maximum(0.0, pb * pb - c)))
    ok = (pb * pb - c > 0.0) & (hi > lo)
    Q, QP, W2, c, lo, hi = Q[ok], QP[ok], W2[ok], c[ok], lo[ok], hi[ok]
    w0 = np.log(lo + np.sqrt(np.maximum(0.0, lo * lo + c)))
    w1 = np.log(hi + np.sqrt(np.maximum(0.0, hi * hi + c)))
    w = 0.5 * (w0 + w1)[:, None] + 0.5 * (w1 - w0)[:, None] * tg[None, :]
    e, ei = np.exp(w), np.exp(-w)
    pi1 = 0.5 * (e - c[:, None] * ei)
    pi2 = 0.5 * (e + c[:, None] * ei)
    Qb, QPb = Q[:, None], QP[:, None]
    x = np.clip((pi1 * pi1 - Qb * Qb - 0.25 * QPb * QPb) / (Qb * QPb), -1.0, 1.0)
    f = G(Qb, QPb, x) / (pi1 ** lp * pi2 ** l)
    if weights == "energy":
        f = f * np.sqrt(2.0 * h2m * pi2) * np.sqrt(2.0 * h2m * pi1)
        W2 = W2 * np.sqrt(1.5 * h2m * Q) * np.sqrt(1.5 * h2m * QP)
    inner = 2.0 * 0.5 * (w1 - w0) * (f @ tw)
    if weights == "energy":
        C = h2m * (p_edges[1:] ** 2 - p_edges[:-1] ** 2)
        B = 0.75 * h2m * (q_edges[1:] ** 2 - q_edges[:-1] ** 2)
        return float(np.dot(W2, inner)) / np.sqrt(C[i] * B[j] * C[ip] * B[jp])
    dp = np.diff(p_edges)
    dq = np.diff(q_edges)
    return float(np.dot(W2, inner)) / np.sqrt(dp[i] * dq[j] * dp[ip] * dq[jp])


def element_bruteforce(p_edges, q_edges, i, j, ip, jp, G, l, lp, n, weights="unit", h2m=41.471):
    """Midpoint sum with n^3 points of the 3D (q, q', x) theta form for any channel pair.

    weights="energy": the integrand is multiplied by w(pi2) w(pi1) f(q) f(q') with |w(p)|^2 =
    2 h2m p and |f(q)|^2 = (3/2) h2m q, and divided by sqrt(C_i B_j C_i' B_j') (energy widths)
    instead of the momentum widths."""
    qa, qb = q_edges[j], q_edges[j + 1]
    qpa, qpb = q_edges[jp], q_edges[jp + 1]
    t = (np.arange(n) + 0.5) / n
    q = qa + (qb - qa) * t
    qp = qpa + (qpb - qpa) * t
    x = -1.0 + 2.0 * t
    Q, QP, X = np.meshgrid(q, qp, x, indexing="ij")
    pi1 = np.sqrt(Q * Q + 0.25 * QP * QP + Q * QP * X)
    pi2 = np.sqrt(0.25 * Q * Q + QP * QP + Q * QP * X)
    th = ((pi1 > p_edges[ip]) & (pi1 <= p_edges[ip + 1]) & (pi2 > p_edges[i]) & (pi2 <= p_edges[i + 1]))
    f = np.where(th, Q * QP * G(Q, QP, X) / (pi1 ** (lp + 1) * pi2 ** (l + 1)), 0.0)
    vol = (qb - qa) * (qpb - qpa) * 2.0 / n ** 3
    if weights == "energy":
        wgt = np.sqrt(2.0 * h2m * pi2) * np.sqrt(2.0 * h2m * pi1) * np.sqrt(1.5 * h2m * Q) * np.sqrt(1.5 * h2m * QP)
        C = h2m * (p_edges[1:] ** 2 - p_edges[:-1] ** 2)
        B = 0.75 * h2m * (q_edges[1:] ** 2 - q_edges[:-1] ** 2)
        return (f * wgt).sum() * vol / np.sqrt(C[i] * B[j] * C[ip] * B[jp])
    dp = np.diff(p_edges)
    dq = np.diff(q_edges)
    return f.sum() * vol / np.sqrt(dp[i] * dq[j] * dp[ip] * dq[jp])
