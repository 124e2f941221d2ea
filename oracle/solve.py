"""Matrix Faddeev equation U = P V1 + P V1 G1 U (eq. m_pvg) in factorised form. Oracle: test-only.

In the SWP basis P = O P0 O^T (eq. perm_z, O block-diagonal over (channel, q-bin)),
V1 = O v O^T and G1 is diagonal (eq. dg1). Only the column of U belonging to the initial
state e0 = Z_{0 j0} (deuteron x q-bin j0) is needed. With y = O^T U e0 the equation becomes a
lattice-space one with the kernel stored as factors (Sec. V.A):

    y = b + K y,   b = P0 (v O^T) e0,   K = P0 (v O^T) G1 O,

and U_00 = e0^T O y. It is solved as in the paper (Sec. II.A; Sec. V.A step 5) by iteration,
y_n = K^n b, a_n = e0^T O y_n, summing sum_n a_n with Pade approximants (Wynn's epsilon
algorithm on the partial sums), and, as a pin, by a direct dense solve of (I - K) y = b.

Reading of the Pade step (the paper names no variant): Wynn epsilon on the partial sums
S_n = a_0 + ... + a_n; the estimate E_n after n + 1 terms is the newest entry of the highest
even column whose magnitude is below 1e200; a zero difference (|d| < 1e-300) makes the next
entry 1e300 (a column that has converged exactly). With
r_n = |E_n - E_{n-1}| / |E_n|:
  * converged when r_n <= tol at two successive n;
  * for a divergent series the estimates reach a rounding floor (about eps * max|S_n| / |U|)
    and wander there, so the iteration also stops once the smallest r seen has not improved
    for PLATEAU terms (or |S_n| exceeds 1e250); it then returns the estimate with the
    smallest r, accepted when that r <= accept;
  * otherwise it fails after n_max terms.
The returned error estimate is that smallest r (times |E|).
"""

from __future__ import annotations

import numpy as np

PLATEAU = 24


class WynnEpsilon:
    """Incremental Wynn epsilon table for a (complex) sequence of partial sums."""

    def __init__(self):
        self.diag = []   # previous anti-diagonal: eps_k^{(n-1-k)} for k = 0..n-1
        self.n = 0

    def push(self, S):
        new = [complex(S)]
        prev = self.diag
        # eps_{k+1}^{(n-1-k)} = eps_{k-1}^{(n-k)} + 1/(eps_k^{(n-k)} - eps_k^{(n-1-k)})
        for k in range(len(prev)):
            d = new[k] - prev[k]
            inv = 1e300 if abs(d) < 1e-300 else 1.0 / d
            lower = prev[k - 1] if k >= 1 else 0.0
            new.append(lower + inv)
        self.diag = new
        self.n += 1
        # newest entry of the highest even column not swamped by a breakdown sentinel
        for k in range((len(new) - 1) // 2 * 2, -1, -2):
            if abs(new[k]) < 1e200:
                return new[k]
        return new[0]


def pade_sum(terms, tol=1e-12, n_min=4):
    """Run Wynn epsilon over a list of series terms; returns (estimate, history)."""
    w = WynnEpsilon()
    S = 0.0
    hist = []
    for a in terms:
        S += a
        hist.append(w.push(S))
    return hist[-1], hist


class FactorizedKernel:
    """K = P0 . blockdiag(W) . diag(G1) . blockdiag(O) in the channel-major layout (g, j, i)."""

    def __init__(self, P0, O_list, W_list, G1_list, M, N):
        self.P0 = P0
        self.O = O_list          # per channel: (M, M), rows = pseudostates
        self.W = W_list          # per channel: v O^T (M, M)
        self.G = G1_list         # per channel: (M, N) indexed [k, j]
        self.M, self.N = M, N
        self.n = len(O_list)

    def rotate(self, y):
        """t = O y: t[g, j, k] = sum_i O_g[k, i] y[g, j, i]."""
        Y = y.reshape(self.n, self.N, self.M)
        return np.stack([Y[g] @ self.O[g].T for g in range(self.n)])

    def apply_rest(self, t):
        """P0 W (G1 * t)."""
        s = np.stack([(t[g] * self.G[g].T) @ self.W[g].T for g in range(self.n)])
        return self.P0 @ s.reshape(-1)

    def apply(self, y):
        return self.apply_rest(self.rotate(y))

    def rhs(self, g0, j0, k0=0):
        e = np.zeros((self.n, self.N, self.M), dtype=complex)
        e[g0, j0, :] = self.W[g0][:, k0]
        return self.P0 @ e.reshape(-1)

    def dense(self):
        D = self.n * self.N * self.M
        K = np.zeros((D, D), dtype=complex)
        for c in range(D):
            e = np.zeros(D, dtype=complex)
            e[c] = 1.0
            K[:, c] = self.apply(e)
        return K


def iterate_pade(K: FactorizedKernel, g0, j0, finals, tol=1e-12, n_max=200, accept=1e-7):
    """Neumann iteration with Wynn-epsilon summation of the on-shell series.

    finals: channels a whose elements U_{a0} = e_a^T O y are summed (e_a = (a, j0, k = 0)).
    Returns (estimates per final, terms used, converged flag, raw terms array, error estimate).
    The stopping rule is applied to the worst of the finals.
    """
    y = K.rhs(g0, j0)
    nf = len(finals)
    ws = [WynnEpsilon() for _ in finals]
    S = np.zeros(nf, dtype=complex)
    last = None
    best, best_r, best_n = None, np.inf, 0
    streak = 0
    terms = []
    for n in range(n_max):
        t = K.rotate(y)
        a = np.array([t[f, j0, 0] for f in finals])
        terms.append(a)
        S += a
        est = np.array([ws[m].push(S[m]) for m in range(nf)])
        if last is not None:
            r = max(abs(est[m] - last[m]) / max(abs(est[m]), 1e-300) for m in range(nf))
            if r < best_r:
                best, best_r, best_n = est.copy(), r, n
            streak = streak + 1 if r <= tol else 0
            if streak >= 2:
                return est, n + 1, True, np.array(terms), r * np.abs(est)
            if n - best_n >= PLATEAU or np.max(np.abs(S)) > 1e250:
                break
        last = est
        y = K.apply_rest(t)
    ok = best is not None and best_r <= accept
    return best, len(terms), ok, np.array(terms), best_r * np.abs(best)


def direct_solution(K: FactorizedKernel, g0, j0):
    """y = (I - K)^{-1} b by dense LU (small lattices only)."""
    import scipy.linalg as sl
    Kd = K.dense()
    b = K.rhs(g0, j0)
    return sl.solve(np.eye(Kd.shape[0]) - Kd, b)


def direct_solve(K: FactorizedKernel, g0, j0, finals):
    """U_{a0} = e_a^T O (I - K)^{-1} b by dense LU (small lattices only)."""
    t = K.rotate(direct_solution(K, g0, j0))
    return np.array([t[f, j0, 0] for f in finals])
