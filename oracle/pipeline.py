"""End-to-end oracle driver: lattice -> pseudostates -> g -> P0 -> G1 -> solve -> amplitude.

Oracle: test-only. Follows the five-step scheme of Sec. V.A: (1) bases and coefficients g,
(2)+(3) the nonzero P0 elements, (4) G1, (5) iteration with Pade summation; then the on-shell
amplitude of Sec. II.B.4.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import amplitude as amp
from . import channels as chmod
from . import lattice, potential, pseudostates, recoupling, resolvent, solve
from .perm import P0Lattice, channel_terms

BE_DEUTERON = 2.2246


@dataclass
class Spec:
    M: int
    N: int
    two_J: int
    parity: int = +1
    j_max: int = 1
    swave_only: bool = True
    alpha: float = 1.0
    p_max: float = 10.0
    q_max: float = 10.0
    n_x: int = 8
    n_phi: int = 8
    pot: str = "yamaguchi"           # or "mt"
    beta: float = 1.394
    V_R: float = 1438.72
    mu_R: float = 3.11
    mu_A: float = 1.55
    singlet_ratio: float = 0.82
    target_BE: float = BE_DEUTERON
    h2m: float = lattice.H2M
    exhaustive: bool = False
    weights: str = "unit"            # or "energy" (w(p) ~ sqrt(p), f(q) ~ sqrt(q); Sec. III.B footnote)


@dataclass
class System:
    spec: Spec
    p_edges: np.ndarray
    q_edges: np.ndarray
    chans: list
    C: np.ndarray
    keys: list
    P0geo: P0Lattice
    pair: dict = field(default_factory=dict)   # (l, s) -> dict(eps, O, v, W, bound, bins)
    strength: float = 0.0
    eps0: float = 0.0


def channel_list(spec: Spec):
    ch = chmod.enumerate_channels(spec.two_J, spec.parity, spec.j_max)
    if spec.swave_only:
        ch = [c for c in ch if c[0] == 0 and c[3] == 0]
    return ch


def pair_potential(spec, pe, l, s, strength, YR=None):
    if spec.pot == "yamaguchi":
        if (l, s) != (0, 1):
            return np.zeros((len(pe) - 1, len(pe) - 1))
        if spec.weights == "energy":
            return potential.yamaguchi_wp_energy(pe, spec.beta, strength)
        return potential.yamaguchi_wp(pe, spec.beta, strength)
    YR_, YA_ = potential.mt_parts(pe, l, spec.mu_R, spec.mu_A, spec.weights)
    VA = strength if s == 1 else spec.singlet_ratio * strength
    return spec.V_R * YR_ - VA * YA_


def build_system(spec: Spec) -> System:
    pe = lattice.tangent_edges(spec.M, spec.alpha, spec.p_max)
    qe = lattice.tangent_edges(spec.N, spec.alpha, spec.q_max)
    chans = channel_list(spec)
    gt = {(a, b): recoupling.g_table(chans[a], chans[b], spec.two_J)
          for a in range(len(chans)) for b in range(len(chans))}
    keys, C = channel_terms(chans, gt)
    P = P0Lattice(pe, qe, keys, spec.n_x, spec.n_phi, exhaustive=spec.exhaustive, weights=spec.weights)
    if spec.pot == "yamaguchi":
        strength = potential.tune_yamaguchi(pe, spec.beta, spec.target_BE, spec.h2m, spec.weights)
    else:
        strength = potential.tune_mt(pe, spec.V_R, spec.mu_R, spec.mu_A, spec.target_BE, spec.h2m, spec.weights)
    sysm = System(spec, pe, qe, chans, C, keys, P, strength=strength)
    nbound = 0
    for c in chans:
        key = (c[0], c[1])
        if key in sysm.pair:
            continue
        v = pair_potential(spec, pe, c[0], c[1], strength)
        eps, O = pseudostates.diagonalize(pe, v, spec.h2m, h0=potential.h0_of(pe, spec.h2m, spec.weights))
        nb = int(np.sum(eps < 0))
        if spec.weights == "energy":
            bins = pseudostates.scattering_bins_energy(eps[nb:], spec.h2m)
        else:
            bins = pseudostates.scattering_bins(eps[nb:], spec.h2m)
        sysm.pair[key] = dict(eps=eps, O=O, v=v, W=v @ O.T, nb=nb, bins=bins)
        nbound += nb
    if sysm.pair.get((0, 1), {}).get("nb", 0) != 1 or nbound != 1:
        raise ValueError("expected exactly one two-body bound state (3S1)")
    sysm.eps0 = float(sysm.pair[(0, 1)]["eps"][0])
    return sysm


def initial_channels(sysm: System):
    """Channels with the deuteron (3S1) as pair state: the open elastic channels."""
    return [a for a, c in enumerate(sysm.chans) if c[0] == 0 and c[1] == 1 and c[2] == 1]


def g1_lists(sysm: System, E):
    out = {}
    for key, d in sysm.pair.items():
        bound = list(d["eps"][:d["nb"]])
        diag = resolvent.channel_diagonal_energy if sysm.spec.weights == "energy" else resolvent.channel_diagonal
        out[key] = diag(sysm.q_edges, E, bound, d["bins"], sysm.spec.h2m)
    return out


def kernel(sysm: System, E, P0full=None):
    G1 = g1_lists(sysm, E)
    if P0full is None:
        P0full = sysm.P0geo.full(sysm.C)
    O = [sysm.pair[(c[0], c[1])]["O"] for c in sysm.chans]
    W = [sysm.pair[(c[0], c[1])]["W"] for c in sysm.chans]
    G = [G1[(c[0], c[1])] for c in sysm.chans]
    return solve.FactorizedKernel(P0full, O, W, G, sysm.spec.M, sysm.spec.N)


def solve_energy(sysm: System, E_lab, tol=1e-12, n_max=200, direct=False, P0full=None):
    E = lattice.total_energy(E_lab, sysm.eps0)
    q0 = lattice.q_onshell(E_lab, sysm.spec.h2m)
    j0 = lattice.onshell_bin(sysm.q_edges, q0)
    K = kernel(sysm, E, P0full)
    opens = initial_channels(sysm)
    U = np.zeros((len(opens), len(opens)), dtype=complex)
    iters, conv, errs, series = [], [], [], []
    for b, g0 in enumerate(opens):
        if direct:
            U[:, b] = solve.direct_solve(K, g0, j0, opens)
            iters.append(0)
            conv.append(True)
            errs.append(0.0)
        else:
            est, n, ok, terms, err = solve.iterate_pade(K, g0, j0, opens, tol=tol, n_max=n_max)
            series.append(terms)
            U[:, b] = est
            errs.append(np.max(err / np.maximum(np.abs(est), 1e-300)))
            iters.append(n)
            conv.append(ok)
    if sysm.spec.weights == "energy":
        B0 = 0.75 * sysm.spec.h2m * (sysm.q_edges[j0 + 1] ** 2 - sysm.q_edges[j0] ** 2)
        A = amp.amplitude_matrix_energy(U, B0)
    else:
        dq0 = sysm.q_edges[j0 + 1] - sysm.q_edges[j0]
        A = amp.amplitude_matrix(U, q0, dq0, sysm.spec.h2m)
    S = amp.s_matrix(A)
    return dict(E=E, q0=q0, j0=j0, U=U, A=A, S=S, iters=iters, converged=all(conv), rel_err=max(errs),
                delta=amp.phase_deg(S), eta=amp.inelasticity(S), series=series)


def breakup_elements(sysm: System, E_lab, P0full=None):
    """Breakup transition elements (Sec. II.A; Sec. II.B.4, end): breakup is an inelastic
    transition into the discretised two-body continuum, so its elements are components of the
    same solution, z = U e0 = O y, on the cells of the three-body continuum the energy shell
    crosses: continuum pseudostates k of each channel's pair wave (after its bound states) and q
    bins j where the resolvent G1 has an imaginary part. y from the dense solve (small lattices).

    Returns (cells, {initial b: elements}) with cells a list of (g, k, j) in (g, k, j) order."""
    E = lattice.total_energy(E_lab, sysm.eps0)
    q0 = lattice.q_onshell(E_lab, sysm.spec.h2m)
    j0 = lattice.onshell_bin(sysm.q_edges, q0)
    K = kernel(sysm, E, P0full)
    G1 = g1_lists(sysm, E)
    cells = []
    for g, c in enumerate(sysm.chans):
        nb = sysm.pair[(c[0], c[1])]["nb"]
        G = G1[(c[0], c[1])]
        for k in range(nb, G.shape[0]):
            for j in range(G.shape[1]):
                if G[k, j].imag != 0.0:
                    cells.append((g, k, j))
    out = {}
    for b, g0 in enumerate(initial_channels(sysm)):
        t = K.rotate(solve.direct_solution(K, g0, j0))   # t[g, j, k]
        out[b] = np.array([t[g, j, k] for (g, k, j) in cells])
    return cells, out

