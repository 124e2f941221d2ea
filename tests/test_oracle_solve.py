"""Pins for the oracle's resolvent, Pade summation, solve and amplitude."""
import mpmath
import numpy as np
import pytest

from oracle import lattice, pipeline, resolvent, solve

H = lattice.H2M
B3 = 0.75 * H


def test_bound_continuum_vs_mpmath():
    qe = lattice.tangent_edges(20)
    eps0 = -2.2246
    E = eps0 + 2.0 * 14.1 / 3.0
    q0 = np.sqrt((E - eps0) / B3)
    G = resolvent.bound_continuum(qe, E, eps0)
    mpmath.mp.dps = 30
    for j in range(20):
        a, b = qe[j], qe[j + 1]
        g = lambda q: 1 / (B3 * (q0 + q))      # 1/(b3 (q0^2 - q^2)) = g(q)/(q0 - q)
        if a < q0 <= b:
            smooth = mpmath.quad(lambda q: (g(q) - g(q0)) / (q0 - q), [a, q0, b])
            pv = smooth + g(q0) * mpmath.log((q0 - a) / (b - q0))
            im = -mpmath.pi * g(q0)
        else:
            pv = mpmath.quad(lambda q: g(q) / (q0 - q), [a, b])
            im = 0
        ref = complex(pv, im) / (b - a)
        assert G[j] == pytest.approx(ref, rel=1e-12, abs=1e-14)


def _continuum_ref(pa, pb, qa, qb, E):
    """Swapped order: q integral analytic for fixed p, p integral by mpmath; delta part by arc."""
    mpmath.mp.dps = 30
    sb = mpmath.sqrt(B3)

    def inner_q(p):
        c2 = E - H * p * p
        if c2 > 0:
            c = mpmath.sqrt(c2)
            f = lambda q: mpmath.log(abs((c + sb * q) / (c - sb * q)))
            return (f(qb) - f(qa)) / (2 * c * sb)
        k = mpmath.sqrt(-c2)
        return -(mpmath.atan(sb * qb / k) - mpmath.atan(sb * qa / k)) / (sb * k)
    pts = [pa]
    for c2q in (E - B3 * qa * qa, E - B3 * qb * qb, E):
        if c2q > 0:
            ps = float(mpmath.sqrt(c2q / H))
            if pa < ps < pb:
                pts.append(ps)
    pts = sorted(pts) + [pb]
    re = mpmath.quad(inner_q, pts)
    # imaginary part: -pi int dp int dq delta(E - H p^2 - b3 q^2) = -pi int dp 1/(2 b3 q(p))
    im = 0
    if E > 0:
        def dens(p):
            c2 = E - H * p * p
            if c2 <= 0:
                return 0
            q = mpmath.sqrt(c2 / B3)
            return 1 / (2 * B3 * q) if qa < q < qb else 0
        lo = pa
        hi = min(pb, float(mpmath.sqrt(E / H)))
        if hi > lo:
            cuts = [lo] + [x for x in (float(mpmath.sqrt(max(0, (E - B3 * qb * qb) / H))),
                                       float(mpmath.sqrt(max(0, (E - B3 * qa * qa) / H)))) if lo < x < hi] + [hi]
            im = -mpmath.pi * mpmath.quad(dens, sorted(cuts))
    return complex(re, im) / ((pb - pa) * (qb - qa))


@pytest.mark.parametrize("E", [-1.5, 4.44, 12.9])
def test_continuum_element_vs_swapped_order(E):
    boxes = [(0.1, 0.4, 0.2, 0.5), (0.3, 0.8, 0.1, 0.45), (0.0, 0.05, 0.0, 0.07), (0.5, 0.6, 0.4, 0.9)]
    for pa, pb, qa, qb in boxes:
        g = resolvent.continuum_element(pa, pb, qa, qb, E)
        ref = _continuum_ref(pa, pb, qa, qb, E)
        assert g == pytest.approx(ref, rel=1e-9, abs=1e-12), (pa, pb, qa, qb)


def _energy_route_ref(pa, pb, qa, qb, E):
    """A third route to the continuum element, in 30-digit arithmetic: with eps = h p^2 + b3 q^2 and
    the polar angle of the ellipse as second variable (dp dq = d eps dt / (2 sqrt(h b3))),
    int int dp dq / (E + i0 - eps) = (1 / (2 sqrt(h b3))) int d eps theta(eps) / (E + i0 - eps),
    theta(eps) = angle of the ellipse eps inside the box (closed form). The principal value is
    taken by subtracting theta(E); the imaginary part is -pi theta(E) / (2 sqrt(h b3)).
    Breakpoints: the four corner energies (kinks of theta) and E."""
    with mpmath.workdps(30):
        h = mpmath.mpf(H)
        b3 = h * 3 / 4
        pa, pb, qa, qb, E = [mpmath.mpf(x) for x in (pa, pb, qa, qb, E)]

        def theta(e):
            if e <= 0:
                return mpmath.mpf(0)
            P, Q = mpmath.sqrt(e / h), mpmath.sqrt(e / b3)
            lo = max(mpmath.acos(min(1, pb / P)), mpmath.asin(min(1, qa / Q)))
            hi = min(mpmath.acos(min(1, pa / P)), mpmath.asin(min(1, qb / Q)))
            return max(mpmath.mpf(0), hi - lo)
        corners = sorted({h * pa * pa + b3 * qa * qa, h * pb * pb + b3 * qa * qa, h * pa * pa + b3 * qb * qb,
                          h * pb * pb + b3 * qb * qb})
        lo, hi = corners[0], corners[-1]
        inside = lo < E < hi
        tE = theta(E) if inside else 0
        re = mpmath.quad(lambda e: (theta(e) - tE) / (E - e), sorted(set(corners + ([E] if inside else []))))
        if inside:
            re += tE * mpmath.log((E - lo) / (hi - E))
        c = 1 / (2 * mpmath.sqrt(h * b3))
        return complex(c * re, -mpmath.pi * c * tE) / float((pb - pa) * (qb - qa))


@pytest.mark.parametrize("E_lab", [3.0, 3.336, 3.34, 14.1, 28.1, 45.0])
def test_continuum_elements_vs_energy_route(E_lab):
    """Every continuum element of a small MT doublet lattice (both pair waves), below and above the
    breakup threshold (E_lab = 3.337 MeV) and next to it, against the energy route to 1e-13."""
    s = pipeline.build_system(pipeline.Spec(M=6, N=7, two_J=1, pot="mt"))
    E = lattice.total_energy(E_lab, s.eps0)
    for d in s.pair.values():
        G = resolvent.channel_diagonal(s.q_edges, E, list(d["eps"][:d["nb"]]), d["bins"])
        bins, nb = d["bins"], d["nb"]
        for k in range(len(bins) - 1):
            for j in range(len(s.q_edges) - 1):
                ref = _energy_route_ref(bins[k], bins[k + 1], s.q_edges[j], s.q_edges[j + 1], E)
                assert abs(G[nb + k, j] - ref) <= 1e-13 * abs(ref), (E_lab, k, j, G[nb + k, j], ref)


def test_wynn_known_series():
    # alternating series for ln 2
    est, _ = solve.pade_sum([(-1) ** n / (n + 1) for n in range(24)])
    assert est == pytest.approx(np.log(2.0), abs=1e-13)
    # divergent geometric series 1 + 2 + 4 + ... = 1/(1 - 2) as a Pade value
    est, _ = solve.pade_sum([2.0 ** n for n in range(6)])
    assert est == pytest.approx(-1.0, abs=1e-13)


@pytest.fixture(scope="module")
def small_systems():
    out = {}
    out["quartet"] = pipeline.build_system(pipeline.Spec(M=16, N=16, two_J=3, pot="yamaguchi"))
    out["doublet"] = pipeline.build_system(pipeline.Spec(M=16, N=16, two_J=1, pot="mt"))
    return out


@pytest.mark.parametrize("name", ["quartet", "doublet"])
@pytest.mark.parametrize("E_lab", [1.0, 3.0, 10.0, 14.1])
def test_pade_matches_direct_solve(small_systems, name, E_lab):
    s = small_systems[name]
    r = pipeline.solve_energy(s, E_lab)
    d = pipeline.solve_energy(s, E_lab, direct=True)
    assert r["converged"]
    err = abs(r["A"][0, 0] - d["A"][0, 0]) / abs(d["A"][0, 0])
    if name == "quartet":
        assert err < 1e-12
    else:   # divergent series: Pade reaches a rounding floor, estimated by the stop rule
        assert err < max(30 * r["rel_err"], 1e-12) and err < 1e-8


@pytest.mark.parametrize("name", ["quartet", "doublet"])
@pytest.mark.parametrize("E_lab", [1.0, 2.0, 3.0])
def test_unitarity_below_breakup(small_systems, name, E_lab):
    """Below breakup G1 has one imaginary entry, so S = (1 - i pi K)/(1 + i pi K) exactly."""
    d = pipeline.solve_energy(small_systems[name], E_lab, direct=True)
    assert abs(d["S"][0, 0]) == pytest.approx(1.0, abs=1e-12)
