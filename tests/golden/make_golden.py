"""Writes tests/golden/*.json from the oracle only (no product code is imported).

    python tests/golden/make_golden.py [name ...]

swave_mt_100.json: the s-wave Malfliet-Tjon workload (V_R seed 0) at M = N = 100, doublet
(J = 1/2+) and quartet (J = 3/2+), E_lab = 14.1 MeV: geometric P0 size, a seeded sample of
P0 elements (recomputed one by one with the rule), the on-shell amplitudes and series terms a_n.

pw_mt_150.json: the 18-channel Malfliet-Tjon workload (J = 1/2+, j <= 2, V_R seed 0) at
M = N = 150: the number of stored cell pairs (blocks), the 2 x 2 amplitudes at E_lab = 3 and
22.7 MeV and the on-shell series terms a_n of every (energy, initial channel) column. Takes
tens of minutes and ~20 GB of host memory.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import pipeline  # noqa: E402
from oracle.perm import element_rule  # noqa: E402
import workloads  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def swave_mt_100():
    wl = workloads.WORKLOADS["swave_mt_100"]
    V_R = workloads.mt_repulsion(wl["V_R_seed"])
    out = dict(workload="swave_mt_100", V_R=V_R, M=wl["M"], N=wl["N"], E_lab=wl["E_lab"], systems={})
    for sysd in wl["systems"]:
        t0 = time.time()
        spec = pipeline.Spec(M=wl["M"], N=wl["N"], two_J=sysd["two_J"], j_max=sysd["j_max"],
                             swave_only=sysd["swave"], pot="mt", V_R=V_R, n_x=wl["n_x"], n_phi=wl["n_phi"])
        s = pipeline.build_system(spec)
        t1 = time.time()
        res = {}
        for E in wl["E_lab"]:
            r = pipeline.solve_energy(s, E)
            res[str(E)] = dict(A_re=float(r["A"][0, 0].real), A_im=float(r["A"][0, 0].imag),
                               rel_err=float(r["rel_err"]), iters=int(r["iters"][0]),
                               converged=bool(r["converged"]), delta=float(r["delta"][0]), eta=float(r["eta"][0]),
                               series_re=r["series"][0][:, 0].real.tolist(),
                               series_im=r["series"][0][:, 0].imag.tolist())
        rng = np.random.default_rng(5)
        idx = rng.choice(s.P0geo.geo_nnz, 64, replace=False)
        M = wl["M"]
        samples = []
        for k in idx:
            j, i = divmod(int(s.P0geo.rows[k]), M)
            jp, ip = divmod(int(s.P0geo.cols[k]), M)
            v = element_rule(s.p_edges, s.q_edges, i, j, ip, jp, (0, 0, 0, 0, 0), wl["n_x"], wl["n_phi"])
            samples.append([i, j, ip, jp, v])
        out["systems"][str(sysd["two_J"])] = dict(
            channels=[list(c) for c in s.chans], geo_nnz=int(s.P0geo.geo_nnz), strength=float(s.strength),
            eps0=float(s.eps0), results=res, p0_samples=samples, oracle_seconds=time.time() - t0,
            build_seconds=t1 - t0)
        print(sysd, "done", time.time() - t0, flush=True)
    with open(os.path.join(HERE, "swave_mt_100.json"), "w") as f:
        json.dump(out, f, indent=1)


def pw_mt_150():
    from oracle import lattice as olat
    wl = workloads.WORKLOADS["pw_mt_150"]
    V_R = workloads.mt_repulsion(wl["V_R_seed"])
    sysd = wl["systems"][0]
    spec = pipeline.Spec(M=wl["M"], N=wl["N"], two_J=sysd["two_J"], j_max=sysd["j_max"],
                         swave_only=sysd["swave"], pot="mt", V_R=V_R, n_x=wl["n_x"], n_phi=wl["n_phi"])
    t0 = time.time()
    s = pipeline.build_system(spec)
    print("P0 moments", s.P0geo.geo_nnz, "blocks", len(s.keys), "moments", time.time() - t0, flush=True)
    P0full = s.P0geo.full(s.C)
    print("P0 assembled, nnz", P0full.nnz, time.time() - t0, flush=True)
    out = dict(workload="pw_mt_150", V_R=V_R, M=wl["M"], N=wl["N"], channels=[list(c) for c in s.chans],
               blocks=int(s.P0geo.geo_nnz), nnz=int(P0full.nnz), strength=float(s.strength), eps0=float(s.eps0),
               results={})
    for E in wl["E_lab"]:
        r = pipeline.solve_energy(s, E, P0full=P0full)
        out["results"][str(E)] = dict(
            A_re=r["A"].real.tolist(), A_im=r["A"].imag.tolist(), rel_err=float(r["rel_err"]),
            iters=[int(n) for n in r["iters"]], converged=bool(r["converged"]), j0=int(r["j0"]),
            series_re=[t.real.tolist() for t in r["series"]], series_im=[t.imag.tolist() for t in r["series"]])
        print("E", E, "iters", r["iters"], "rel_err", r["rel_err"], time.time() - t0, flush=True)
    out["oracle_seconds"] = time.time() - t0
    with open(os.path.join(HERE, "pw_mt_150.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    names = sys.argv[1:] or ["swave_mt_100"]
    for n in names:
        globals()[n]()
