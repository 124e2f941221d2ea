"""Benchmark of the WPCD hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]

Workload (the s-wave Malfliet-Tjon lattice pair, M = N = 100): the doublet (J = 1/2+, 1S0 + 3S1,
D = 20000) and quartet (J = 3/2+, D = 10000) systems with V_R drawn from seed 0, V_A tuned to
the deuteron, 8 x 8 (x, phi) nodes per cell pair, E_lab = 14.1 MeV. Inputs (lattice tables,
pseudostates) are resident before timing.

One step = the whole hot path for both systems: P0 build (selection, quadrature, compaction;
FP64) and one FP64 solve at 14.1 MeV (G1, Neumann iteration, Pade). The JSON line reports
  value        P-elements/s of the P0 build phase (stored channel entries / wall time of the
               synchronised build calls inside the timed region);
  ms_per_step  wall time per step (build + solves);
plus solves/s, the roofline of the dominant kernel (HIP events around every launch, inside the
timed region) and the oracle timed on the host (cpu_baseline).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import workloads  # noqa: E402

WORKLOAD = "swave_mt_100"
HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # FP64 VALU lane-ops/s (one op per lane per clock)
FP64_PEAK_TFLOPS = 78.6

# Algorithmic work per unit (measurement section)
PBUILD_OPS_PER_NODE = 14          # FP64 VALU ops per (cell pair, quadrature node)
AMP_TARGET = 1e-6                 # amplitude error at which the solve paths are compared


def measured_traffic(workload, kernel):
    """HBM bytes (read + written) per launch of `kernel` from the committed rocprofv3 PMC summary
    (profiles/hbm_traffic.json), or None once the kernel sources differ from the profiled ones."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    path = os.path.join(root, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    src = b"".join(open(os.path.join(root, "paper_1404_5253_amd", "csrc", n), "rb").read()
                   for n in ("kernels.hip", "kernels_mixed.hip"))
    if hashlib.sha256(src).hexdigest() != d.get("source_sha256"):
        return None
    e = d.get("kernels", {}).get(workload, {}).get(kernel)
    return None if e is None else e["read_bytes"] + e["write_bytes"]


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched-energy and serving measurements")
    ap.add_argument("--serve-seconds", type=float, default=2.0)
    ap.add_argument("--sweep", action="store_true", help="also time the s-wave P0 build for M = N in 40..400")
    ap.add_argument("--only", choices=["batched", "serving", "pw150"], default=None,
                    help="run only this extra section (no headline step); for profiling runs")
    return ap.parse_args()


def batched_energies_section(wp, torch, L, reps=3):
    """64 energies U[1, 50] MeV (seed 1234) on the resident doublet lattice.

    FP64 path to its rounding floor, then every path at 1e-6 amplitude error: each path's
    tolerance (and Arnoldi cycle length) is chosen by the autotuner on a separate calibration
    draw of 64 energies (seed 4321) against the converged FP64 amplitudes, then timed on the
    bench energies, where the error against the converged FP64 amplitudes is reported."""
    from paper_1404_5253_amd.tune import tune
    Es = workloads.batched_energies()
    Ecal = workloads.batched_energies(seed=4321)
    best, _ = tune(L, Ecal, target=AMP_TARGET, sync=torch.cuda.synchronize)
    out = {"autotuned": {k: {kk: (float(vv) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                         for k, v in best.items()}}
    amps = {}
    runs = [("fp64", "fp64", 1e-12, 0)] + [(f"{m}_at_1e-6", m, v["tol"], v["refine_every"]) for m, v in best.items()]
    for label, mode, tol, cyc in runs:
        L.solve(Es, mode, tol=tol, refine_every=cyc, allow_noconv=True)   # warm-up
        torch.cuda.synchronize()
        wp.wp_profile_reset()
        wp.wp_profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            sol = L.solve(Es, mode, tol=tol, refine_every=cyc, allow_noconv=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        wp.wp_profile_enable(False)
        out[f"kernels_ms_per_batch_{label}"] = {k: round(v[1] / reps, 3) for k, v in wp.wp_profile_read().items()}
        out[f"iters_{label}"] = int(np.max([sol.amplitude(k)["iters"][0] for k in range(len(Es))]))
        amps[label] = np.array([sol.amplitude(k)["A"][0, 0] for k in range(len(Es))])
        out[f"solves_per_s_{label}"] = len(Es) / dt
        out[f"ms_per_batch_{label}"] = dt * 1e3
    out["n_energies"] = len(Es)
    for label in amps:
        if label != "fp64":
            out[f"max_abs_dA_{label}_vs_fp64"] = float(np.max(np.abs(amps[label] - amps["fp64"])))
    fp = out.get("solves_per_s_fp64_at_1e-6")
    mixed = [l for l in amps if l.startswith("mixed")]
    if fp and mixed:
        top = max(mixed, key=lambda l: out[f"solves_per_s_{l}"])
        out["best_mixed"] = top
        out["speedup_best_mixed_over_fp64_at_1e-6"] = out[f"solves_per_s_{top}"] / fp
    return out


SERVING_LATTICES = (   # M = N, two_J, j_max, s-wave only  (channel counts 2, 2, 18, 10)
    (60, 1, 1, True), (100, 1, 1, True), (150, 1, 2, False), (200, 1, 1, False))
SERVING_MODES = (("fp64", dict(tol=3e-7, accept=1e-7, refine_every=0)),
                 ("mixed_split", dict(tol=1e-5, accept=1e-5, refine_every=8)))


def serving_section(wp, torch, V_R, seconds, lats_by_key=None):
    """Poisson stream (200 req/s, seed 2026) over four resident lattices, continuous batching, once
    with FP64 batches and once with split-BF16 mixed batches, each at a stop tolerance that keeps
    the amplitude error below 1e-6; afterwards every served amplitude is compared with a converged
    FP64 solve of the same energy (outside the timing)."""
    from paper_1404_5253_amd.serve import BatchBackend, run_stream
    lats = []
    for (M, two_J, j_max, sw) in SERVING_LATTICES:
        L = (lats_by_key or {}).get((M, two_J, j_max, sw))
        if L is None:
            L = wp.Lattice(M, M, two_J=two_J, j_max=j_max, swave_only=sw)
            L.pseudostates(kind="mt", V_R=V_R)
            L.build_perm("fp64")
        lats.append(L)
    reqs = workloads.serving_requests(len(lats), rate=200.0, duration=seconds)
    # saturation: the same kind of stream at 10x the rate, so that solves/s is the service rate
    sat = workloads.serving_requests(len(lats), rate=2000.0, duration=0.25, seed=7)
    out = {"lattices": [f"M=N={M}, {L.nch} ch" for (M, *_), L in zip(SERVING_LATTICES, lats)], "requests": len(reqs),
           "saturation_requests": len(sat)}
    served = {}
    for mode, kw in SERVING_MODES:
        backs = []
        for L in lats:
            st = torch.cuda.Stream()
            b = BatchBackend(L, slots=32, hbm_budget=16 << 30, terms=8, stream=wp.C.c_void_p(st.cuda_stream),
                             mode=mode, max_iter=400, **kw)
            b._torch_stream = st
            backs.append(b)
        _, sstats = run_stream(backs, sat)
        for b in backs:
            b.close()
        out[f"saturated_{mode}"] = {k: sstats[k] for k in ("n", "p50_ms", "p99_ms", "solves_per_s", "wall_s")}
        backs = []
        for L in lats:
            st = torch.cuda.Stream()
            b = BatchBackend(L, slots=32, hbm_budget=16 << 30, terms=8, stream=wp.C.c_void_p(st.cuda_stream),
                             mode=mode, max_iter=400, **kw)
            b._torch_stream = st
            backs.append(b)
        done, stats = run_stream(backs, reqs)
        for b in backs:
            b.close()
        stats["accepted"] = sum(1 for r in done if r.result.get("accepted", True))
        out[mode] = stats
        served[mode] = {r.rid: (r.lattice, r.E_lab, r.result["A"]) for r in done}
    # accuracy of every served amplitude against a converged FP64 solve (batched per lattice)
    for mode in served:
        worst = 0.0
        for li, L in enumerate(lats):
            items = [(rid, E, A) for rid, (l, E, A) in served[mode].items() if l == li]
            for k0 in range(0, len(items), 64):
                chunk = items[k0:k0 + 64]
                ref = L.solve([E for _, E, _ in chunk], "fp64", tol=1e-12, max_iter=400, allow_noconv=True)
                for k, (_, _, A) in enumerate(chunk):
                    worst = max(worst, float(np.max(np.abs(A - ref.amplitude(k)["A"]))))
        out[mode]["max_abs_dA_vs_converged_fp64"] = worst
    out["speedup_mixed_split_over_fp64_solves_per_s"] = out["mixed_split"]["solves_per_s"] / out["fp64"]["solves_per_s"]
    out["speedup_mixed_split_over_fp64_saturated"] = (out["saturated_mixed_split"]["solves_per_s"]
                                                      / out["saturated_fp64"]["solves_per_s"])
    return out


def pw150_section(wp, torch, V_R, reps=3):
    """18-channel J = 1/2+ lattice (j <= 2), M = N = 150: P0 build rate, the FP64 SpMV against the
    HBM roofline, and the FP64 and mixed solves of E_lab = 3 and 22.7 MeV (one call each)."""
    wl = workloads.WORKLOADS["pw_mt_150"]
    sysd = wl["systems"][0]
    M = wl["M"]
    L = wp.Lattice(M, M, two_J=sysd["two_J"], j_max=sysd["j_max"], swave_only=sysd["swave"], n_x=wl["n_x"],
                   n_phi=wl["n_phi"])
    L.pseudostates(kind="mt", V_R=V_R)
    L.build_perm("fp64")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        st = L.build_perm("fp64")
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    out = dict(channels=L.nch, P_elements=st["nnz"], P_blocks=st["blocks"], P_bytes=st["bytes"],
               build_ms=dt * 1e3, build_device_ms=st["device_ms"], P_elements_per_s=st["nnz"] / dt)
    Es = wl["E_lab"]
    amps = {}
    for mode, tol in (("fp64", 1e-10), ("mixed", 1e-8), ("mixed_split", 1e-8)):
        L.solve(Es, mode, tol=tol, max_iter=400, allow_noconv=True)
        torch.cuda.synchronize()
        wp.wp_profile_reset()
        wp.wp_profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            sol = L.solve(Es, mode, tol=tol, max_iter=400, allow_noconv=True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        wp.wp_profile_enable(False)
        prof = wp.wp_profile_read()
        amps[mode] = np.array([sol.amplitude(k)["A"] for k in range(len(Es))])
        out[f"ms_per_call_{mode}"] = dt * 1e3
        out[f"solves_per_s_{mode}"] = len(Es) / dt
        out[f"kernels_ms_per_call_{mode}"] = {k: round(v[1] / reps, 3) for k, v in prof.items()}
        if mode == "fp64":
            n, ms = prof["spmv64"]
            us = ms / n * 1e3
            byts = st["bytes"] + 2 * 16 * M * M * L.nch * len(Es) * 2
            out["spmv64_roofline"] = dict(bound="hbm", achieved=byts / us / 1e3, peak=HBM_PEAK_GBS, unit="GB/s",
                                          frac=byts / us / 1e3 / HBM_PEAK_GBS, avg_us=us, bytes_per_launch=byts)
    for mode in ("mixed", "mixed_split"):
        out[f"max_abs_dA_{mode}_vs_fp64"] = float(np.max(np.abs(amps[mode] - amps["fp64"])))
        out[f"speedup_{mode}_over_fp64"] = out[f"solves_per_s_{mode}"] / out["solves_per_s_fp64"]
    S = L.solve([Es[0]], "fp64", tol=1e-10, max_iter=400).amplitude(0)["S"]
    out["unitarity_defect_3MeV"] = float(np.max(np.abs(S @ S.conj().T - np.eye(len(S)))))
    return out


def sweep_section(wp, torch, V_R, sizes=(40, 100, 200, 400), reps=3):
    """P0 build of the s-wave quartet lattice (one channel) against M = N: the paper's scaling axis
    (its headline point is M = N = 400 with about 256 million P0 elements)."""
    out = {}
    for M in sizes:
        L = wp.Lattice(M, M, two_J=3, swave_only=True)
        L.pseudostates(kind="mt", V_R=V_R)
        L.build_perm("fp64")
        torch.cuda.synchronize()
        wp.wp_profile_reset()
        wp.wp_profile_enable(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            st = L.build_perm("fp64")
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        wp.wp_profile_enable(False)
        prof = wp.wp_profile_read()
        out[str(M)] = dict(P_elements=st["nnz"], candidates=st["candidates"], build_ms=dt * 1e3,
                           device_ms=st["device_ms"], P_elements_per_s=st["nnz"] / dt,
                           fill=st["nnz"] / float(M * M) ** 2,
                           kernels_ms={k: round(v[1] / reps, 4) for k, v in prof.items()},
                           pbuild_Tops=(st["candidates"] * 64 * PBUILD_OPS_PER_NODE / (prof["pbuild"][1] / reps / 1e3) / 1e12
                                        if "pbuild" in prof else None))
        del L
    return out


def cpu_baseline(V_R, M, N, budget_s=25.0):
    """The oracle as it stands, on a bounded sample: the doublet P0 over a subset of q-boxes
    (rows j < n_rows) and one oracle solve of a smaller lattice; scaled to P-elements/s."""
    from oracle import channels, recoupling
    from oracle.perm import P0Lattice, box_nodes, candidate_pairs, F_values, moment_weight
    import oracle.lattice as olat
    pe = olat.tangent_edges(M)
    qe = olat.tangent_edges(N)
    ch = channels.swave_doublet()
    t0 = time.perf_counter()
    n_el = 0
    boxes = 0
    dp, dq = np.diff(pe), np.diff(qe)
    key = (0, 0, 0, 0, 0)
    for j in range(N):
        for jp in range(N):
            nodes = box_nodes(qe, j, jp, 8, 8)
            ii, iip = candidate_pairs(pe, nodes)
            if len(ii):
                F = F_values(pe, nodes, ii, iip)
                mom = F @ moment_weight(nodes, key) / np.sqrt(dp[ii] * dq[j] * dp[iip] * dq[jp])
                n_el += int(np.count_nonzero(mom)) * len(ch) ** 2
            boxes += 1
        if time.perf_counter() - t0 > budget_s:
            break
    dt = time.perf_counter() - t0
    return dict(value=n_el / dt, unit="P-elements/s", cores=1, kind="oracle",
                sample=f"oracle P0 rule (numpy, 1 thread) for the doublet lattice M=N={M}: {boxes} of {N * N} "
                       f"q-boxes ({n_el} stored elements) in {dt:.1f} s")


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import torch
    import paper_1404_5253_amd as wp

    torch.cuda.set_device(0)
    wl = workloads.WORKLOADS[WORKLOAD]
    V_R = workloads.mt_repulsion(wl["V_R_seed"])
    M, N = wl["M"], wl["N"]
    E = wl["E_lab"][0]
    lats = []
    for sysd in wl["systems"]:
        L = wp.Lattice(M, N, two_J=sysd["two_J"], j_max=sysd["j_max"], swave_only=sysd["swave"],
                       n_x=wl["n_x"], n_phi=wl["n_phi"])
        L.pseudostates(kind="mt", V_R=V_R)
        lats.append(L)
    if args.only:
        if args.only == "pw150":
            res = pw150_section(wp, torch, V_R)
        else:
            for L in lats:
                L.build_perm("fp64")
            res = (batched_energies_section(wp, torch, lats[0]) if args.only == "batched"
                   else serving_section(wp, torch, V_R, args.serve_seconds, {(M, 1, 1, True): lats[0]}))
        print(json.dumps({"section": args.only, "result": res}))
        return

    def step(times):
        for L in lats:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L.build_perm("fp64")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            sol = L.solve([E], "fp64")
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            times["build"] += t1 - t0
            times["solve"] += t2 - t1
            times["amps"].append(sol.amplitude(0)["A"][0, 0])

    for _ in range(args.warmup):
        step(dict(build=0.0, solve=0.0, amps=[]))
    times = dict(build=0.0, solve=0.0, amps=[])
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(times)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # the same K steps again with HIP events recorded around every launch (on its stream): the
    # per-kernel durations for the roofline (the events' host cost is kept out of the timing above)
    wp.wp_profile_reset()
    wp.wp_profile_enable(True)
    for _ in range(args.steps):
        step(dict(build=0.0, solve=0.0, amps=[]))
    torch.cuda.synchronize()
    wp.wp_profile_enable(False)
    prof = wp.wp_profile_read()
    K = args.steps
    elems = sum(L.perm_stats["nnz"] for L in lats)
    cand = sum(L.perm_stats["candidates"] for L in lats)
    blocks = sum(L.perm_stats["blocks"] for L in lats)
    ms_per_step = (t1 - t0) / K * 1e3
    value = elems * K / times["build"]

    # dominant kernel by total event time inside the timed region
    dom = max(prof, key=lambda k: prof[k][1])
    n_launch, tot_ms = prof[dom]
    avg_s = tot_ms / n_launch / 1e3
    nodes = wl["n_x"] * wl["n_phi"]
    if dom == "pbuild":
        work = cand / len(lats) * nodes * PBUILD_OPS_PER_NODE   # per launch (average over systems)
        roof = dict(bound="alu", achieved=work / avg_s / 1e12, peak=FP64_VALU_PEAK_TOPS, unit="Tops/s")
    elif dom == "select":
        work = N * N * nodes * M * 12 / 1.0
        roof = dict(bound="alu", achieved=work / avg_s / 1e12, peak=FP64_VALU_PEAK_TOPS, unit="Tops/s")
    elif dom == "step64":
        # two complex-by-real M x M products per column (j, channel): 2 x 4 M^2 flops
        flops = np.mean([8.0 * M * M * N * L.nch for L in lats])
        roof = dict(bound="alu", achieved=flops / avg_s / 1e12, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s")
    elif dom == "g1":
        roof = dict(bound="alu", achieved=None, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s")
    else:   # spmv64: block values + column index + row pointer + vector in/out
        byts = np.mean([L.perm_stats["bytes"] + 2 * 16 * M * N * L.nch for L in lats])
        roof = dict(bound="hbm", achieved=byts / avg_s / 1e9, peak=HBM_PEAK_GBS, unit="GB/s")
    roof["frac"] = roof["achieved"] / roof["peak"] if roof["achieved"] is not None else None
    roof["kernel"] = dom
    roof["avg_us"] = avg_s * 1e6
    roof["traffic"] = measured_traffic(WORKLOAD, dom)
    out = {
        "metric": "P-elements/s; nd solves/s + p50/p99 latency vs FP64 path at 1e-6 amp error",
        "value": value,
        "unit": "P-elements/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "M": M, "N": N, "systems": ["doublet J=1/2+ (2 ch)", "quartet J=3/2+ (1 ch)"],
                   "potential": f"MT V_R={V_R:.3f} (seed 0), V_A tuned", "E_lab": E, "nodes_per_pair": nodes,
                   "P_elements_per_step": elems, "P_blocks_per_step": blocks, "candidates_per_step": cand},
        "solves_per_s_fp64": 2 * K / times["solve"],
        "build_ms_per_step": times["build"] / K * 1e3,
        "solve_ms_per_step": times["solve"] / K * 1e3,
        "amplitudes": [f"{a.real:.12f}{a.imag:+.12f}j" for a in times["amps"][:2]],
        "kernels_ms_per_step": {k: round(v[1] / K, 4) for k, v in prof.items()},
        "roofline": roof,
    }
    if not args.no_extras:
        out["batched_64_energies"] = batched_energies_section(wp, torch, lats[0])
        out["serving"] = serving_section(wp, torch, V_R, args.serve_seconds, {(M, 1, 1, True): lats[0]})
        out["pw_mt_150"] = pw150_section(wp, torch, V_R)
    if args.sweep:
        out["swave_sweep"] = sweep_section(wp, torch, V_R)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(V_R, M, N)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
