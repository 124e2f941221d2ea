"""Benchmark of the WPCD hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-extras]

Headline workload (the 18-channel lattice, `pw_mt_150`): J = 1/2+ nd channels with pair waves
j <= 2 (18 channels, 10 pair waves), Malfliet-Tjon form in every pair wave (V_R drawn from seed 0,
V_A tuned to the deuteron, singlet 0.82 V_A), M = N = 150 tangent-mapped bins up to 10 fm^-1,
8 x 8 (x, phi) nodes per cell pair, E_lab = 3 MeV (below breakup) and 22.7 MeV (above).
Lattice tables and pseudostates are resident before timing.

One step = the whole hot path on that lattice: the P0 build (selection, quadrature, compaction;
FP64 arithmetic, FP32 storage) and one mixed-precision solve of both energies in one call (G1 in
FP64, FP32 P0, BF16 v1/O blocks on MFMA with FP32 accumulation as hi + lo pairs, FP64 residual
refinement; 2 energies x 2 open channels = 4 solves). The JSON line reports
  value        P-elements/s of the build (stored channel entries / wall time of the synchronised
               build call inside the timed region);
  ms_per_step  wall time per step (build + solve);
plus solves/s, the largest amplitude error against the oracle's values of the same lattice
(tests/golden/pw_mt_150.json), the roofline of the dominant kernel (HIP events around every
launch, inside the timed region) and the oracle timed on the host cores (cpu_baseline, run first,
before the GPU is touched). Extras: breakup elements, energy-weight packets on the same lattice,
elastic observables summed over 18 J^pi blocks,
the s-wave M = N = 100 lattice pair, 64 batched energies, the continuous-batching service, and
(--sweep) the s-wave build for M = N = 40..400.
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

WORKLOAD = "pw_mt_150"
HBM_PEAK_GBS = 8000.0
FP64_VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12   # FP64 VALU lane-ops/s (one op per lane per clock)
FP64_PEAK_TFLOPS = 78.6

# Algorithmic work per unit (measurement section)
PBUILD_OPS_PER_NODE = 14          # FP64 VALU ops per (cell pair, quadrature node)
AMP_TARGET = 1e-6                 # amplitude error at which the solve paths are compared
HEADLINE_MODE, HEADLINE_TOL = "mixed_split", 1e-8   # the headline solve: split-BF16 mixed path


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
    ap.add_argument("--no-extras", action="store_true", help="skip the s-wave, batched and serving sections")
    ap.add_argument("--serve-seconds", type=float, default=30.0, help="measured length of the serving stream")
    ap.add_argument("--serve-warmup", type=float, default=5.0, help="warm-up length of the serving stream")
    ap.add_argument("--sweep", action="store_true", help="also time the s-wave P0 build for M = N in 40..400")
    ap.add_argument("--only", choices=["batched", "serving", "swave", "sweep", "energy", "jsum"], default=None,
                    help="run only this extra section (no headline step); for profiling runs")
    return ap.parse_args()


def batched_energies_section(wp, torch, L, reps=3):
    """64 energies U[1, 50] MeV (seed 1234) on the resident doublet lattice.

    FP64 path to its rounding floor, then every path at 1e-6 amplitude error: each path's
    tolerance (and Arnoldi cycle length) is chosen by the autotuner on a separate calibration
    draw of 64 energies (seed 4321) against the converged FP64 amplitudes, then timed on the
    bench energies, where the error against the converged FP64 amplitudes is reported."""
    from paper_1404_5253_amd.tune import LAUNCH_DEFAULTS, solve_amplitudes, tune
    Es = workloads.batched_energies()
    Ecal = workloads.batched_energies(seed=4321)
    best, _ = tune(L, Ecal, target=AMP_TARGET, sync=torch.cuda.synchronize)
    out = {"autotuned": {k: {kk: (float(vv) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                         for k, v in best.items()}}
    amps = {}
    runs = [("fp64", "fp64", dict(LAUNCH_DEFAULTS, tol=1e-12, refine_every=0))] + \
           [(f"{m}_at_1e-6", m, v) for m, v in best.items()]
    for label, mode, cfg in runs:
        launch = {k: cfg[k] for k in ("graph", "step_tile", "spmm_cols")}
        run = lambda it=False: solve_amplitudes(L, Es, mode, cfg["tol"], cfg["refine_every"], cfg["width"], iters=it,
                                                **launch)
        run()   # warm-up (and graph capture)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            A, it = run(True)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        # kernel breakdown from one more pass with events around every launch (launched, not replayed)
        wp.wp_profile_reset()
        wp.wp_profile_enable(True)
        run()
        torch.cuda.synchronize()
        wp.wp_profile_enable(False)
        out[f"kernels_ms_per_batch_{label}"] = {k: round(v[1], 3) for k, v in wp.wp_profile_read().items()}
        out[f"iters_{label}"] = int(it)
        amps[label] = A[:, 0]
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
SERVING_BUDGET = 12 << 30   # one device-memory budget for all serving batches
SERVING_MODES = (("fp64", dict(tol=3e-7, accept=1e-7, refine_every=0)),
                 ("mixed_split", dict(tol=3e-6, accept=3e-6, refine_every=8)))


def serving_section(wp, torch, V_R, seconds, warmup, lats_by_key=None, n_check=200):
    """Poisson stream (200 req/s, seed 2026; `warmup` s served but not counted, then `seconds` s
    measured) over four resident lattices, continuous batching, once with FP64 batches and once
    with split-BF16 mixed batches, each at a stop tolerance that keeps the amplitude error below
    1e-6; afterwards a seeded sample of n_check served amplitudes per mode is compared with a
    converged FP64 solve of the same energy (outside the timing). Every request must be served."""
    from paper_1404_5253_amd.serve import BatchBackend, divide_budget, run_stream, slot_bytes
    lats = []
    for (M, two_J, j_max, sw) in SERVING_LATTICES:
        L = (lats_by_key or {}).get((M, two_J, j_max, sw))
        if L is None:
            L = wp.Lattice(M, M, two_J=two_J, j_max=j_max, swave_only=sw)
            L.pseudostates(kind="mt", V_R=V_R)
            L.build_perm("fp64")
        lats.append(L)
    reqs = workloads.serving_requests(len(lats), rate=200.0, duration=warmup + seconds)
    # saturation: the same kind of stream at 10x the rate, so that solves/s is the service rate
    sat = workloads.serving_requests(len(lats), rate=2000.0, duration=1.0, seed=7)
    out = {"lattices": [f"M=N={M}, {L.nch} ch" for (M, *_), L in zip(SERVING_LATTICES, lats)], "requests": len(reqs),
           "budget_GB": SERVING_BUDGET / 2**30,
           "warmup_s": warmup, "measured_s": seconds, "saturation_requests": len(sat),
           "P0_bytes": [L.perm_stats["bytes"] for L in lats]}
    served = {}

    def backends(mode, kw):
        # one device-memory budget for the four lattices' batches, divided by request share
        sb = [slot_bytes(L, mode, kw.get("refine_every", 0)) for L in lats]
        slots = divide_budget(SERVING_BUDGET, sb, [1.0] * len(lats), max_slots=32)
        out[f"slots_{mode}"] = slots
        out[f"slot_MB_{mode}"] = [round(b / 2**20, 1) for b in sb]
        out_ = []
        for L, k, b_ in zip(lats, slots, sb):
            st = torch.cuda.Stream()
            b = BatchBackend(L, slots=k, hbm_budget=k * b_, terms=8, stream=wp.C.c_void_p(st.cuda_stream),
                             mode=mode, max_iter=400, **kw)
            b._torch_stream = st
            out_.append(b)
        return out_

    for mode, kw in SERVING_MODES:
        backs = backends(mode, kw)
        done, sstats = run_stream(backs, sat)
        for b in backs:
            b.close()
        assert sstats["n_served"] == len(sat), (mode, sstats["n_served"], len(sat))
        out[f"saturated_{mode}"] = {k: sstats[k] for k in ("n", "p50_ms", "p99_ms", "solves_per_s", "wall_s")}
        backs = backends(mode, kw)
        done, stats = run_stream(backs, reqs, measure_from=warmup)
        for b in backs:
            b.close()
        assert stats["n_served"] == len(reqs), (mode, stats["n_served"], len(reqs))
        stats["accepted"] = sum(1 for r in done if r.result.get("accepted", True))
        out[mode] = stats
        served[mode] = {r.rid: (r.lattice, r.E_lab, r.result["A"]) for r in done}
    # accuracy of a seeded sample of served amplitudes against converged FP64 solves
    for mode in served:
        rids = sorted(served[mode])
        pick = set(np.random.default_rng(3).choice(rids, min(n_check, len(rids)), replace=False).tolist())
        worst = [0.0] * len(lats)
        for li, L in enumerate(lats):
            items = [(E, A) for rid, (l, E, A) in served[mode].items() if l == li and rid in pick]
            for k0 in range(0, len(items), 64):
                chunk = items[k0:k0 + 64]
                ref = L.solve([E for E, _ in chunk], "fp64", tol=1e-12, max_iter=400, accept=1e-6)
                for k, (_, A) in enumerate(chunk):
                    worst[li] = max(worst[li], float(np.max(np.abs(A - ref.amplitude(k)["A"]))))
        out[mode]["max_abs_dA_vs_converged_fp64"] = max(worst)
        out[mode]["max_abs_dA_per_lattice"] = worst
        out[mode]["checked"] = len(pick)
    out["speedup_mixed_split_over_fp64_solves_per_s"] = out["mixed_split"]["solves_per_s"] / out["fp64"]["solves_per_s"]
    out["speedup_mixed_split_over_fp64_saturated"] = (out["saturated_mixed_split"]["solves_per_s"]
                                                      / out["saturated_fp64"]["solves_per_s"])
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


def breakup_section(wp, torch, L, Es, reps=5):
    """Breakup transition elements of the headline solve (the same U projected onto every
    energy-shell cell of the three-body continuum): cells per energy and the cost of the
    projections on top of the solve."""
    def run(bu):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            sol = L.solve(Es, HEADLINE_MODE, tol=HEADLINE_TOL, breakup=bu)
        torch.cuda.synchronize()
        return sol, (time.perf_counter() - t0) / reps
    run(True)
    _, t_plain = run(False)
    sol, t_bu = run(True)
    wp.wp_profile_reset()
    wp.wp_profile_enable(True)
    L.solve(Es, HEADLINE_MODE, tol=HEADLINE_TOL, breakup=True)
    torch.cuda.synchronize()
    wp.wp_profile_enable(False)
    prof = wp.wp_profile_read()
    cells = [int(sol.breakup(k, 0)[0].shape[0]) for k in range(len(Es))]
    return dict(E_lab=list(Es), cells_per_energy=cells, solve_ms=t_plain * 1e3, solve_ms_with_breakup=t_bu * 1e3,
                projection_kernel_ms=round(prof.get("breakup", (0, 0.0))[1], 4),
                max_abs_element=[float(np.max(np.abs(sol.breakup(k, 0)[1]), initial=0.0)) for k in range(len(Es))])


def energy_weights_section(wp, torch, V_R, Es, unit_lat, unit_g1_ms, reps=3):
    """Energy-weight packets (weights ~ sqrt(p), sqrt(q); closed-form G1) on the headline lattice:
    one step (build + the headline solve) against the unit-weight step, the G1 launch of each,
    and both weightings' amplitudes. Then the quartet s-wave phase (Yamaguchi, 1 and 3 MeV) of
    both weightings as the lattice grows: the result is independent of the partition only in the
    limit, and how fast each weighting gets there is the accuracy comparison."""
    wl = workloads.WORKLOADS[WORKLOAD]
    sysd = wl["systems"][0]
    L = wp.Lattice(wl["M"], wl["N"], two_J=sysd["two_J"], j_max=sysd["j_max"], swave_only=sysd["swave"],
                   n_x=wl["n_x"], n_phi=wl["n_phi"], weights="energy")
    L.pseudostates(kind="mt", V_R=V_R)

    def step(acc):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.build_perm("fp32")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sol = L.solve(Es, HEADLINE_MODE, tol=HEADLINE_TOL)
        torch.cuda.synchronize()
        acc["build"] += t1 - t0
        acc["solve"] += time.perf_counter() - t1
        acc["sol"] = sol
    step(dict(build=0.0, solve=0.0))
    acc = dict(build=0.0, solve=0.0)
    for _ in range(reps):
        step(acc)
    wp.wp_profile_reset()
    wp.wp_profile_enable(True)
    step(dict(build=0.0, solve=0.0))
    torch.cuda.synchronize()
    wp.wp_profile_enable(False)
    prof = wp.wp_profile_read()
    unit = unit_lat.solve(Es, HEADLINE_MODE, tol=HEADLINE_TOL)
    amps = {}
    for k, E in enumerate(Es):
        Ae, Au = acc["sol"].amplitude(k), unit.amplitude(k)
        amps[str(E)] = dict(delta_deg_energy=[float(x) for x in Ae["delta"]],
                            delta_deg_unit=[float(x) for x in Au["delta"]],
                            max_abs_dA_energy_vs_unit=float(np.max(np.abs(Ae["A"] - Au["A"]))))
    conv = []
    for Mq in (24, 48, 64, 100, 150):
        row = dict(M=Mq)
        for w in ("unit", "energy"):
            Lq = wp.Lattice(Mq, Mq, two_J=3, weights=w)
            Lq.pseudostates(kind="yamaguchi")
            Lq.build_perm("fp64")
            sq = Lq.solve([1.0, 3.0], "fp64", accept=1e-6)
            row[w] = [float(sq.amplitude(k)["delta"][0]) for k in range(2)]
        conv.append(row)
    return dict(step_ms_build=acc["build"] / reps * 1e3, step_ms_solve=acc["solve"] / reps * 1e3,
                P_elements=L.perm_stats["nnz"], P_elements_per_s=L.perm_stats["nnz"] * reps / acc["build"],
                g1_ms_per_call_energy=round(prof.get("g1", (1, 0.0))[1] / max(1, prof.get("g1", (1, 0.0))[0]), 4),
                g1_ms_per_call_unit=unit_g1_ms, kernels_ms_per_step={k: round(v[1], 4) for k, v in prof.items()},
                amplitudes=amps, quartet_phase_deg_1_and_3_MeV_vs_M=conv)


def jsum_section(wp, torch, V_R, M=100, two_J_max=17):
    """Elastic nd observables over J^pi blocks (Sec. IV): every block 2J = 1 .. two_J_max of both
    parities is a lattice of its own (pair waves j <= 1, 10-14 channels, M = N = 100, MT), built
    and solved in FP64 at 13 and 35 MeV; dsigma/dOmega and A_y from the blocks' elastic S. Then the
    channel-spin eigenphases of the J = 1/2+ and 3/2+ blocks at 3 MeV (below breakup)."""
    from paper_1404_5253_amd.jsum import JBlocks
    blocks = [(tJ, p) for tJ in range(1, two_J_max + 1, 2) for p in (1, -1)]
    Es = [13.0, 35.0]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    jb = JBlocks(blocks, M, M, j_max=1, kind="mt", V_R=V_R)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per_E, q0 = jb.solve(Es, "fp64", accept=1e-6)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    th_deg = np.array([10.0, 30.0, 60.0, 90.0, 120.0, 150.0, 170.0])
    obs = {}
    t3 = time.perf_counter()
    for e, E in enumerate(Es):
        ds, ay = wp.nd_elastic_observables(per_E[e], q0[e], np.radians(th_deg))
        obs[str(E)] = dict(theta_deg=th_deg.tolist(), dsigma_dOmega_mb_sr=(10.0 * ds).tolist(), A_y=ay.tolist())
    t4 = time.perf_counter()
    low = JBlocks([(1, 1), (3, 1)], M, M, j_max=1, kind="mt", V_R=V_R)
    lowE, _ = low.solve([3.0], "fp64", accept=1e-6)
    eig = {}
    for two_J, chans, S in lowE[0]:
        sig, Ss = wp.nd_sigma_rep(two_J, chans, S)
        d, _ = wp.nd_eigenphases(Ss)
        eig[f"{two_J}/2+"] = dict(channels_lam_2Sigma=sig, eigenphases_deg=np.degrees(d).tolist())
    n_ch = [L.nch for _, L in jb.lats]
    return dict(blocks=len(blocks), M=M, N=M, j_max=1, channels_per_block=n_ch, E_lab=Es,
                build_s=t1 - t0, solve_s=t2 - t1, solves=len(blocks) * len(Es),
                solves_per_s=len(blocks) * len(Es) / (t2 - t1), observables_host_ms=(t4 - t3) * 1e3,
                observables=obs, eigenphases_3MeV=eig)


def swave_section(wp, torch, V_R, reps=10):
    """The s-wave Malfliet-Tjon lattice pair at M = N = 100 (doublet J = 1/2+, 2 channels, and
    quartet J = 3/2+, 1 channel; V_R seed 0): P0 build in FP64 and one FP64 solve at 14.1 MeV each,
    per step."""
    wl = workloads.WORKLOADS["swave_mt_100"]
    M, N = wl["M"], wl["N"]
    E = wl["E_lab"][0]
    lats = []
    for sysd in wl["systems"]:
        L = wp.Lattice(M, N, two_J=sysd["two_J"], j_max=sysd["j_max"], swave_only=sysd["swave"],
                       n_x=wl["n_x"], n_phi=wl["n_phi"])
        L.pseudostates(kind="mt", V_R=V_R)
        lats.append(L)
    times = dict(build=0.0, solve=0.0)

    def step(acc):
        for L in lats:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            L.build_perm("fp64")
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            L.solve([E], "fp64")
            torch.cuda.synchronize()
            acc["build"] += t1 - t0
            acc["solve"] += time.perf_counter() - t1

    step(dict(build=0.0, solve=0.0))
    t0 = time.perf_counter()
    for _ in range(reps):
        step(times)
    dt = (time.perf_counter() - t0) / reps
    wp.wp_profile_reset()
    wp.wp_profile_enable(True)
    step(dict(build=0.0, solve=0.0))
    torch.cuda.synchronize()
    wp.wp_profile_enable(False)
    prof = wp.wp_profile_read()
    # the single-energy FP64 solves again, launched and replayed from HIP graphs (term chunks)
    graph_cmp = {}
    for g in (False, True):
        for L in lats:
            L.solve([E], "fp64", graph=g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            for L in lats:
                L.solve([E], "fp64", graph=g)
        torch.cuda.synchronize()
        graph_cmp["graph" if g else "launched"] = 2 * reps / (time.perf_counter() - t0)
    elems = sum(L.perm_stats["nnz"] for L in lats)
    return dict(M=M, N=N, E_lab=E, systems=["doublet J=1/2+ (2 ch)", "quartet J=3/2+ (1 ch)"],
                solves_per_s_fp64_launched_vs_graph=graph_cmp,
                P_elements=elems, P_elements_per_s=elems * reps / times["build"], ms_per_step=dt * 1e3,
                build_ms_per_step=times["build"] / reps * 1e3, solve_ms_per_step=times["solve"] / reps * 1e3,
                solves_per_s_fp64=2 * reps / times["solve"],
                kernels_ms_per_step={k: round(v[1], 4) for k, v in prof.items()}), lats


# ---------------------------------------------------------------- oracle timed on the host

def _oracle_p0_rows(task):
    """Worker: the oracle's P0 rule for every q-box (j, j') of the rows j given, contracted with the
    coefficient table; returns (stored entries, stored blocks) of those rows."""
    from threadpoolctl import threadpool_limits
    from oracle.perm import box_nodes, candidate_pairs, F_values, moment_weight
    rows, pe, qe, keys, C, n_x, n_phi = task
    with threadpool_limits(1):   # one process per core
        return _oracle_p0_rows_1(rows, pe, qe, keys, C, n_x, n_phi)


def _oracle_p0_rows_1(rows, pe, qe, keys, C, n_x, n_phi):
    from oracle.perm import box_nodes, candidate_pairs, F_values, moment_weight
    dp, dq = np.diff(pe), np.diff(qe)
    entries = blocks = 0
    for j in rows:
        for jp in range(len(qe) - 1):
            nodes = box_nodes(qe, j, jp, n_x, n_phi)
            ii, iip = candidate_pairs(pe, nodes)
            if not len(ii):
                continue
            F = F_values(pe, nodes, ii, iip)
            Wm = np.stack([moment_weight(nodes, key) for key in keys], axis=1)
            mom = (F @ Wm) / np.sqrt(dp[ii] * dq[j] * dp[iip] * dq[jp])[:, None]
            mom = mom[np.any(mom != 0.0, axis=1)]
            vals = np.einsum("abm,nm->nab", C, mom)
            entries += int(np.count_nonzero(vals))
            blocks += len(mom)
    return entries, blocks


def cpu_baseline(budget_s=12.0):
    """The oracle as it stands on the host cores, on bounded samples of the headline workload:
    P0 rows (q bins j in a fixed shuffled order, one process per core, until budget_s of wall time
    has passed or every row is done), a sample of G1 elements, and per-stage times. Runs before the
    GPU is touched (the worker processes are forked)."""
    import multiprocessing as mp
    import platform
    from oracle import lattice as olat, pipeline, potential, pseudostates, recoupling, resolvent
    from oracle.perm import channel_terms
    wl = workloads.WORKLOADS[WORKLOAD]
    sysd = wl["systems"][0]
    V_R = workloads.mt_repulsion(wl["V_R_seed"])
    M, N = wl["M"], wl["N"]
    spec = pipeline.Spec(M=M, N=N, two_J=sysd["two_J"], j_max=sysd["j_max"], swave_only=sysd["swave"], pot="mt",
                         V_R=V_R, n_x=wl["n_x"], n_phi=wl["n_phi"])
    stages = {}
    t0 = time.perf_counter()
    pe, qe = olat.tangent_edges(M), olat.tangent_edges(N)
    chans = pipeline.channel_list(spec)
    gt = {(a, b): recoupling.g_table(chans[a], chans[b], spec.two_J) for a in range(len(chans))
          for b in range(len(chans))}
    keys, C = channel_terms(chans, gt)
    stages["lattice_channels_coefficients_s"] = time.perf_counter() - t0
    t0 = time.perf_counter()
    strength = potential.tune_mt(pe, V_R, spec.mu_R, spec.mu_A, spec.target_BE)
    waves = {}
    for c in chans:
        if (c[0], c[1]) not in waves:
            v = pipeline.pair_potential(spec, pe, c[0], c[1], strength)
            eps, O = pseudostates.diagonalize(pe, v)
            nb = int(np.sum(eps < 0))
            waves[(c[0], c[1])] = (eps, nb, pseudostates.scattering_bins(eps[nb:]))
    stages["pseudostates_s"] = time.perf_counter() - t0
    eps0 = float(waves[(0, 1)][0][0])
    # P0: rows in a fixed shuffled order, all cores
    cores = max(1, min(16, os.cpu_count() or 1))
    order = list(np.random.default_rng(0).permutation(N))
    ctx = mp.get_context("fork")
    entries = blocks = done = 0
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        while done < N and time.perf_counter() - t0 < budget_s:
            batch = order[done:done + cores]
            tasks = [([j], pe, qe, keys, C, spec.n_x, spec.n_phi) for j in batch]
            for e, b in pool.map(_oracle_p0_rows, tasks):
                entries += e
                blocks += b
            done += len(batch)
    t_p0 = time.perf_counter() - t0
    stages["P0_rows_sampled"] = done
    stages["P0_sample_s"] = t_p0
    stages["P0_full_lattice_estimate_s"] = t_p0 * N / done
    # G1: a seeded sample of continuum elements of every pair wave at 22.7 MeV, one core
    E = olat.total_energy(wl["E_lab"][1], eps0)
    rng = np.random.default_rng(1)
    t0 = time.perf_counter()
    n_el = 0
    for key, (eps, nb, bins) in waves.items():
        for _ in range(20):
            k, j = int(rng.integers(0, len(bins) - 1)), int(rng.integers(0, N))
            resolvent.continuum_element(bins[k], bins[k + 1], qe[j], qe[j + 1], E)
            n_el += 1
    t_g1 = time.perf_counter() - t0
    stages["G1_elements_per_s_1core"] = n_el / t_g1
    stages["G1_one_energy_estimate_s_1core"] = len(waves) * M * N / (n_el / t_g1)
    # a whole oracle solve where it finishes in seconds: the quartet Yamaguchi lattice M = N = 40
    t0 = time.perf_counter()
    s1 = pipeline.build_system(pipeline.Spec(M=40, N=40, two_J=3, pot="yamaguchi"))
    t1 = time.perf_counter()
    pipeline.solve_energy(s1, 10.0)
    t2 = time.perf_counter()
    stages["oracle_quartet_40"] = dict(build_s=t1 - t0, solve_s=t2 - t1, solves_per_s=1.0 / (t2 - t1))
    try:
        model = next((ln.split(":", 1)[1].strip() for ln in open("/proc/cpuinfo") if ln.startswith("model name")),
                     platform.processor())
    except OSError:
        model = platform.processor()
    return dict(value=entries / t_p0, unit="P-elements/s", cores=cores, kind="oracle",
                sample=f"oracle P0 rule (numpy) for the 18-channel lattice M=N={M}: {done} of {N} q-bin rows "
                       f"({blocks} blocks, {entries} stored entries) in {t_p0:.1f} s on {cores} processes; "
                       f"host {model}, os.cpu_count()={os.cpu_count()}, "
                       f"OPENBLAS_NUM_THREADS={os.environ.get('OPENBLAS_NUM_THREADS', 'unset')}",
                stages=stages)


def roofline(label, avg_s, L, B, nodes):
    """Algorithmic work of one launch of the kernel behind `label` over its average duration,
    against the peak of the resource that bounds it (the per-unit figures are in the design doc)."""
    st = L.perm_stats
    M, N, nch = L.M, L.N, L.nch
    R = M * N
    D = R * nch
    idx = st["blocks"] * 4 + (R + 1) * 8          # block column indices and row pointer
    if label in ("spmv_f32", "spmm_arnoldi"):      # FP32 P0, complex FP32 vectors in and out
        byts = st["nnz"] * 4 + idx + 2 * D * B * 8
    elif label == "spmv_f32v_f64x":                # FP32 P0, complex FP64 vectors
        byts = st["nnz"] * 4 + idx + 2 * D * B * 16
    elif label == "spmv64":                        # FP64 P0, complex FP64 vectors
        byts = st["nnz"] * 8 + idx + 2 * D * B * 16
    else:
        byts = None
    if byts is not None:
        return dict(bound="hbm", achieved=byts / avg_s / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                    bytes_per_launch=byts)
    if label == "step64":                          # two complex-by-real M x M products per column
        flops = 8.0 * M * M * N * nch * B
        return dict(bound="alu", achieved=flops / avg_s / 1e12, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    flops_per_launch=flops)
    if label == "pbuild_fused":                    # FP64 MFMA: moments of the kept pairs at every node
        flops = 2.0 * st["blocks"] * nodes * L.nmom
        return dict(bound="mfma", achieved=flops / avg_s / 1e12, peak=FP64_PEAK_TFLOPS, unit="TFLOP/s",
                    flops_per_launch=flops)
    if label in ("pbuild", "pbuild_mom"):          # FP64 VALU ops over the candidates' nodes
        nmom = getattr(L, "nmom", None)
        ops = st["candidates"] * nodes * (PBUILD_OPS_PER_NODE + 2 * (nmom or 1))
        return dict(bound="alu", achieved=ops / avg_s / 1e12, peak=FP64_VALU_PEAK_TOPS, unit="Tops/s",
                    ops_per_launch=ops)
    if label == "combine":                         # candidate values written once (FP64)
        byts = st["candidates"] * (nch * nch * 8 + 1)
        return dict(bound="hbm", achieved=byts / avg_s / 1e9, peak=HBM_PEAK_GBS, unit="GB/s",
                    bytes_per_launch=byts)
    return dict(bound="alu", achieved=None, peak=None, unit=None)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    # the oracle first, in forked worker processes, before anything touches the GPU
    cpu = None if (args.no_cpu_baseline or args.only) else cpu_baseline()
    import torch
    import paper_1404_5253_amd as wp

    torch.cuda.set_device(0)
    V_R = workloads.mt_repulsion(0)
    if args.only:
        if args.only == "swave":
            res, _ = swave_section(wp, torch, V_R)
        elif args.only == "sweep":
            res = sweep_section(wp, torch, V_R)
        elif args.only == "jsum":
            res = jsum_section(wp, torch, V_R)
        elif args.only == "energy":
            wl = workloads.WORKLOADS[WORKLOAD]
            sysd = wl["systems"][0]
            L = wp.Lattice(wl["M"], wl["N"], two_J=sysd["two_J"], j_max=sysd["j_max"], swave_only=sysd["swave"],
                           n_x=wl["n_x"], n_phi=wl["n_phi"])
            L.pseudostates(kind="mt", V_R=V_R)
            L.build_perm("fp32")
            Es = list(wl["E_lab"])
            L.solve(Es, HEADLINE_MODE, tol=HEADLINE_TOL)
            wp.wp_profile_reset()
            wp.wp_profile_enable(True)
            L.solve(Es, HEADLINE_MODE, tol=HEADLINE_TOL)
            torch.cuda.synchronize()
            wp.wp_profile_enable(False)
            g1u = wp.wp_profile_read().get("g1", (1, 0.0))
            res = energy_weights_section(wp, torch, V_R, Es, L, round(g1u[1] / max(1, g1u[0]), 4))
        else:
            L = wp.Lattice(100, 100, two_J=1)
            L.pseudostates(kind="mt", V_R=V_R)
            L.build_perm("fp64")
            res = (batched_energies_section(wp, torch, L) if args.only == "batched"
                   else serving_section(wp, torch, V_R, args.serve_seconds, args.serve_warmup,
                                        {(100, 1, 1, True): L}))
        print(json.dumps({"section": args.only, "result": res}))
        return

    wl = workloads.WORKLOADS[WORKLOAD]
    sysd = wl["systems"][0]
    M, N = wl["M"], wl["N"]
    Es = list(wl["E_lab"])
    nodes = wl["n_x"] * wl["n_phi"]
    L = wp.Lattice(M, N, two_J=sysd["two_J"], j_max=sysd["j_max"], swave_only=sysd["swave"], n_x=wl["n_x"],
                   n_phi=wl["n_phi"])
    L.pseudostates(kind="mt", V_R=V_R)
    B = len(Es) * 2                               # columns: energies x open channels

    def step(acc):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        L.build_perm("fp32")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sol = L.solve(Es, HEADLINE_MODE, tol=HEADLINE_TOL)
        torch.cuda.synchronize()
        acc["build"] += t1 - t0
        acc["solve"] += time.perf_counter() - t1
        acc["sol"] = sol

    for _ in range(args.warmup):
        step(dict(build=0.0, solve=0.0))
    times = dict(build=0.0, solve=0.0)
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
        step(dict(build=0.0, solve=0.0))
    torch.cuda.synchronize()
    wp.wp_profile_enable(False)
    prof = wp.wp_profile_read()
    K = args.steps
    st = L.perm_stats
    ms_per_step = (t1 - t0) / K * 1e3
    value = st["nnz"] * K / times["build"]
    # amplitudes against the oracle's values of the same lattice
    with open(os.path.join(ROOT, "tests", "golden", "pw_mt_150.json")) as f:
        gold = json.load(f)
    dA = 0.0
    for k, E in enumerate(Es):
        g = gold["results"][str(E)]
        Ar = np.array(g["A_re"]) + 1j * np.array(g["A_im"])
        dA = max(dA, float(np.max(np.abs(times["sol"].amplitude(k)["A"] - Ar))))
    dom = max(prof, key=lambda k: prof[k][1])
    n_launch, tot_ms = prof[dom]
    avg_s = tot_ms / n_launch / 1e3
    roof = roofline(dom, avg_s, L, B, nodes)
    roof["frac"] = roof["achieved"] / roof["peak"] if roof.get("achieved") is not None else None
    roof["kernel"] = dom
    roof["avg_us"] = avg_s * 1e6
    roof["launches_per_step"] = n_launch / K
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
        "config": {"workload": WORKLOAD, "M": M, "N": N, "channels": L.nch, "J": "1/2+", "j_max": sysd["j_max"],
                   "potential": f"MT V_R={V_R:.3f} (seed 0), V_A tuned", "E_lab": Es, "nodes_per_pair": nodes,
                   "P0_storage": "f32 (computed in f64)",
                   "solve": f"{HEADLINE_MODE} (bf16 hi+lo MFMA, fp32 P0 and vectors, fp64 G1 and refinement), "
                            f"tol {HEADLINE_TOL}",
                   "P_elements_per_step": st["nnz"], "P_blocks_per_step": st["blocks"],
                   "candidates_per_step": st["candidates"], "P0_bytes": st["bytes"]},
        "solves_per_s": B * K / times["solve"],
        "build_ms_per_step": times["build"] / K * 1e3,
        "solve_ms_per_step": times["solve"] / K * 1e3,
        "max_abs_dA_vs_oracle": dA,
        "kernels_ms_per_step": {k: round(v[1] / K, 4) for k, v in prof.items()},
        "launches_per_step": {k: v[0] // K for k, v in prof.items()},
        "roofline": roof,
    }
    if not args.no_extras:
        out["breakup"] = breakup_section(wp, torch, L, Es)
        g1u = prof.get("g1", (1, 0.0))
        out["energy_weights"] = energy_weights_section(wp, torch, V_R, Es, L, round(g1u[1] / max(1, g1u[0]), 4))
        out["jsum_observables"] = jsum_section(wp, torch, V_R)
        sw, sw_lats = swave_section(wp, torch, V_R)
        out["swave_mt_100"] = sw
        out["batched_64_energies"] = batched_energies_section(wp, torch, sw_lats[0])
        out["serving"] = serving_section(wp, torch, V_R, args.serve_seconds, args.serve_warmup,
                                         {(100, 1, 1, True): sw_lats[0]})
    if args.sweep:
        out["swave_sweep"] = sweep_section(wp, torch, V_R)
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
