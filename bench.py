"""Benchmark: RRMHD+M1 zone-updates/s of the FP64 hot path on one MI355X.

Workload: the 2D magnetised cylindrical blast, 512 x 512 cells, periodic,
seeded 1 % density perturbation, oblique B = 0.5, overpressure 1e3 inside
r < 0.1, opacity field from kappa dx ~ 3e-3 to ~1e2, PVM-int-8, PLM MinMod,
IMEX RK2, CFL 0.4, 200 steps. A step is one full pass of the hot path: the
CFL signal-speed reduction (one device->host value) and one IMEX step (two
stages of cell recovery, face fluxes in both directions, flux divergence and
implicit source solve). The state is resident in HBM before timing starts.

  python bench.py [--gpus 1] [--steps 200] [--warmup 5] [--no-cpu-baseline]

Prints ONE JSON line. Zone-update: one interior cell advanced by one full IMEX
step. `roofline` covers the dominant kernel (the face-flux kernel): achieved
algorithmic FLOP/s = measured per-face operation count x faces per launch /
mean launch time (HIP events on the library's stream during the timed
region), against the FP64 vector peak.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector (256 CUs, 2.4 GHz, 128 flop/clk/CU with FMA)
HBM_PEAK_GBS = 8000.0
METRIC = "RRMHD+M1 zone-updates/s FP64 vs mixed; p50/p99 serve latency"


KERNEL_SOURCES = ("paper_2212_00370_amd/csrc/rrmhd_api.hip", "paper_2212_00370_amd/csrc/rrmhd_device.hpp",
                  "include/rrmhd.h")


def kernel_sources_digest() -> str:
    """SHA-256 over the sources the kernels are built from. HBM counters
    stored under profiles/ carry the digest of the sources they were taken
    with; a mismatch means the kernels changed since and the stored traffic
    no longer describes them."""
    import hashlib
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def load_json(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return None


def op_counts(path, steps):
    """Algorithmic operation counts of the oracle (oracle/count_ops.py),
    averaged over the timed steps: the per-step counts of the snapshots that
    lie within them, integrated by the trapezoid rule over the snapshot steps
    (one snapshot: its counts; none: all of them). The per-cell work grows as
    the blast develops, so a short run is measured against its own steps."""
    d = load_json(path)
    if not d:
        return None
    snaps = sorted([r for r in d["snapshots"] if r["step"] <= steps] or d["snapshots"], key=lambda r: r["step"])

    def mean(k):
        if len(snaps) == 1 or snaps[-1]["step"] == snaps[0]["step"]:
            return sum(r[k] for r in snaps) / len(snaps)
        area = sum(0.5 * (a[k] + b[k]) * (b["step"] - a["step"]) for a, b in zip(snaps, snaps[1:]))
        return area / (snaps[-1]["step"] - snaps[0]["step"])
    res = {"faces_ops_per_face": mean("faces_ops_per_face"), "prims_ops_per_cell": mean("prims_ops_per_cell"),
           "implicit_ops_per_cell": mean("implicit_ops_per_cell"),
           "divergence_ops_per_cell": d["divergence_ops_per_cell"], "snapshot_steps": [r["step"] for r in snaps]}
    if all("implicit_newton_ops_per_cell" in r for r in snaps):
        res["implicit_newton_ops_per_cell"] = mean("implicit_newton_ops_per_cell")
    return res


def cpu_baseline(P, steps: int, solver: int = 0, compare=None):
    """The CPU oracle (as it stands, OpenMP over cells) on the first `steps`
    steps of the same workload from the same initial state. compare:
    (k, U_gpu): the GPU state after k steps (k <= steps), checked against the
    oracle's state after k steps (same time-step rule, so the same dt)."""
    import numpy as np
    from oracle import oracle as O
    nthreads = O.threads(0)
    par = O.params(gamma=P.gamma, a_rad=P.a_rad, beta_mode=1, solver=solver)
    g = O.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    U = O.p2c(P.V, par)
    check = None
    t0 = time.perf_counter()
    for k in range(steps):
        s, _ = O.max_speed(g, U, par)
        dt = P.cfl * min(P.dx) / s
        U, st, rep = O.step(g, U, dt, P.kappa, P.sigma, par)
        if compare is not None and k + 1 == compare[0]:
            c0 = time.perf_counter()
            Ug = compare[1]
            scale = np.maximum(np.abs(U), 1e-3 * np.abs(U).max(axis=1, keepdims=True))
            scale[scale == 0] = 1.0
            check = {"step": k + 1, "bitwise": bool(np.array_equal(Ug, U)),
                     "max_rel_err": float(np.max(np.abs(Ug - U) / scale))}
            t0 += time.perf_counter() - c0
    el = time.perf_counter() - t0
    out = dict(value=P.ncell * steps / el, unit="zone-updates/s", cores=nthreads, kind="oracle",
               sample=f"first {steps} steps of the same {P.shape[0]}x{P.shape[1]} blast "
                      f"(CFL signal speed + IMEX step), {el:.1f} s")
    return out, check


def log(msg):
    """Progress of a long leg, on stderr (the JSON line is the only stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def serving_run(mix, loads, seed, seq_sample, budget_frac=0.5, label="serving"):
    """Continuous batching of independent problems (serving.Server: light
    and heavy size classes on their own streams, batched launches, time steps
    formed on the device, admission by HBM footprint).
    Capacity is measured first with every request present at t = 0; each timed
    run then draws Poisson arrivals at load x capacity. The comparison runs the
    first `seq_sample` requests one at a time in FP64 through rrmhd_max_speed +
    rrmhd_step (the single-simulation entry points)."""
    import numpy as np
    import torch
    from paper_2212_00370_amd import inputs as I
    from paper_2212_00370_amd import rrmhd as R
    from paper_2212_00370_amd import serving as S

    def reqs(arrivals, subset=None):
        idx = range(len(mix)) if subset is None else subset
        return [S.Request(rid=i, problem=mix[i]["problem"], precision=R.MIXED if mix[i]["mixed"] else R.FP64,
                          t_end=mix[i]["t_end"], steps=mix[i]["steps"], arrival=float(a))
                for i, a in zip(idx, arrivals)]
    free, total = torch.cuda.mem_get_info()
    budget = int(budget_frac * free)
    srv = S.Server(budget, max_sims=256)
    t0 = time.perf_counter()
    res0 = srv.run(reqs(np.zeros(len(mix))))
    cap_s = time.perf_counter() - t0
    srv.close()
    zu = sum(r.zone_updates for r in res0)
    mu = len(mix) / cap_s
    fails = sum(1 for r in res0 if r.report.get("imp_fail", 0) or r.report.get("c2p_fail", 0))
    by_kind = {}
    for r in res0:
        m = mix[r.rid]
        kind = f"{m['problem'].ndim}d_{'mixed' if m['mixed'] else 'fp64'}"
        e = by_kind.setdefault(kind, {"requests": 0, "with_counted_failures": 0})
        e["requests"] += 1
        e["with_counted_failures"] += int(bool(r.report.get("imp_fail", 0) or r.report.get("c2p_fail", 0)))
    log(f"{label}: capacity run, {len(mix)} requests in {cap_s:.1f} s")
    runs = []
    for li, load in enumerate(loads):
        rate = load * mu
        arr = I.poisson_arrivals(seed + 1 + li, len(mix), rate)
        srv = S.Server(budget, max_sims=256)
        t0 = time.perf_counter()
        res = srv.run(reqs(arr))
        wall = time.perf_counter() - t0
        srv.close()
        tts = [r.time_to_solution for r in res]
        runs.append({"load": load, "arrival_rate_per_s": rate,
                     "p50_time_to_solution_s": S.percentile(tts, 50),
                     "p99_time_to_solution_s": S.percentile(tts, 99),
                     "zone_updates_per_s": sum(r.zone_updates for r in res) / wall, "wall_s": wall,
                     "rounds": srv.ticks, "mean_resident": float(np.mean(srv.batch_sizes)),
                     "peak_resident_bytes": srv.peak_in_use})
        log(f"{label}: load {load}, p50 {runs[-1]['p50_time_to_solution_s']:.3f} s, "
            f"p99 {runs[-1]['p99_time_to_solution_s']:.3f} s, {wall:.1f} s")
    # one at a time, FP64, single-simulation entry points, on a sample
    ns = min(seq_sample, len(mix))
    zs = 0
    t0 = time.perf_counter()
    for m in mix[:ns]:
        P = m["problem"]
        p = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad)
        g = R.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
        sv = R.Solver(g, p)
        U = sv.prim_to_cons(torch.from_numpy(P.V).cuda())
        o = R.make_opacities(torch.from_numpy(P.kappa).cuda(), torch.from_numpy(P.sigma).cuda())
        t, k = 0.0, 0
        while (m["steps"] is not None and k < m["steps"]) or (m["t_end"] is not None and t < m["t_end"] * (1 - 1e-14)):
            dt = P.cfl * min(P.dx) / sv.max_speed(U)
            if m["t_end"] is not None:
                dt = min(dt, m["t_end"] - t)
            sv.step(U, dt, o)
            t += dt
            k += 1
        torch.cuda.synchronize()
        sv.close()
        zs += k * P.ncell
    seq_s = time.perf_counter() - t0
    log(f"{label}: one-at-a-time FP64 on {ns} requests in {seq_s:.1f} s")
    return {"requests": len(mix), "capacity_req_per_s": mu, "capacity_zone_updates_per_s": zu / cap_s,
            "requests_with_counted_failures": fails, "counted_failures_by_kind": by_kind, "runs": runs,
            "one_at_a_time_fp64": {"requests": ns, "zone_updates_per_s": zs / seq_s, "wall_s": seq_s},
            "batched_capacity_over_one_at_a_time_fp64": (zu / cap_s) / (zs / seq_s),
            "hbm_budget_bytes": budget}


def serving_bench(args):
    """The serving workload as specified: >= 1000 requests, half 1D Riemann
    problems (N ~ logU[256, 8192], to t = 0.4), half 2D blasts (N^2 cells,
    N ~ logU[64, 512], 100 steps), FP64 / mixed 50/50, Poisson arrivals at
    each load x capacity."""
    from paper_2212_00370_amd import inputs as I
    mix = I.serving_mix(args.seed, args.requests, t_end_1d=args.t_end_1d, steps_2d=(args.steps_2d, args.steps_2d))
    loads = [float(x) for x in args.loads.split(",")]
    r = serving_run(mix, loads, args.seed, args.seq_sample)
    main = min(r["runs"], key=lambda x: abs(x["load"] - 0.8))
    return {
        "metric": METRIC, "value": main["zone_updates_per_s"], "unit": "zone-updates/s", "n_gpus": 1,
        "mode": "serving", "higher_is_better": True, "data": "synthetic",
        "dtype": "f64 and f32+f64 requests (50/50)",
        "p50_time_to_solution_s": main["p50_time_to_solution_s"],
        "p99_time_to_solution_s": main["p99_time_to_solution_s"], "load": main["load"],
        "config": {"workload": f"Poisson stream of {args.requests} requests: 1D Riemann N~logU[256,8192] to "
                               f"t={args.t_end_1d}, 2D blast N^2 with N~logU[64,512] for {args.steps_2d} steps, "
                               f"FP64/mixed 50/50, loads {args.loads}"},
        "serving": r,
    }


def riemann1d_bench(args):
    """A batch of seeded 1D Riemann problems (400 cells on [0, 1], PLM MinMod,
    PVM-int-8, IMEX RK2, CFL 0.4) run to t = 0.4 together through
    rrmhd_advance_batch: one problem cannot fill the GPU, so the throughput
    figure is for `--batch` seeds at once, each with its own CFL time step
    formed on the device (`--chunk` steps per call and synchronization;
    finished problems are skipped)."""
    import numpy as np
    import torch
    from paper_2212_00370_amd import inputs as I
    from paper_2212_00370_amd import rrmhd as R

    nb = args.batch
    prec = R.MIXED if args.precision == "mixed" else R.FP64
    sims = []
    for seed in range(nb):
        P = I.riemann_1d(seed, 400)
        p = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad, precision=prec)
        g = R.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
        sv = R.Solver(g, p)
        U = sv.prim_to_cons(torch.from_numpy(P.V).cuda())
        o = R.make_opacities(torch.from_numpy(P.kappa).cuda(), torch.from_numpy(P.sigma).cuda())
        sims.append(dict(P=P, s=sv, U=U, U0=U.clone(), o=o, t=0.0, k=0))
    batch = R.Batch(nb)
    torch.cuda.synchronize()

    cfl_dx = np.array([d["P"].cfl * d["P"].dx[0] for d in sims])
    t_end = np.array([d["P"].t_end for d in sims])

    no_count = np.full(nb, -1, dtype=np.int64)
    batch.set_active([d["s"] for d in sims], [d["U"] for d in sims], [d["o"] for d in sims])

    def run_all(max_steps=None):
        # each problem's CFL loop on the device, `chunk` steps per call; a
        # problem at t_end is skipped by the launches that follow
        for d in sims:
            d["U"].copy_(d["U0"])
            d["s"].report()
        torch.cuda.synchronize()
        t = np.zeros(nb)
        k = np.zeros(nb, dtype=np.int64)
        calls = 0
        while not (t >= t_end * (1 - 1e-14)).all() and (max_steps is None or k.max() < max_steps):
            chunk = args.chunk if max_steps is None else min(args.chunk, max_steps - int(k.max()))
            batch.advance_active(cfl_dx, t_end, no_count, t, k, chunk)
            t, k = batch.clock_active()
            calls += 1
        torch.cuda.synchronize()
        for i, d in enumerate(sims):
            d["k"] = int(k[i])
        return int(k.max()), calls

    run_all(max_steps=5)                      # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ticks, calls = run_all()
    el = time.perf_counter() - t0
    zu = sum(d["k"] * d["P"].ncell for d in sims)
    reps = [d["s"].report() for d in sims]
    failing = sorted(i for i, r in enumerate(reps) if r["imp_fail"] or r["c2p_fail"])
    batch.close()
    for d in sims:
        d["s"].close()
    return {"metric": METRIC, "value": zu / el, "unit": "zone-updates/s", "n_gpus": 1,
            "steps": int(np.max([d["k"] for d in sims])), "warmup": 5, "ms_per_step": 1e3 * el / ticks,
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f32+f64" if prec == R.MIXED else "f64", "data": "synthetic", "mode": "riemann1d",
            "config": {"workload": f"{nb} seeded 1D RRMHD+M1 Riemann problems x 400 cells, PVM-int-8, PLM MinMod, "
                                   f"IMEX RK2, CFL 0.4, to t=0.4, batched (rrmhd_advance_batch, {args.chunk} "
                                   f"device-side CFL steps per call)",
                       "problems": nb, "cells_per_problem": 400},
            "ticks": ticks, "calls": calls, "zone_updates": zu, "wall_s": el,
            "steps_per_problem": {"min": int(min(d["k"] for d in sims)), "max": int(max(d["k"] for d in sims))},
            "problems_with_counted_failures": len(failing), "failing_seeds_below_32": [i for i in failing if i < 32]}


def beam3d_bench(args):
    """3D beam (W = 7, B_phi = 0.3, inflow mask on z = 0) into a thick ambient
    medium, n^3 cells (default 512^3) in mixed precision, CFL 0.3. Also runs the
    256^3 problem in FP64 and in mixed precision with the FP64 run's dt
    sequence and reports L1(rho), L1(E_r) of mixed vs FP64 (the FP64 GPU path
    is bit-identical to the CPU oracle per step)."""
    import numpy as np
    import torch
    from paper_2212_00370_amd import inputs as I
    from paper_2212_00370_amd import rrmhd as R

    n = args.n if args.n != 512 or True else 512
    steps = args.steps if args.steps != 200 else 50
    solver = {"pvm": R.SOLVER_PVM, "hll": R.SOLVER_HLL, "jvp": R.SOLVER_PVM_JVP}[args.solver]

    def setup(P, prec):
        p = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad, precision=prec, e_floor=1e-14, solver=solver)
        Vin = torch.from_numpy(P.extra["inflow_V"]).cuda()
        mask = torch.from_numpy(P.extra["inflow_mask"]).cuda()
        g0 = R.make_grid(P.shape[:2], P.dx[:2])        # transverse plane, for the inflow state's p2c
        s0 = R.Solver(g0, p)
        Uin = s0.prim_to_cons(Vin)
        torch.cuda.synchronize(); s0.close()
        g = R.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi, inflow_U=Uin, inflow_mask=mask)
        s = R.Solver(g, p)
        V = torch.from_numpy(P.V).cuda()
        U = s.prim_to_cons(V)
        del V
        o = R.make_opacities(torch.from_numpy(P.kappa).cuda(), None, 0.0, 0.0)
        torch.cuda.synchronize()
        return s, U, o, (Uin, mask)

    # full grid, mixed precision
    P = I.beam_3d(args.seed, n)
    s, U, o, keep = setup(P, R.MIXED)
    Uw = U.clone()
    s.advance(Uw, P.cfl, 2, o)
    del Uw
    s.report()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s.advance(U, P.cfl, steps, o)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rep = s.report()
    s.close()
    del U, s, o, keep
    torch.cuda.empty_cache()
    # 256^3 sub-box problem: FP64 vs mixed
    Q = I.beam_3d(args.seed, 256)
    s64, U64, o64, k64 = setup(Q, R.FP64)
    smx, Umx, omx, kmx = setup(Q, R.MIXED)
    t64 = tmx = 0.0
    for _ in range(steps):
        dt = Q.cfl * min(Q.dx) / s64.max_speed(U64)
        torch.cuda.synchronize(); a = time.perf_counter()
        s64.step(U64, dt, o64); torch.cuda.synchronize(); b_ = time.perf_counter()
        smx.step(Umx, dt, omx); torch.cuda.synchronize(); c = time.perf_counter()
        t64 += b_ - a; tmx += c - b_
    V64 = s64.cons_to_prim(U64); Vmx = smx.cons_to_prim(Umx)
    l1 = lambda x, y: float((x - y).abs().sum() / y.abs().sum())
    sub = {"cells": Q.ncell, "steps": steps, "L1_rho_mixed_vs_fp64": l1(Vmx[0], V64[0]),
           "L1_Er_mixed_vs_fp64": l1(Umx[8], U64[8]),
           "fp64_step_zone_updates_per_s": Q.ncell * steps / t64,
           "mixed_step_zone_updates_per_s": Q.ncell * steps / tmx,
           "fp64_report": s64.report(), "mixed_report": smx.report()}
    s64.close(); smx.close()
    return {"metric": METRIC, "value": P.ncell * steps / el, "unit": "zone-updates/s", "n_gpus": 1,
            "steps": steps, "warmup": 2, "ms_per_step": 1e3 * el / steps, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64", "data": "synthetic", "mode": "beam3d",
            "config": {"workload": f"3D RRMHD+M1 beam {n}^3 mixed FP32/FP64, "
                                   f"{ {'pvm': 'PVM-int-8', 'hll': 'Rad-HLL', 'jvp': 'exact-JVP PVM-int-8'}[args.solver] } "
                                   f"(W=7, B_phi 0.3, inflow mask, "
                                   f"kappa logU[10,1e3]), CFL 0.3, {steps} steps", "cells": P.ncell},
            "failures": rep, "subbox_256": sub}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=int(os.environ.get("WORLD_SIZE", "1")))
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-steps", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--precision", choices=("fp64", "mixed"), default="fp64")
    ap.add_argument("--solver", choices=("pvm", "hll", "jvp"), default="pvm",
                    help="face flux: PVM-int-8 (the method), Rad-HLL (the paper's comparison solver) or "
                         "PVM-int-8 with exact Jacobian-vector products")
    ap.add_argument("--mode", choices=("step", "serving", "riemann1d", "beam3d", "copycal"), default="step")
    ap.add_argument("--no-variants", dest="variants", action="store_false",
                    help="skip the Rad-HLL / exact-JVP / mixed-precision lines of the default run")
    ap.add_argument("--no-serving", dest="serving", action="store_false",
                    help="skip the short serving leg of the default run")
    ap.add_argument("--requests", type=int, default=1000, help="--mode serving: number of requests")
    ap.add_argument("--loads", default="0.5,0.8,0.95", help="--mode serving: arrival rate / measured capacity")
    ap.add_argument("--t-end-1d", type=float, default=0.4, help="--mode serving: end time of the 1D requests")
    ap.add_argument("--steps-2d", type=int, default=100, help="--mode serving: steps of the 2D requests")
    ap.add_argument("--seq-sample", type=int, default=100,
                    help="--mode serving: requests run one at a time in FP64 for the comparison")
    ap.add_argument("--batch", type=int, default=1024, help="--mode riemann1d: problems run together")
    ap.add_argument("--chunk", type=int, default=64,
                    help="--mode riemann1d: device-side steps per rrmhd_advance_batch call")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU only (asked for {args.gpus}); "
              "multi-GPU sharding is designed but not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2212_00370_amd import inputs as I
    from paper_2212_00370_amd import rrmhd as R

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")
    if args.mode == "serving":
        print(json.dumps(serving_bench(args)), flush=True)
        return
    if args.mode == "riemann1d":
        print(json.dumps(riemann1d_bench(args)), flush=True)
        return
    if args.mode == "beam3d":
        print(json.dumps(beam3d_bench(args)), flush=True)
        return
    if args.mode == "copycal":
        # Plain device copy of a known size (256 MiB, 5 times): the reference
        # that scales the HBM byte counters (FETCH_SIZE / WRITE_SIZE).
        x = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device=dev)
        y = torch.empty_like(x)
        for _ in range(5):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"mode": "copycal", "bytes_per_copy": x.numel() * 8, "copies": 5}), flush=True)
        return
    P = I.blast_2d(args.seed, args.n, steps=args.steps)
    mixed = args.precision == "mixed"
    hll = args.solver == "hll"
    solver_id = {"pvm": R.SOLVER_PVM, "hll": R.SOLVER_HLL, "jvp": R.SOLVER_PVM_JVP}[args.solver]
    solver_name = {"pvm": "PVM-int-8", "hll": "Rad-HLL", "jvp": "PVM-int-8 (exact JVP)"}[args.solver]
    params = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad, precision=R.MIXED if mixed else R.FP64,
                                    solver=solver_id)
    grid = R.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    solver = R.Solver(grid, params, device=dev)
    V = torch.from_numpy(P.V).to(dev)
    U0 = solver.prim_to_cons(V)
    kap = torch.from_numpy(P.kappa).to(dev)
    sig = torch.from_numpy(P.sigma).to(dev)
    opac = R.make_opacities(kap, sig)
    dxmin = min(P.dx)

    def run(U, nsteps, dt_out=None):
        # each step: signal speed, dt = cfl dx_min / s_max on the device, IMEX step
        solver.advance(U, P.cfl, nsteps, opac, dt_out)

    # The first profiling enable creates the library's HIP events (host time
    # only); done here, before the warm-up, so that it does not sit between
    # the warm-up and the timed steps.
    R.rrmhd_profile_enable(solver.ctx, 1 << R.K_FACES)
    R.rrmhd_profile_enable(solver.ctx, 0)
    U = U0.clone()
    dts = torch.zeros(args.steps, dtype=torch.float64, device=dev)
    # warm-up on a copy, then restart from the initial state
    Uw = U0.clone()
    run(Uw, args.warmup)
    torch.cuda.synchronize()
    solver.report()
    # Inside the timed region only the face kernel (the roofline's kernel) is
    # bracketed by HIP events, every 7th launch (odd, so both stages are
    # sampled; each event pair serializes the stream around its launch).
    R.rrmhd_profile_enable(solver.ctx, 1 << R.K_FACES)
    R.rrmhd_profile_stride(solver.ctx, 7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(U, args.steps, dts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    rep = solver.report()
    prof = {"faces": R.rrmhd_profile_read(solver.ctx, R.K_FACES)}
    R.rrmhd_profile_enable(solver.ctx, False)
    R.rrmhd_profile_stride(solver.ctx, 1)
    # Per-kernel breakdown from a separate short run with every launch timed
    # ("prims": stage recoveries, the first stage's fused with the speeds).
    Ub = U0.clone()
    torch.cuda.synchronize()
    R.rrmhd_profile_enable(solver.ctx, True)
    nb = min(args.steps, 20)
    run(Ub, nb)
    torch.cuda.synchronize()
    breakdown = {name: R.rrmhd_profile_read(solver.ctx, k) for name, k in
                 (("prims", R.K_PRIMS), ("faces", R.K_FACES), ("update", R.K_UPDATE), ("newton", R.K_NEWTON),
                  ("speed", R.K_SPEED))}
    breakdown = {k: round(v[0] / nb, 4) for k, v in breakdown.items() if v[1] > 0}
    R.rrmhd_profile_enable(solver.ctx, False)
    solver.report()
    del Ub

    value = P.ncell * args.steps / elapsed
    ms_step = 1e3 * elapsed / args.steps

    # the spread of the timed figure: four more runs of the same steps from
    # the same initial state, timed the same way but without the first run's
    # face-kernel event pairs (not part of `value`)
    reps = [ms_step]
    for _ in range(4):
        Ur = U0.clone()
        torch.cuda.synchronize()
        r0 = time.perf_counter()
        run(Ur, args.steps)
        torch.cuda.synchronize()
        reps.append(1e3 * (time.perf_counter() - r0) / args.steps)
        del Ur
    solver.report()

    # roofline of the dominant kernel (face fluxes)
    sfx = {"pvm": "", "hll": "_hll", "jvp": "_jvp"}[args.solver]
    ops = op_counts(os.path.join(ROOT, "oracle", f"opcount_blast2d_{args.n}{sfx}.json"), args.steps)
    fms, flaunch, ffaces = prof["faces"]
    roof = None
    if ops and flaunch > 0 and not mixed:
        per_face = ops["faces_ops_per_face"]
        mean_s = fms / 1e3 / flaunch
        flops_per_launch = per_face * ffaces / flaunch
        achieved = flops_per_launch / mean_s / 1e12
        traffic = None
        tr = None if args.solver != "pvm" else load_json(
            os.path.join(ROOT, "profiles", f"traffic_k_faces_blast2d_{args.n}.json"))
        if tr and tr.get("sources_sha256") == kernel_sources_digest():
            traffic = tr.get("hbm_bytes_per_launch")
        roof = {"bound": "alu", "achieved": round(achieved, 3), "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(achieved / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "kernel": "k_faces (PLM MinMod + " + solver_name + " face flux)",
                "ops_per_face": round(per_face, 1), "ops_snapshots": ops["snapshot_steps"],
                "ops_average": "trapezoid rule over the snapshot steps",
                "faces_per_launch": ffaces // flaunch, "mean_launch_ms": round(1e3 * mean_s, 4)}

    # the implicit pass (flux divergence + implicit solve + next-stage
    # recovery: k_update and k_newton), per stage, from the breakdown run
    imp = None
    if ops and not mixed and "update" in breakdown and "newton" in breakdown:
        per_cell = ops["divergence_ops_per_cell"] + ops["implicit_ops_per_cell"] + ops["prims_ops_per_cell"]
        stage_s = (breakdown["update"] + breakdown["newton"]) / 2 / 1e3
        a = per_cell * P.ncell / stage_s / 1e12
        imp = {"bound": "alu", "kernels": "k_update + k_newton", "ops_per_cell": round(per_cell, 1),
               "ops_snapshots": ops["snapshot_steps"],
               "cells_per_stage": P.ncell, "us_per_stage": round(1e6 * stage_s, 1), "achieved": round(a, 3),
               "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(a / FP64_PEAK_TFLOPS, 4)}
        if "implicit_newton_ops_per_cell" in ops:
            # per kernel: the update pass does the divergence, the Picard phase
            # and the recoveries (those of its listed cells too, a small share);
            # the work-list pass does the Newton phase
            nw = ops["implicit_newton_ops_per_cell"]
            for name, cell_ops, ms in (("k_update", per_cell - nw, breakdown["update"]),
                                       ("k_newton", nw, breakdown["newton"])):
                t = ms / 2 / 1e3
                ak = cell_ops * P.ncell / t / 1e12
                imp[name] = {"ops_per_cell_of_grid": round(cell_ops, 1), "us_per_stage": round(1e6 * t, 1),
                             "achieved": round(ak, 3), "frac": round(ak / FP64_PEAK_TFLOPS, 4)}

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "zone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if mixed else "f64",
        "data": "synthetic",
        "config": {"workload": f"2D RRMHD+M1 magnetised blast {P.shape[0]}x{P.shape[1]} "
                               f"{'mixed FP32/FP64' if mixed else 'FP64'}, seed {args.seed}, "
                               f"{solver_name}, PLM MinMod, IMEX RK2, CFL {P.cfl}, "
                               f"{args.steps} steps",
                   "cells": P.ncell, "precision": args.precision, "solver": args.solver,
                   "beta_mode": "radiation rows" if not hll else None},
        "roofline": roof,
        "roofline_implicit_pass": imp,
        "kernels_ms_per_step": breakdown,
        "kernels_ms_per_step_note": "separate run of min(steps, 20) steps with every launch timed",
        "ms_per_step_repeats": [round(x, 4) for x in reps],
        "ms_per_step_median_of_5": round(sorted(reps)[2], 4),
        "failures": {k: rep[k] for k in ("c2p_fail", "pvm_fallback", "imp_fail", "nonfinite")},
    }
    Ufinal = U.cpu().numpy()
    dts_host = dts.cpu().numpy()
    if args.variants and args.solver == "pvm" and not mixed:
        out["variants"] = variants_bench(R, P, grid, V, opac, args.steps, args.warmup)
        log("variants done")
        out["mixed_vs_fp64"] = mixed_accuracy(R, P, grid, V, opac, dts_host, Ufinal)
        log("mixed-precision accuracy done")
    if args.serving and args.solver == "pvm" and not mixed:
        out["serving"] = serving_leg(args.seed)
    if not args.no_cpu_baseline:
        cmp = None
        if not mixed:
            if args.steps <= args.cpu_steps:
                cmp = (args.steps, Ufinal)
            else:
                # the oracle's sample is shorter than the timed run: the same
                # path advanced from the initial state by the sample's steps
                Uc = U0.clone()
                run(Uc, args.cpu_steps)
                torch.cuda.synchronize()
                solver.report()
                cmp = (args.cpu_steps, Uc.cpu().numpy())
                del Uc
        out["cpu_baseline"], chk = cpu_baseline(P, args.cpu_steps, solver_id, cmp)
        if chk is not None:
            out["fp64_vs_oracle"] = dict(chk, note="GPU state (rrmhd_advance, as timed) after these steps "
                                                   "against the CPU oracle's state after the same steps from "
                                                   "the same initial state")
    print(json.dumps(out), flush=True)


def serving_leg(seed):
    """A short serving run inside the default benchmark: 48 requests of the
    serving mix with shorter runs (1D to t = 0.05, 2D 10-50 steps), Poisson
    arrivals at 0.8 x capacity, and the same requests one at a time in FP64."""
    from paper_2212_00370_amd import inputs as I
    mix = I.serving_mix(seed, 48, t_end_1d=0.05, steps_2d=(10, 50))
    r = serving_run(mix, [0.8], seed, len(mix), label="serving leg")
    run = r["runs"][0]
    return {"workload": "48 Poisson requests at 0.8 x capacity: 1D Riemann N~logU[256,8192] to t=0.05, "
                        "2D blast N^2, N~logU[64,512], 10-50 steps; FP64/mixed 50/50",
            "p50_time_to_solution_s": run["p50_time_to_solution_s"],
            "p99_time_to_solution_s": run["p99_time_to_solution_s"],
            "zone_updates_per_s": run["zone_updates_per_s"],
            "capacity_zone_updates_per_s": r["capacity_zone_updates_per_s"],
            "one_at_a_time_fp64_zone_updates_per_s": r["one_at_a_time_fp64"]["zone_updates_per_s"],
            "batched_capacity_over_one_at_a_time_fp64": r["batched_capacity_over_one_at_a_time_fp64"],
            "mean_resident": run["mean_resident"], "requests_with_counted_failures": r["requests_with_counted_failures"]}


def mixed_accuracy(R, P, grid, V, opac, dts, U64_final):
    """L1 of each mixed-precision form against the FP64 path with the same
    face flux, both advanced from the same initial state with the same time
    steps (those of the timed FP64 run): L1_rel(q) = sum|q_mixed - q_fp64| /
    sum|q_fp64| for q = rho and E_r, at steps 1, 10, 50, 200 (those within the
    run). The FP64 PVM-int-8 state is first checked to equal the timed run's
    (and so the oracle's, bit for bit)."""
    import torch
    marks = [k for k in (1, 10, 50, 200) if k <= len(dts)]
    if len(dts) not in marks:
        marks.append(len(dts))

    def trajectory(solver, prec):
        params = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad, precision=prec, solver=solver)
        sv = R.Solver(grid, params, device=V.device)
        U = sv.prim_to_cons(V)
        snaps = {}
        for k, dt in enumerate(dts, start=1):
            sv.step(U, float(dt), opac)
            if k in marks:
                Vp = sv.cons_to_prim(U)
                snaps[k] = (Vp[0].clone(), U[8].clone())
        rep = sv.report()
        Uf = U.cpu().numpy()
        sv.close()
        return snaps, Uf, rep

    l1 = lambda a, b: float((a - b).abs().sum() / b.abs().sum())
    res = {"steps": marks, "dt_sequence": "that of the timed FP64 PVM-int-8 run",
           "accumulation": "face fluxes binary32; flux divergence, recoveries and implicit solve binary64"}
    import numpy as np
    for name, solver in (("pvm", R.SOLVER_PVM), ("pvm_jvp", R.SOLVER_PVM_JVP), ("rad_hll", R.SOLVER_HLL)):
        ref, Uref, rep64 = trajectory(solver, R.FP64)
        if solver == R.SOLVER_PVM:
            res["fp64_host_dt_equals_timed_run"] = bool(np.array_equal(Uref, U64_final))
        mix, _, rep = trajectory(solver, R.MIXED)
        res[name] = {"L1_rho": [l1(mix[k][0], ref[k][0]) for k in marks],
                     "L1_Er": [l1(mix[k][1], ref[k][1]) for k in marks],
                     "mixed_failures": {k: rep[k] for k in ("c2p_fail", "pvm_fallback", "imp_fail", "nonfinite")},
                     "fp64_failures": {k: rep64[k] for k in ("c2p_fail", "pvm_fallback", "imp_fail", "nonfinite")}}
        del ref, mix
        torch.cuda.empty_cache()
    return res


def variants_bench(R, P, grid, V, opac, steps, warmup):
    """The same workload with the other face fluxes and precisions (each its own
    context; same step count; timed like the main line), for the cost ratios:
    Rad-HLL (the paper's comparison solver), the exact-JVP PVM-int-8 flux,
    PVM-int-8 with constrained transport, and mixed precision with the
    difference, the exact-JVP and the Rad-HLL flux."""
    import torch
    from paper_2212_00370_amd import inputs as I
    res = {}
    for name, solver, prec, ct in (("rad_hll_fp64", R.SOLVER_HLL, R.FP64, 0),
                                   ("pvm_jvp_fp64", R.SOLVER_PVM_JVP, R.FP64, 0),
                                   ("pvm_ct_fp64", R.SOLVER_PVM, R.FP64, 1),
                                   ("pvm_mixed", R.SOLVER_PVM, R.MIXED, 0),
                                   ("pvm_jvp_mixed", R.SOLVER_PVM_JVP, R.MIXED, 0),
                                   ("rad_hll_mixed", R.SOLVER_HLL, R.MIXED, 0)):
        params = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad, precision=prec, solver=solver, ct=ct)
        sv = R.Solver(grid, params, device=V.device)
        U0 = sv.prim_to_cons(V)
        if ct:
            # constrained transport: the face-field planes of the uniform initial field
            U0 = torch.cat([U0, torch.from_numpy(I.uniform_face_fields(P)).to(V.device)]).contiguous()
        # CT runs this blast at CFL 0.3: at 0.4 its face-mean cell field
        # undershoots the pressure at the foot of the blast front until
        # recoveries fail (the cell-centred scheme is clean there)
        cfl = 0.3 if ct else P.cfl
        Uw = U0.clone()
        sv.advance(Uw, cfl, warmup, opac)
        torch.cuda.synchronize()
        sv.report()
        U = U0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv.advance(U, cfl, steps, opac)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rep = sv.report()
        Ub = U0.clone()
        R.rrmhd_profile_enable(sv.ctx, 1 << R.K_FACES)
        nb = min(steps, 20)
        sv.advance(Ub, cfl, nb, opac)
        torch.cuda.synchronize()
        fms, fl, _ = R.rrmhd_profile_read(sv.ctx, R.K_FACES)
        R.rrmhd_profile_enable(sv.ctx, False)
        sv.report()
        res[name] = {"value": P.ncell * steps / el, "ms_per_step": 1e3 * el / steps,
                     "faces_ms_per_step": round(fms / nb, 4), "faces_mean_launch_ms": round(fms / max(fl, 1), 4),
                     "failures": {k: rep[k] for k in ("c2p_fail", "pvm_fallback", "imp_fail", "nonfinite")}}
        if prec == R.MIXED:
            res[name]["accumulation"] = "binary32 face fluxes, binary64 flux divergence"
        if ct:
            res[name]["note"] = "constrained transport (staggered face fields, CT-contact edge EMFs), CFL 0.3"
        sv.close()
        del U, Ub, Uw, U0
    return res


if __name__ == "__main__":
    main()
