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


def cpu_baseline(P, steps: int, solver: int = 0):
    """The CPU oracle (as it stands, OpenMP over cells) on the first `steps`
    steps of the same workload from the same initial state."""
    from oracle import oracle as O
    nthreads = O.threads(0)
    par = O.params(gamma=P.gamma, a_rad=P.a_rad, beta_mode=1, solver=solver)
    g = O.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    U = O.p2c(P.V, par)
    t0 = time.perf_counter()
    for _ in range(steps):
        s, _ = O.max_speed(g, U, par)
        dt = P.cfl * min(P.dx) / s
        U, st, rep = O.step(g, U, dt, P.kappa, P.sigma, par)
    el = time.perf_counter() - t0
    return dict(value=P.ncell * steps / el, unit="zone-updates/s", cores=nthreads, kind="oracle",
                sample=f"first {steps} steps of the same {P.shape[0]}x{P.shape[1]} blast "
                       f"(CFL signal speed + IMEX step), {el:.1f} s")


def serving_bench(args):
    """Continuous batching of a Poisson stream of independent problems (1D
    Riemann N ~ logU[256, 8192] to t = 0.05; 2D blasts N^2, N ~ logU[64, 512],
    10-50 steps; FP64 / mixed 50/50). Capacity is measured first with every
    request present at t = 0; the timed run uses Poisson arrivals at
    `load` x capacity. The comparison runs the same requests one at a time in
    FP64 through rrmhd_step."""
    import numpy as np
    import torch
    from paper_2212_00370_amd import inputs as I
    from paper_2212_00370_amd import rrmhd as R
    from paper_2212_00370_amd import serving as S

    mix = I.serving_mix(args.seed, args.requests)
    def reqs(arrivals, force_fp64=False):
        return [S.Request(rid=i, problem=m["problem"], precision=R.FP64 if (force_fp64 or not m["mixed"]) else R.MIXED,
                          t_end=m["t_end"], steps=m["steps"], arrival=float(a)) for i, (m, a) in enumerate(zip(mix, arrivals))]
    free, total = torch.cuda.mem_get_info()
    budget = int(0.5 * free)
    # capacity: all requests present at once
    srv = S.Server(budget, max_sims=256)
    t0 = time.perf_counter()
    res0 = srv.run(reqs(np.zeros(len(mix))))
    cap_s = time.perf_counter() - t0
    srv.close()
    zu = sum(r.zone_updates for r in res0)
    mu = len(mix) / cap_s
    rate = args.load * mu
    arr = I.poisson_arrivals(args.seed + 1, len(mix), rate)
    srv = S.Server(budget, max_sims=256)
    t0 = time.perf_counter()
    res = srv.run(reqs(arr))
    wall = time.perf_counter() - t0
    tts = [r.time_to_solution for r in res]
    # one at a time, FP64, single-simulation entry points
    t0 = time.perf_counter()
    for m in mix:
        P = m["problem"]
        p = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad)
        g = R.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
        s = R.Solver(g, p)
        U = s.prim_to_cons(torch.from_numpy(P.V).cuda())
        o = R.make_opacities(torch.from_numpy(P.kappa).cuda(), torch.from_numpy(P.sigma).cuda())
        t, k = 0.0, 0
        while (m["steps"] is not None and k < m["steps"]) or (m["t_end"] is not None and t < m["t_end"] * (1 - 1e-14)):
            dt = P.cfl * min(P.dx) / s.max_speed(U)
            if m["t_end"] is not None:
                dt = min(dt, m["t_end"] - t)
            s.step(U, dt, o)
            t += dt; k += 1
        torch.cuda.synchronize()
        s.close()
    seq_s = time.perf_counter() - t0
    return {
        "metric": METRIC, "value": zu / wall, "unit": "zone-updates/s", "n_gpus": 1,
        "mode": "serving", "requests": len(mix), "higher_is_better": True, "data": "synthetic",
        "dtype": "f64 and f32+f64 requests (50/50)",
        "p50_time_to_solution_s": S.percentile(tts, 50), "p99_time_to_solution_s": S.percentile(tts, 99),
        "arrival_rate_per_s": rate, "capacity_req_per_s": mu, "load": args.load,
        "capacity_zone_updates_per_s": zu / cap_s, "sequential_fp64_zone_updates_per_s": zu / seq_s,
        "wall_s": wall, "ticks": srv.ticks, "mean_batch": float(np.mean(srv.batch_sizes)),
        "hbm_budget_bytes": budget, "peak_resident_bytes": srv.peak_in_use,
        "config": {"workload": "Poisson stream: 1D Riemann N~logU[256,8192] to t=0.05, 2D blast N^2 with "
                               "N~logU[64,512] for 10-50 steps, FP64/mixed 50/50"},
    }


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
    ap.add_argument("--mode", choices=("step", "serving", "beam3d", "copycal"), default="step")
    ap.add_argument("--no-variants", dest="variants", action="store_false",
                    help="skip the Rad-HLL / exact-JVP / mixed-precision lines of the default run")
    ap.add_argument("--requests", type=int, default=120)
    ap.add_argument("--load", type=float, default=0.8, help="arrival rate / measured capacity")
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

    def run(U, nsteps):
        # each step: signal speed, dt = cfl dx_min / s_max on the device, IMEX step
        solver.advance(U, P.cfl, nsteps, opac)

    # warm-up on a copy, then restart from the initial state
    Uw = U0.clone()
    run(Uw, args.warmup)
    torch.cuda.synchronize()
    solver.report()
    U = U0.clone()
    torch.cuda.synchronize()
    # Inside the timed region only the face kernel (the roofline's kernel) is
    # bracketed by HIP events, every 7th launch (odd, so both stages are
    # sampled; each event pair serializes the stream around its launch).
    R.rrmhd_profile_enable(solver.ctx, 1 << R.K_FACES)
    R.rrmhd_profile_stride(solver.ctx, 7)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(U, args.steps)
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

    # roofline of the dominant kernel (face fluxes)
    sfx = {"pvm": "", "hll": "_hll", "jvp": "_jvp"}[args.solver]
    ops = load_json(os.path.join(ROOT, "oracle", f"opcount_blast2d_{args.n}{sfx}.json"))
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
                "ops_per_face": round(per_face, 1), "faces_per_launch": ffaces // flaunch,
                "mean_launch_ms": round(1e3 * mean_s, 4)}

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
        "kernels_ms_per_step": breakdown,
        "kernels_ms_per_step_note": "separate run of min(steps, 20) steps with every launch timed",
        "failures": {k: rep[k] for k in ("c2p_fail", "pvm_fallback", "imp_fail", "nonfinite")},
    }
    if args.variants and args.solver == "pvm" and not mixed:
        out["variants"] = variants_bench(R, P, grid, V, opac, args.steps, args.warmup)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(P, args.cpu_steps, solver_id)
    print(json.dumps(out), flush=True)


def variants_bench(R, P, grid, V, opac, steps, warmup):
    """The same workload with the other face fluxes and precisions (each its own
    context; same step count; timed like the main line), for the cost ratios:
    Rad-HLL (the paper's comparison solver), the exact-JVP PVM-int-8 flux, and
    mixed precision with the difference, the exact-JVP and the Rad-HLL flux."""
    import torch
    res = {}
    for name, solver, prec in (("rad_hll_fp64", R.SOLVER_HLL, R.FP64), ("pvm_jvp_fp64", R.SOLVER_PVM_JVP, R.FP64),
                               ("pvm_mixed", R.SOLVER_PVM, R.MIXED), ("pvm_jvp_mixed", R.SOLVER_PVM_JVP, R.MIXED),
                               ("rad_hll_mixed", R.SOLVER_HLL, R.MIXED)):
        params = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad, precision=prec, solver=solver)
        sv = R.Solver(grid, params, device=V.device)
        U0 = sv.prim_to_cons(V)
        Uw = U0.clone()
        sv.advance(Uw, P.cfl, warmup, opac)
        torch.cuda.synchronize()
        sv.report()
        U = U0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sv.advance(U, P.cfl, steps, opac)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rep = sv.report()
        Ub = U0.clone()
        R.rrmhd_profile_enable(sv.ctx, 1 << R.K_FACES)
        nb = min(steps, 20)
        sv.advance(Ub, P.cfl, nb, opac)
        torch.cuda.synchronize()
        fms, fl, _ = R.rrmhd_profile_read(sv.ctx, R.K_FACES)
        R.rrmhd_profile_enable(sv.ctx, False)
        sv.report()
        res[name] = {"value": P.ncell * steps / el, "ms_per_step": 1e3 * el / steps,
                     "faces_ms_per_step": round(fms / nb, 4), "faces_mean_launch_ms": round(fms / max(fl, 1), 4),
                     "failures": {k: rep[k] for k in ("c2p_fail", "pvm_fallback", "imp_fail", "nonfinite")}}
        sv.close()
        del U, Ub, Uw, U0
    return res


if __name__ == "__main__":
    main()
