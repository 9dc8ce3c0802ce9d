"""Algorithmic operation counts of the method on the 2D blast workload.

Runs the plain oracle (OpenMP build) on the 512^2 magnetised blast from its
seeded initial state, and at several snapshots counts, with the op-counting
build of the same source, the floating-point operations (+ - * / sqrt, one
each) of
  * the face-flux computation (PLM MinMod + Jacobian-free PVM-int-8 + beta),
    per face, both directions;
  * the cell primitive recovery of a stage, per cell;
  * the implicit radiation-matter solve of the first stage, per cell, and
    the part of it spent in the Newton phase (per cell of the grid).
With --solver hll (jvp) the run and the face count use Rad-HLL (the exact-JVP
PVM-int-8 flux) instead (``opcount_blast2d_512_hll.json``, ``..._jvp.json``).
Writes ``opcount_blast2d_512.json`` next to this file. Test infrastructure:
the GPU library does not read it; the benchmark reads the per-face figure to
turn measured kernel time into achieved FLOP/s.

usage: python oracle/count_ops.py [--n 512] [--snapshots 0,100,200] [--solver pvm|hll|jvp]
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(HERE))

from oracle import oracle as O  # noqa: E402
from paper_2212_00370_amd import inputs as I  # noqa: E402


def counted(fn, newton=False):
    """Operations of fn; with newton=True also those of the implicit solve's
    Newton phase alone (a subset of the first)."""
    L = O.lib(count=True)
    L.or_opcount_reset()
    fn(L)
    out = (C.c_ulonglong * 4)()
    L.or_opcount_get(out)
    res = dict(add=out[0], mul=out[1], div=out[2], sqrt=out[3])
    if not newton:
        return res
    L.or_opcount_get_newton(out)
    return res, dict(add=out[0], mul=out[1], div=out[2], sqrt=out[3])


def total(c):
    return c["add"] + c["mul"] + c["div"] + c["sqrt"]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=512)
    ap.add_argument("--snapshots", default="0,100,200")
    ap.add_argument("--solver", choices=("pvm", "hll", "jvp"), default="pvm")
    args = ap.parse_args()
    sid = {"pvm": O.SOLVER_PVM, "hll": O.SOLVER_HLL, "jvp": O.SOLVER_PVM_JVP}[args.solver]
    sname = {"pvm": "beta on radiation rows, PVM-int-8", "hll": "Rad-HLL",
             "jvp": "beta on radiation rows, PVM-int-8 with exact JVP"}[args.solver]
    snaps = sorted(int(s) for s in args.snapshots.split(","))
    O.threads(0)
    P = I.blast_2d(0, args.n)
    par = O.params(gamma=P.gamma, a_rad=P.a_rad, beta_mode=1, solver=sid)
    g = O.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    U = O.p2c(P.V, par)
    N = P.ncell
    nf = [(P.shape[0] + 1) * P.shape[1], P.shape[0] * (P.shape[1] + 1)]
    ka = np.ascontiguousarray(P.kappa); sa = np.ascontiguousarray(P.sigma)
    rows = []
    step = 0
    t0 = time.time()
    for target in snaps:
        while step < target:
            s, _ = O.max_speed(g, U, par)
            dt = P.cfl * min(P.dx) / s
            U, st, rep = O.step(g, U, dt, P.kappa, P.sigma, par)
            assert st == 0, (step, rep.c2p_fail, rep.imp_fail)
            step += 1
        s, _ = O.max_speed(g, U, par)
        dt = P.cfl * min(P.dx) / s
        Uc = np.ascontiguousarray(U)
        out = np.zeros(12 * sum(nf))
        c_all = counted(lambda L: L.or_face_fluxes(C.byref(g), C.byref(par), O._dp(Uc), O._dp(ka),
                                                   O._dp(sa), 0.0, 0.0, O._dp(out)))
        V = np.empty_like(Uc); Z = np.zeros(N); stt = np.zeros(N, np.int32); it = np.zeros(N, np.int32)
        c_c2p = counted(lambda L: L.or_c2p(N, O._dp(Uc), N, C.byref(par), None, O._dp(V), N, O._dp(Z),
                                           O._dp(stt), O._dp(it)))
        # stage prims = cold recovery + D (kappa + sigma): 2 more ops per cell
        prims = total(c_c2p) + 2 * N
        faces = {k: c_all[k] - c_c2p[k] for k in c_all}
        faces["add"] -= N
        faces["mul"] -= N
        Ust, _ = O.explicit_stage(g, Uc, Uc, P.kappa, P.sigma, 1.0, 0.0, 1.0, dt, par)
        Us = np.ascontiguousarray(Ust)
        Un = np.empty_like(Us); h = np.full(N, dt); st2 = np.zeros(N, np.int32); it2 = np.zeros(N, np.int32)
        c_imp, c_newton = counted(lambda L: L.or_implicit(N, O._dp(Us), N, O._dp(h), O._dp(ka), O._dp(sa),
                                                          C.byref(par), O._dp(Un), N, O._dp(st2), O._dp(it2)),
                                  newton=True)
        row = dict(step=step, faces_ops_per_face=total(faces) / sum(nf), faces_breakdown_per_face=
                   {k: v / sum(nf) for k, v in faces.items()}, prims_ops_per_cell=prims / N,
                   implicit_ops_per_cell=total(c_imp) / N,
                   implicit_breakdown_per_cell={k: v / N for k, v in c_imp.items()},
                   implicit_newton_ops_per_cell=total(c_newton) / N,
                   elapsed_s=time.time() - t0)
        print(json.dumps(row), flush=True)
        rows.append(row)
    mean = lambda k: float(np.mean([r[k] for r in rows]))
    res = dict(
        workload=f"2D RRMHD+M1 blast {args.n}x{args.n}, seed 0, {sname}, PLM MinMod, RK2",
        counting="+ - * / sqrt of the oracle (op-counting build), one each; no fused multiply-add is used",
        snapshots=rows,
        faces_ops_per_face=mean("faces_ops_per_face"),
        prims_ops_per_cell=mean("prims_ops_per_cell"),
        implicit_ops_per_cell=mean("implicit_ops_per_cell"),
        implicit_newton_ops_per_cell=mean("implicit_newton_ops_per_cell"),
        divergence_ops_per_cell=12 * (2 * 2 + 3),
    )
    sfx = {"pvm": "", "hll": "_hll", "jvp": "_jvp"}[args.solver]
    with open(os.path.join(HERE, f"opcount_blast2d_{args.n}{sfx}.json"), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps({k: v for k, v in res.items() if k != "snapshots"}))


if __name__ == "__main__":
    main()
