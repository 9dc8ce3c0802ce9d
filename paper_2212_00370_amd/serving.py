"""Continuous-batching server for independent RRMHD+M1 simulations.

Requests (a seeded problem, a precision, an end time or a step count) arrive
over time. The server keeps admitted simulations resident on the device and,
on every tick, advances all of them by one IMEX step each with a single
batched launch per kernel class (rrmhd_max_speed_batch then
rrmhd_step_batch): simulations of different sizes and precisions share every
launch. A request is admitted, in arrival order, as soon as its HBM
footprint (state, opacities, workspace) fits in the budget and a batch slot
is free; finished simulations are copied to the host and their memory is
released, which admits the next ones. Results do not depend on the batch
composition (each simulation's arithmetic is that of rrmhd_step).
"""
from __future__ import annotations

import time
from dataclasses import dataclass, field

import numpy as np

from . import rrmhd as R
from .inputs import Problem


@dataclass
class Request:
    rid: int
    problem: Problem
    precision: int = R.FP64
    t_end: float | None = None      # run to this time (CFL steps, last clipped) ...
    steps: int | None = None        # ... or this many CFL steps
    arrival: float = 0.0            # seconds after the server starts


@dataclass
class Result:
    rid: int
    U: np.ndarray
    steps: int
    t: float
    arrival: float
    admitted: float
    finished: float
    zone_updates: int
    report: dict = field(default_factory=dict)

    @property
    def time_to_solution(self) -> float:
        return self.finished - self.arrival


class _Sim:
    def __init__(self, req: Request, device, torch):
        P = req.problem
        self.req = req
        self.params = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad, t_coeff=P.t_coeff,
                                             precision=req.precision)
        self.grid = R.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
        self.solver = R.Solver(self.grid, self.params, device=device)
        V = torch.from_numpy(np.ascontiguousarray(P.V)).to(device)
        self.U = self.solver.prim_to_cons(V)
        self.kappa = torch.from_numpy(np.ascontiguousarray(P.kappa)).to(device)
        self.sigma = torch.from_numpy(np.ascontiguousarray(P.sigma)).to(device)
        self.opac = R.make_opacities(self.kappa, self.sigma)
        self.t = 0.0
        self.steps = 0
        self.dxmin = min(P.dx)

    def done(self) -> bool:
        r = self.req
        if r.steps is not None:
            return self.steps >= r.steps
        return self.t >= r.t_end * (1.0 - 1e-14)

    def close(self):
        self.solver.close()


def footprint_bytes(problem: Problem, precision: int = R.FP64) -> int:
    """Device bytes a request holds while resident: state, opacities, workspace."""
    p = R.rrmhd_default_params(gamma=problem.gamma, a_rad=problem.a_rad, precision=precision)
    g = R.make_grid(problem.shape, problem.dx, problem.bc_lo, problem.bc_hi)
    n = problem.ncell
    return 8 * n * (R.NVAR + 2) + R.rrmhd_workspace_bytes(g, p) + 256


class Server:
    def __init__(self, hbm_budget: int, max_sims: int = 256, device="cuda:0"):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(hbm_budget)
        self.max_sims = max_sims
        self.batch = R.Batch(max_sims, device=self.device)
        self.in_use = 0
        self.peak_in_use = 0
        self.ticks = 0
        self.batch_sizes = []

    def run(self, requests: list[Request], clock=time.perf_counter) -> list[Result]:
        """Serve `requests` (sorted by arrival) to completion; returns results
        in completion order. Arrival times are wall-clock offsets from the
        start of this call."""
        torch = self.torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            if footprint_bytes(r.problem, r.precision) > self.budget:
                raise ValueError(f"request {r.rid} does not fit the HBM budget")
        active: list[_Sim] = []
        results: list[Result] = []
        changed = True          # the active set differs from the batch's
        t = nstep = None        # time and steps of the active set while it is unchanged

        def sync():
            """Write the active set's time and step count back to its sims."""
            if t is not None and not changed:
                for i, sim in enumerate(active):
                    sim.t = float(t[i])
                    sim.steps = int(nstep[i])

        t0 = clock()
        qi = 0
        while qi < len(pending) or active:
            now = clock() - t0
            # admit in arrival order while memory and slots allow
            while (qi < len(pending) and pending[qi].arrival <= now and len(active) < self.max_sims):
                r = pending[qi]
                need = footprint_bytes(r.problem, r.precision)
                if self.in_use + need > self.budget:
                    break
                sim = _Sim(r, self.device, torch)
                sim.need = need
                sim.admitted = now
                self.in_use += need
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                sync()
                active.append(sim)
                changed = True
                qi += 1
            if not active:
                # idle until the next arrival
                if qi < len(pending):
                    wait = pending[qi].arrival - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            if changed:
                self.batch.set_active([s.solver for s in active], [s.U for s in active], [s.opac for s in active])
                # per-simulation time-step data of the active set, as arrays
                cfl_dx = np.array([s.req.problem.cfl * s.dxmin for s in active])
                t_end = np.array([s.req.t_end if s.req.t_end is not None else np.inf for s in active])
                t = np.array([s.t for s in active])
                nstep = np.array([s.steps for s in active], dtype=np.int64)
                max_steps = np.array([s.req.steps if s.req.steps is not None else -1 for s in active], dtype=np.int64)
                changed = False
            smax = self.batch.max_speed_active()
            dts = np.minimum(cfl_dx / smax, t_end - t)
            self.batch.step_active(dts)
            self.ticks += 1
            self.batch_sizes.append(len(active))
            t += dts
            nstep += 1
            done = np.where(max_steps >= 0, nstep >= max_steps, t >= t_end * (1.0 - 1e-14))
            if done.any():
                sync()
                finished = [sim for sim, d in zip(active, done) if d]
                torch.cuda.synchronize(self.device)
                end = clock() - t0
                for sim in finished:
                    results.append(Result(rid=sim.req.rid, U=sim.U.cpu().numpy(), steps=sim.steps, t=sim.t,
                                          arrival=sim.req.arrival, admitted=sim.admitted, finished=end,
                                          zone_updates=sim.steps * sim.req.problem.ncell,
                                          report=sim.solver.report()))
                    self.in_use -= sim.need
                    sim.close()
                active = [sim for sim, d in zip(active, done) if not d]
                changed = True
        return results

    def close(self):
        self.batch.close()


def percentile(values, q):
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        return float("nan")
    return float(np.percentile(v, q))
