"""Continuous-batching server for independent RRMHD+M1 simulations.

Requests (a seeded problem, a precision, an end time or a step count) arrive
over time. The server keeps admitted simulations resident on the device, in
two size classes, each a batch on its own stream: every launch of a class
covers all its simulations (different sizes and precisions share it), and
each simulation's CFL time step is formed on the device, so a round of
several steps needs one synchronization (rrmhd_advance_batch, then
rrmhd_batch_clock). A request is admitted, in arrival order, as soon as its
HBM footprint (state, opacities, workspace) fits in the budget and a slot of
its class is free; finished simulations are copied to the host and their
memory is released, which admits the next ones. Results do not depend on the
batch composition (each simulation's arithmetic is that of rrmhd_step with
the host loop's time steps).
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


class _Class:
    """Admitted simulations of one size class: one batch on its own stream,
    advanced on the device (rrmhd_advance_batch) several steps per round."""

    def __init__(self, name: str, max_sims: int, device, torch):
        self.name = name
        self.stream = torch.cuda.Stream(device=device)
        self.batch = R.Batch(max_sims, device=device, stream=self.stream)
        self.max_sims = max_sims
        self.active: list[_Sim] = []
        self.changed = True
        self.step_s = None          # measured device time per step (moving average)
        self.k = 0                  # steps of the current round
        self.ev = None

    def set_arrays(self):
        a = self.active
        self.batch.set_active([s.solver for s in a], [s.U for s in a], [s.opac for s in a])
        self.cfl_dx = np.array([s.req.problem.cfl * s.dxmin for s in a])
        self.t_end = np.array([s.req.t_end if s.req.t_end is not None else np.inf for s in a])
        self.max_steps = np.array([s.req.steps if s.req.steps is not None else -1 for s in a], dtype=np.int64)
        self.changed = False

    def close(self):
        self.batch.close()


class Server:
    """Continuous batching in two size classes. Simulations of at most
    `light_cells` cells (the 1D requests of the serving mix) form the light
    class, larger ones the heavy class; each class is one batch on its own
    stream, so the two advance concurrently on the device and a light
    simulation takes its many small steps at its own pace instead of one per
    heavy step. Each round enqueues up to k steps per class with the time step
    formed on the device, k chosen from the class's measured time per step so
    that a round lasts about `round_s`; between rounds the server admits
    arrivals (in arrival order, within the HBM budget and the slots) and
    retires finished simulations."""

    def __init__(self, hbm_budget: int, max_sims: int = 256, device="cuda:0", light_cells: int = 8192,
                 round_s: float = 0.004, max_round_steps: int = 256):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(hbm_budget)
        self.max_sims = max_sims
        self.light_cells = int(light_cells)
        self.round_s = float(round_s)
        self.max_round_steps = int(max_round_steps)
        self.classes = [_Class("light", max_sims, self.device, torch), _Class("heavy", max_sims, self.device, torch)]
        self.in_use = 0
        self.peak_in_use = 0
        self.ticks = 0              # rounds
        self.batch_sizes = []       # simulations resident per round

    def _class_of(self, r: Request) -> _Class:
        return self.classes[0] if r.problem.ncell <= self.light_cells else self.classes[1]

    def _round_steps(self, c: _Class) -> int:
        if c.step_s is None:
            return 1
        return int(min(self.max_round_steps, max(1, round(self.round_s / c.step_s))))

    def run(self, requests: list[Request], clock=time.perf_counter) -> list[Result]:
        """Serve `requests` to completion; returns results in completion
        order. Arrival times are wall-clock offsets from the start of this
        call."""
        torch = self.torch
        pending = sorted(requests, key=lambda r: (r.arrival, r.rid))
        for r in pending:
            if footprint_bytes(r.problem, r.precision) > self.budget:
                raise ValueError(f"request {r.rid} does not fit the HBM budget")
        results: list[Result] = []
        t0 = clock()
        qi = 0
        while qi < len(pending) or any(c.active for c in self.classes):
            now = clock() - t0
            admitted = False
            while qi < len(pending) and pending[qi].arrival <= now:
                r = pending[qi]
                c = self._class_of(r)
                need = footprint_bytes(r.problem, r.precision)
                if len(c.active) >= c.max_sims or self.in_use + need > self.budget:
                    break
                sim = _Sim(r, self.device, torch)
                sim.need = need
                sim.admitted = now
                self.in_use += need
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                c.active.append(sim)
                c.changed = True
                admitted = True
                qi += 1
            if not any(c.active for c in self.classes):
                # idle until the next arrival
                if qi < len(pending):
                    wait = pending[qi].arrival - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.01))
                continue
            if admitted:
                # initial states are written on the default stream
                torch.cuda.synchronize(self.device)
            running = [c for c in self.classes if c.active]
            for c in running:
                if c.changed:
                    c.set_arrays()
                c.k = self._round_steps(c)
                c.t_before = np.array([s.t for s in c.active])
                c.n_before = np.array([s.steps for s in c.active], dtype=np.int64)
                c.ev = (torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                c.ev[0].record(c.stream)
                c.batch.advance_active(c.cfl_dx, c.t_end, c.max_steps, c.t_before, c.n_before, c.k)
                c.ev[1].record(c.stream)
            self.ticks += 1
            self.batch_sizes.append(sum(len(c.active) for c in running))
            for c in running:
                t, n = c.batch.clock_active()
                c.ev[1].synchronize()
                per = c.ev[0].elapsed_time(c.ev[1]) / 1e3 / c.k
                c.step_s = per if c.step_s is None else 0.7 * c.step_s + 0.3 * per
                for i, sim in enumerate(c.active):
                    sim.t = float(t[i])
                    sim.steps = int(n[i])
                done = np.where(c.max_steps >= 0, n >= c.max_steps, t >= c.t_end * (1.0 - 1e-14))
                # a simulation that took no step in a round it was due one
                # (non-finite time step, counted in its report) ends here
                stuck = (n == c.n_before) & ~done
                fin = done | stuck
                if fin.any():
                    end = clock() - t0
                    for sim, f in zip(c.active, fin):
                        if not f:
                            continue
                        results.append(Result(rid=sim.req.rid, U=sim.U.cpu().numpy(), steps=sim.steps, t=sim.t,
                                              arrival=sim.req.arrival, admitted=sim.admitted, finished=end,
                                              zone_updates=sim.steps * sim.req.problem.ncell,
                                              report=sim.solver.report()))
                        self.in_use -= sim.need
                        sim.close()
                    c.active = [sim for sim, f in zip(c.active, fin) if not f]
                    c.changed = True
        return results

    def close(self):
        for c in self.classes:
            c.close()


def percentile(values, q):
    v = np.sort(np.asarray(values, dtype=np.float64))
    if v.size == 0:
        return float("nan")
    return float(np.percentile(v, q))
