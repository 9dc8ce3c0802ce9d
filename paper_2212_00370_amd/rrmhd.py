"""Thin ctypes binding of ``librrmhd.so`` (the C ABI declared in
``include/rrmhd.h``). Argument marshalling only: every step of the method runs
in the library's HIP kernels. PyTorch provides device memory and streams.

There is no CPU fallback: importing this module raises if the library has not
been built.
"""
from __future__ import annotations

import ctypes as C
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "librrmhd.so")

NVAR = 12
RRMHD_OK, RRMHD_E_INVALID, RRMHD_E_C2P, RRMHD_E_IMPLICIT = 0, -1, -2, -3
RRMHD_E_NONFINITE, RRMHD_E_DEVICE, RRMHD_E_WORKSPACE = -4, -5, -6
BC_PERIODIC, BC_OUTFLOW, BC_INFLOW = 0, 1, 2
RECON_GODUNOV, RECON_MINMOD, RECON_MC, RECON_VANLEER = 0, 1, 2, 3
SOLVER_PVM, SOLVER_HLL, SOLVER_PVM_JVP = 0, 1, 2
BETA_ALL, BETA_RAD_ONLY, BETA_OFF = 0, 1, 2
IMP_PICARD_NEWTON, IMP_NEWTON, IMP_PICARD = 0, 1, 2
FP64, MIXED = 0, 1
K_PRIMS, K_FACES, K_UPDATE, K_SPEED, K_NEWTON, K_COUNT = 0, 1, 2, 3, 4, 5
PROFILE_ALL = (1 << K_COUNT) - 1


class rrmhd_grid(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3),
        ("bc_lo", C.c_int * 3), ("bc_hi", C.c_int * 3), ("var_stride", C.c_longlong),
        ("inflow_U", C.c_void_p), ("inflow_mask", C.c_void_p),
    ]


class rrmhd_params(C.Structure):
    _fields_ = [
        ("gamma", C.c_double), ("a_rad", C.c_double), ("t_coeff", C.c_double),
        ("pvm_eps", C.c_double), ("c2p_tol", C.c_double), ("imp_tol", C.c_double),
        ("rho_floor", C.c_double), ("p_floor", C.c_double),
        ("pvm_k", C.c_int), ("beta_mode", C.c_int), ("recon", C.c_int), ("rk_order", C.c_int),
        ("c2p_maxit", C.c_int), ("imp_maxit", C.c_int), ("imp_picard_it", C.c_int),
        ("imp_method", C.c_int), ("precision", C.c_int), ("pvm_eps_mixed", C.c_double),
        ("e_floor", C.c_double), ("solver", C.c_int), ("ct", C.c_int),
    ]


class rrmhd_opacities(C.Structure):
    _fields_ = [("kappa", C.c_void_p), ("sigma", C.c_void_p), ("kappa0", C.c_double), ("sigma0", C.c_double)]


class rrmhd_report(C.Structure):
    _fields_ = [
        ("c2p_fail", C.c_longlong), ("pvm_fallback", C.c_longlong), ("imp_fail", C.c_longlong),
        ("nonfinite", C.c_longlong), ("e_floor_hits", C.c_longlong), ("first_bad_cell", C.c_longlong),
        ("max_c2p_it", C.c_int), ("max_imp_it", C.c_int),
    ]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


# Exported symbols and their signatures (kept in the order of rrmhd.h).
_vp, _ll, _d = C.c_void_p, C.c_longlong, C.c_double
SIGNATURES = {
    "rrmhd_default_params": ([_vp], None),
    "rrmhd_workspace_bytes": ([_vp, _vp], C.c_size_t),
    "rrmhd_init": ([_vp, _vp, _vp, _vp, C.c_size_t, _vp], C.c_int),
    "rrmhd_prim_to_cons": ([_vp, _vp, _vp], C.c_int),
    "rrmhd_cons_to_prim": ([_vp, _vp, _vp], C.c_int),
    "rrmhd_step": ([_vp, _vp, _vp, _d, _vp], C.c_int),
    "rrmhd_max_speed": ([_vp, _vp, _vp, _vp], C.c_int),
    "rrmhd_advance": ([_vp, _vp, _vp, _d, C.c_int, _vp, _vp], C.c_int),
    "rrmhd_advance_noalloc": ([_vp, _vp, _vp, _d, C.c_int, _vp, _vp, _vp, _vp], C.c_int),
    "rrmhd_face_fluxes": ([_vp, _vp, _vp, _vp], C.c_int),
    "rrmhd_profile_enable": ([_vp, C.c_int], C.c_int),
    "rrmhd_profile_stride": ([_vp, C.c_int], C.c_int),
    "rrmhd_profile_read": ([_vp, C.c_int, _vp, _vp, _vp], C.c_int),
    "rrmhd_report_sync": ([_vp, _vp], C.c_int),
    "rrmhd_batch_workspace_bytes": ([C.c_int], C.c_size_t),
    "rrmhd_batch_init": ([_vp, C.c_int, _vp, C.c_size_t, _vp], C.c_int),
    "rrmhd_max_speed_batch": ([_vp, C.c_int, _vp, _vp, _vp], C.c_int),
    "rrmhd_step_batch": ([_vp, C.c_int, _vp, _vp, _vp, _vp], C.c_int),
    "rrmhd_advance_batch": ([_vp, C.c_int, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, C.c_int], C.c_int),
    "rrmhd_batch_clock": ([_vp, C.c_int, _vp, _vp], C.c_int),
    "rrmhd_batch_destroy": ([_vp], None),
    "rrmhd_destroy": ([_vp], None),
    "rrmhd_strerror": ([C.c_int], C.c_char_p),
}


def load(path: str = LIB_PATH):
    if not os.path.exists(path):
        raise ImportError(f"{path} not built: run paper_2212_00370_amd.build.build() "
                          "(hipcc --offload-arch=gfx950); there is no CPU fallback")
    lib = C.CDLL(path)
    for name, (args, res) in SIGNATURES.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = res
    return lib


_lib = load()


class RRMHDError(RuntimeError):
    pass


def _check(st: int, what: str) -> None:
    if st != RRMHD_OK:
        raise RRMHDError(f"{what}: {_lib.rrmhd_strerror(st).decode()} ({st})")


def _ptr(t) -> int | None:
    return None if t is None else t.data_ptr()


# ---- entry points, same names as the C ABI --------------------------------------
def rrmhd_default_params(**overrides) -> rrmhd_params:
    p = rrmhd_params()
    _lib.rrmhd_default_params(C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def rrmhd_workspace_bytes(grid: rrmhd_grid, params: rrmhd_params) -> int:
    return int(_lib.rrmhd_workspace_bytes(C.byref(grid), C.byref(params)))


def rrmhd_init(grid: rrmhd_grid, params: rrmhd_params, workspace, stream=None):
    """workspace: a CUDA (HIP) uint8 tensor of at least rrmhd_workspace_bytes."""
    ctx = C.c_void_p()
    st = _lib.rrmhd_init(C.byref(ctx), C.byref(grid), C.byref(params), _ptr(workspace),
                         workspace.numel() * workspace.element_size(),
                         None if stream is None else C.c_void_p(stream.cuda_stream))
    _check(st, "rrmhd_init")
    return ctx


def rrmhd_prim_to_cons(ctx, V, U) -> None:
    _check(_lib.rrmhd_prim_to_cons(ctx, _ptr(V), _ptr(U)), "rrmhd_prim_to_cons")


def rrmhd_cons_to_prim(ctx, U, V) -> None:
    _check(_lib.rrmhd_cons_to_prim(ctx, _ptr(U), _ptr(V)), "rrmhd_cons_to_prim")


def rrmhd_step(ctx, U, grid: rrmhd_grid, dt: float, opac: rrmhd_opacities) -> None:
    _check(_lib.rrmhd_step(ctx, _ptr(U), C.byref(grid), float(dt), C.byref(opac)), "rrmhd_step")


def rrmhd_advance(ctx, U, grid: rrmhd_grid, cfl: float, nsteps: int, opac: rrmhd_opacities, dt_out=None) -> None:
    """nsteps steps with the time step formed on the device; enqueued.
    dt_out: optional device tensor of nsteps float64 receiving each dt."""
    if dt_out is not None:
        import torch
        assert dt_out.dtype == torch.float64 and dt_out.is_cuda and dt_out.numel() >= nsteps
    _check(_lib.rrmhd_advance(ctx, _ptr(U), C.byref(grid), float(cfl), int(nsteps), C.byref(opac),
                              None if dt_out is None else _ptr(dt_out)), "rrmhd_advance")


def rrmhd_advance_noalloc(grid: rrmhd_grid, params: rrmhd_params, U, cfl: float, nsteps: int,
                          opac: rrmhd_opacities, dt_out=None, report_dev=None, stream=None) -> None:
    """rrmhd_advance without a context or workspace (the library's per-device
    scratch array); enqueued. report_dev: optional device tensor of at least
    sizeof(rrmhd_report) bytes receiving the call's failure counters."""
    if dt_out is not None:
        import torch
        assert dt_out.dtype == torch.float64 and dt_out.is_cuda and dt_out.numel() >= nsteps
    if report_dev is not None:
        assert report_dev.is_cuda and report_dev.numel() * report_dev.element_size() >= C.sizeof(rrmhd_report)
    _check(_lib.rrmhd_advance_noalloc(C.byref(grid), C.byref(params), _ptr(U), float(cfl), int(nsteps),
                                      C.byref(opac), None if dt_out is None else _ptr(dt_out),
                                      None if report_dev is None else _ptr(report_dev),
                                      None if stream is None else C.c_void_p(stream.cuda_stream)),
           "rrmhd_advance_noalloc")


def report_from_bytes(raw: bytes) -> dict:
    """The rrmhd_report written by rrmhd_advance_noalloc, from its bytes."""
    return rrmhd_report.from_buffer_copy(raw[: C.sizeof(rrmhd_report)]).as_dict()


def rrmhd_max_speed(ctx, U, grid: rrmhd_grid) -> float:
    out = C.c_double(0.0)
    _check(_lib.rrmhd_max_speed(ctx, _ptr(U), C.byref(grid), C.byref(out)), "rrmhd_max_speed")
    return out.value


def rrmhd_face_fluxes(ctx, U, opac: rrmhd_opacities, Fh) -> None:
    _check(_lib.rrmhd_face_fluxes(ctx, _ptr(U), C.byref(opac), _ptr(Fh)), "rrmhd_face_fluxes")


def rrmhd_profile_enable(ctx, enable=True) -> None:
    """enable: True (every kernel class), False (off) or a bit mask of
    (1 << K_*) classes."""
    mask = (PROFILE_ALL if enable else 0) if isinstance(enable, bool) else int(enable)
    _check(_lib.rrmhd_profile_enable(ctx, mask), "rrmhd_profile_enable")


def rrmhd_profile_stride(ctx, stride: int) -> None:
    _check(_lib.rrmhd_profile_stride(ctx, int(stride)), "rrmhd_profile_stride")


def rrmhd_profile_read(ctx, k: int):
    """(total_ms, launches, units) of the timed launches of kernel class k."""
    ms, n, u = C.c_double(0.0), C.c_longlong(0), C.c_longlong(0)
    _check(_lib.rrmhd_profile_read(ctx, int(k), C.byref(ms), C.byref(n), C.byref(u)), "rrmhd_profile_read")
    return ms.value, n.value, u.value


def rrmhd_report_sync(ctx) -> dict:
    r = rrmhd_report()
    _check(_lib.rrmhd_report_sync(ctx, C.byref(r)), "rrmhd_report_sync")
    return r.as_dict()


def rrmhd_batch_workspace_bytes(max_sims: int) -> int:
    return int(_lib.rrmhd_batch_workspace_bytes(int(max_sims)))


def rrmhd_batch_init(max_sims: int, workspace, stream=None):
    bh = C.c_void_p()
    st = _lib.rrmhd_batch_init(C.byref(bh), int(max_sims), _ptr(workspace),
                               workspace.numel() * workspace.element_size(),
                               None if stream is None else C.c_void_p(stream.cuda_stream))
    _check(st, "rrmhd_batch_init")
    return bh


def rrmhd_max_speed_batch(batch, ctxs, Us):
    n = len(ctxs)
    cv = (C.c_void_p * n)(*[c.value for c in ctxs])
    uv = (C.c_void_p * n)(*[u.data_ptr() for u in Us])
    out = (C.c_double * n)()
    _check(_lib.rrmhd_max_speed_batch(batch, n, cv, uv, out), "rrmhd_max_speed_batch")
    return list(out)


def rrmhd_step_batch(batch, ctxs, Us, dts, opacs) -> None:
    n = len(ctxs)
    cv = (C.c_void_p * n)(*[c.value for c in ctxs])
    uv = (C.c_void_p * n)(*[u.data_ptr() for u in Us])
    dv = (C.c_double * n)(*[float(x) for x in dts])
    ov = (C.c_void_p * n)(*[C.addressof(o) for o in opacs])
    _check(_lib.rrmhd_step_batch(batch, n, cv, uv, dv, ov), "rrmhd_step_batch")


def rrmhd_batch_destroy(batch) -> None:
    _lib.rrmhd_batch_destroy(batch)


def rrmhd_destroy(ctx) -> None:
    _lib.rrmhd_destroy(ctx)


def rrmhd_strerror(st: int) -> str:
    return _lib.rrmhd_strerror(st).decode()


# ---- helpers for building the C structs -------------------------------------------
def make_grid(shape, dx, bc_lo=(BC_OUTFLOW,) * 3, bc_hi=(BC_OUTFLOW,) * 3, var_stride=None,
              inflow_U=None, inflow_mask=None) -> rrmhd_grid:
    g = rrmhd_grid()
    g.ndim = len(shape)
    n = list(shape) + [1] * (3 - len(shape))
    dxs = list(dx) + [1.0] * (3 - len(dx))
    for e in range(3):
        g.n[e] = int(n[e]); g.dx[e] = float(dxs[e])
        g.bc_lo[e] = int(bc_lo[e]); g.bc_hi[e] = int(bc_hi[e])
    ncell = int(n[0] * n[1] * n[2])
    g.var_stride = ncell if var_stride is None else int(var_stride)
    g.inflow_U = _ptr(inflow_U)
    g.inflow_mask = _ptr(inflow_mask)
    g._keep = (inflow_U, inflow_mask)
    return g


def make_opacities(kappa=None, sigma=None, kappa0=0.0, sigma0=0.0) -> rrmhd_opacities:
    o = rrmhd_opacities()
    o.kappa = _ptr(kappa); o.sigma = _ptr(sigma)
    o.kappa0 = float(kappa0); o.sigma0 = float(sigma0)
    o._keep = (kappa, sigma)
    return o


class Batch:
    """Device descriptor table for stepping many Solvers with one launch per
    kernel class (rrmhd_step_batch)."""

    def __init__(self, max_sims: int, device="cuda:0", stream=None):
        import torch
        nbytes = rrmhd_batch_workspace_bytes(max_sims)
        if nbytes == 0:
            raise RRMHDError("invalid max_sims")
        self.max_sims = max_sims
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[off: off + nbytes]
        self.handle = rrmhd_batch_init(max_sims, self.ws, stream)

    def max_speed(self, solvers, Us):
        return rrmhd_max_speed_batch(self.handle, [s.ctx for s in solvers], Us)

    def step(self, solvers, Us, dts, opacs):
        rrmhd_step_batch(self.handle, [s.ctx for s in solvers], Us, dts, opacs)

    # A fixed active set: its pointer arrays are built once (set_active) and
    # each tick marshals only the time steps. The library keeps the device
    # descriptor table of an unchanged set and uploads only those.
    def set_active(self, solvers, Us, opacs):
        n = len(solvers)
        self._n = n
        self._cv = (C.c_void_p * n)(*[s.ctx.value for s in solvers])
        self._uv = (C.c_void_p * n)(*[u.data_ptr() for u in Us])
        self._ov = (C.c_void_p * n)(*[C.addressof(o) for o in opacs])
        self._keep = (list(Us), list(opacs))
        self._out = (C.c_double * n)()
        self._dv = (C.c_double * n)()

    def max_speed_active(self):
        """Signal speeds of the active set, as a numpy view of the result
        buffer (valid until the next call)."""
        import numpy as np
        _check(_lib.rrmhd_max_speed_batch(self.handle, self._n, self._cv, self._uv, self._out),
               "rrmhd_max_speed_batch")
        return np.ctypeslib.as_array(self._out)

    def step_active(self, dts):
        import numpy as np
        np.ctypeslib.as_array(self._dv)[:] = dts
        _check(_lib.rrmhd_step_batch(self.handle, self._n, self._cv, self._uv, self._dv, self._ov),
               "rrmhd_step_batch")

    def advance_active(self, cfl_dx, t_end, max_steps, t, n, nsteps: int) -> None:
        """Enqueue up to `nsteps` steps of each simulation of the active set
        with its own CFL time step on the device (rrmhd_advance_batch).
        cfl_dx, t_end, t: float64 arrays; max_steps, n: int64 arrays (< 0
        max_steps: run to t_end). Read the clock with clock_active()."""
        import numpy as np
        arrs = [np.ascontiguousarray(a, dtype=dt) for a, dt in
                ((cfl_dx, np.float64), (t_end, np.float64), (max_steps, np.int64), (t, np.float64), (n, np.int64))]
        for a in arrs:
            if a.shape != (self._n,):
                raise RRMHDError("advance_active: one value per simulation of the active set")
        self._clock_keep = arrs
        _check(_lib.rrmhd_advance_batch(self.handle, self._n, self._cv, self._uv, self._ov,
                                        *[a.ctypes.data for a in arrs], int(nsteps)), "rrmhd_advance_batch")

    def clock_active(self):
        """(t, n) of the active set after the last advance_active (waits for
        it)."""
        import numpy as np
        t = np.empty(self._n, np.float64)
        n = np.empty(self._n, np.int64)
        _check(_lib.rrmhd_batch_clock(self.handle, self._n, t.ctypes.data, n.ctypes.data), "rrmhd_batch_clock")
        return t, n

    def close(self):
        if self.handle is not None:
            rrmhd_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Solver:
    """Device-resident state of one problem: U, opacities and workspace as torch
    tensors on ``device``; each method is one C-ABI call."""

    def __init__(self, grid: rrmhd_grid, params: rrmhd_params, device="cuda:0", stream=None):
        import torch
        self.torch = torch
        self.grid = grid
        self.params = params
        self.device = torch.device(device)
        nbytes = rrmhd_workspace_bytes(grid, params)
        if nbytes == 0:
            raise RRMHDError("invalid grid or parameters")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self.ws = self.workspace[off: off + nbytes]
        self.stream = stream
        self.ctx = rrmhd_init(grid, params, self.ws, stream)

    def close(self):
        if self.ctx is not None:
            rrmhd_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def prim_to_cons(self, V):
        U = self.torch.empty_like(V)
        rrmhd_prim_to_cons(self.ctx, V, U)
        return U

    def cons_to_prim(self, U):
        V = self.torch.empty_like(U)
        rrmhd_cons_to_prim(self.ctx, U, V)
        return V

    def step(self, U, dt, opac):
        rrmhd_step(self.ctx, U, self.grid, dt, opac)

    def max_speed(self, U):
        return rrmhd_max_speed(self.ctx, U, self.grid)

    def advance(self, U, cfl, nsteps, opac, dt_out=None):
        rrmhd_advance(self.ctx, U, self.grid, cfl, nsteps, opac, dt_out)

    def face_fluxes(self, U, opac):
        sizes = []
        n = [self.grid.n[e] for e in range(3)]
        for d in range(self.grid.ndim):
            m = list(n); m[d] += 1
            sizes.append(m[0] * m[1] * m[2])
        out = self.torch.empty(NVAR * sum(sizes), dtype=self.torch.float64, device=self.device)
        rrmhd_face_fluxes(self.ctx, U, opac, out)
        res, off = [], 0
        for s in sizes:
            res.append(out[off: off + NVAR * s].view(NVAR, s)); off += NVAR * s
        return res

    def report(self):
        return rrmhd_report_sync(self.ctx)
