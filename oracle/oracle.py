"""ctypes wrapper of the plain FP64 CPU oracle (``rrmhd_oracle.cpp``).

TEST INFRASTRUCTURE ONLY: imported by the test suite, by the smoke check and
by the CPU-baseline leg of the benchmark. The GPU library never imports it.

Arrays are float64 structure-of-arrays ``[12, n]`` (variable planes), the
variable order being
  U: D, S_x, S_y, S_z, tau_e, B_x, B_y, B_z, E_r, F_x, F_y, F_z
  V: rho, v_x, v_y, v_z, p, B_x, B_y, B_z, E_r, F_x, F_y, F_z
(Section 2.1 of the paper).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "rrmhd_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")
LIB_COUNT = os.path.join(HERE, "liboracle_count.so")

_CFLAGS = ["-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = True) -> None:
    """Compile the oracle (OpenMP build and the op-counting build)."""
    if force or not os.path.exists(LIB):
        subprocess.check_call(["g++", *_CFLAGS, "-fopenmp", "-o", LIB, SRC])
    if force or not os.path.exists(LIB_COUNT):
        subprocess.check_call(["g++", *_CFLAGS, "-DORACLE_COUNT_OPS", "-o", LIB_COUNT, SRC])


class OPar(C.Structure):
    _fields_ = [
        ("gamma", C.c_double), ("a_rad", C.c_double), ("t_coeff", C.c_double),
        ("pvm_eps", C.c_double), ("c2p_tol", C.c_double), ("imp_tol", C.c_double),
        ("rho_floor", C.c_double), ("p_floor", C.c_double),
        ("pvm_k", C.c_int), ("beta_mode", C.c_int), ("recon", C.c_int), ("rk_order", C.c_int),
        ("c2p_maxit", C.c_int), ("imp_maxit", C.c_int), ("imp_picard_it", C.c_int),
        ("imp_method", C.c_int), ("e_floor", C.c_double), ("solver", C.c_int), ("ct", C.c_int),
    ]


class OGrid(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("n", C.c_int * 3), ("dx", C.c_double * 3),
        ("bc_lo", C.c_int * 3), ("bc_hi", C.c_int * 3), ("var_stride", C.c_longlong),
        ("inflow_U", C.c_void_p), ("inflow_mask", C.c_void_p),
    ]


class OReport(C.Structure):
    _fields_ = [
        ("c2p_fail", C.c_longlong), ("pvm_fallback", C.c_longlong), ("imp_fail", C.c_longlong),
        ("nonfinite", C.c_longlong), ("e_floor_hits", C.c_longlong), ("first_bad_cell", C.c_longlong),
        ("max_c2p_it", C.c_int), ("max_imp_it", C.c_int),
    ]


DEFAULTS = dict(
    gamma=5.0 / 3.0, a_rad=1.0, t_coeff=1.0, pvm_eps=1e-8, c2p_tol=1e-12, imp_tol=1e-13,
    rho_floor=1e-12, p_floor=1e-12, pvm_k=3, beta_mode=1, recon=1, rk_order=2,
    c2p_maxit=100, imp_maxit=50, imp_picard_it=8, imp_method=0, e_floor=0.0, solver=0, ct=0,
)

SOLVER_PVM, SOLVER_HLL, SOLVER_PVM_JVP = 0, 1, 2


def params(**kw) -> OPar:
    d = dict(DEFAULTS)
    d.update(kw)
    return OPar(**d)


_lib = None
_lib_count = None


def _dp(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _setup(lib):
    vp, ll, i, d = C.c_void_p, C.c_longlong, C.c_int, C.c_double
    lib.or_threads.argtypes = [i]; lib.or_threads.restype = i
    lib.or_p2c.argtypes = [ll, vp, ll, vp, vp, ll]; lib.or_p2c.restype = None
    lib.or_flux.argtypes = [ll, vp, ll, i, vp, vp, ll]; lib.or_flux.restype = None
    lib.or_c2p.argtypes = [ll, vp, ll, vp, vp, vp, ll, vp, vp, vp]; lib.or_c2p.restype = None
    lib.or_c2p_lw.argtypes = [ll, vp, ll, vp, vp, ll, vp, vp]; lib.or_c2p_lw.restype = None
    lib.or_c2p_eval.argtypes = [ll, vp, ll, vp, vp, vp]; lib.or_c2p_eval.restype = None
    lib.or_pvm_face.argtypes = [ll, vp, vp, ll, vp, vp, i, vp, vp, ll, vp, vp]; lib.or_pvm_face.restype = None
    lib.or_hll_face.argtypes = [ll, vp, vp, ll, vp, vp, i, vp, vp, ll, vp]; lib.or_hll_face.restype = None
    lib.or_fast_speeds.argtypes = [ll, vp, ll, i, vp, vp, vp, vp]; lib.or_fast_speeds.restype = None
    lib.or_rad_speeds.argtypes = [ll, vp, ll, i, vp, vp]; lib.or_rad_speeds.restype = None
    lib.or_quartic.argtypes = [ll, vp, ll, i, vp, vp, vp]; lib.or_quartic.restype = None
    lib.or_jvp.argtypes = [ll, vp, vp, ll, i, vp, vp, ll, vp]; lib.or_jvp.restype = None
    lib.or_poly_coef.argtypes = [i, vp]; lib.or_poly_coef.restype = i
    lib.or_implicit.argtypes = [ll, vp, ll, vp, vp, vp, vp, vp, ll, vp, vp]; lib.or_implicit.restype = None
    lib.or_four_force.argtypes = [ll, vp, ll, vp, vp, vp, vp, ll]; lib.or_four_force.restype = None
    lib.or_cell_speed.argtypes = [ll, vp, ll, i, vp, vp]; lib.or_cell_speed.restype = None
    lib.or_max_speed.argtypes = [vp, vp, vp, vp]; lib.or_max_speed.restype = d
    lib.or_step.argtypes = [vp, vp, vp, vp, vp, d, d, d, vp]; lib.or_step.restype = i
    lib.or_face_fluxes.argtypes = [vp, vp, vp, vp, vp, d, d, vp]; lib.or_face_fluxes.restype = ll
    lib.or_explicit_stage.argtypes = [vp, vp, vp, vp, vp, vp, d, d, d, d, d, d, vp]; lib.or_explicit_stage.restype = ll
    return lib


def lib(count: bool = False):
    global _lib, _lib_count
    if count:
        if _lib_count is None:
            if not os.path.exists(LIB_COUNT):
                build(force=False)
            _lib_count = _setup(C.CDLL(LIB_COUNT))
            _lib_count.or_opcount_reset.argtypes = []
            _lib_count.or_opcount_get.argtypes = [C.c_void_p]
            _lib_count.or_opcount_get_newton.argtypes = [C.c_void_p]
        return _lib_count
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        _lib = _setup(C.CDLL(LIB))
    return _lib


def threads(n: int = 0) -> int:
    return lib().or_threads(n)


def _soa(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.ndim == 2 and a.shape[0] == 12
    return a


def _state(a):
    """A grid state: the 12 conserved planes, plus with constrained transport
    one staggered normal-field plane per grid dimension (the face on the lower
    side of each cell)."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.ndim == 2 and 12 <= a.shape[0] <= 15
    return a


def p2c(V, par=None):
    V = _soa(V); n = V.shape[1]
    U = np.empty_like(V)
    par = par or params()
    lib().or_p2c(n, _dp(V), n, C.byref(par), _dp(U), n)
    return U


def flux(V, d, par=None):
    V = _soa(V); n = V.shape[1]
    F = np.empty_like(V)
    par = par or params()
    lib().or_flux(n, _dp(V), n, d, C.byref(par), _dp(F), n)
    return F


def c2p(U, par=None, Z_in=None):
    U = _soa(U); n = U.shape[1]
    V = np.empty_like(U)
    Z = np.zeros(n); st = np.zeros(n, np.int32); it = np.zeros(n, np.int32)
    par = par or params()
    zin = None if Z_in is None else np.ascontiguousarray(Z_in, dtype=np.float64)
    lib().or_c2p(n, _dp(U), n, C.byref(par), _dp(zin), _dp(V), n, _dp(Z), _dp(st), _dp(it))
    return V, Z, st, it


def c2p_lw(U, par=None):
    """Cold-start recovery; returns (V, [1 - v^2, 1/W] as the recovery formed
    them, status)."""
    U = _soa(U); n = U.shape[1]
    V = np.empty_like(U); lw = np.zeros((2, n)); st = np.zeros(n, np.int32)
    par = par or params()
    lib().or_c2p_lw(n, _dp(U), n, C.byref(par), _dp(V), n, _dp(lw), _dp(st))
    return V, lw, st


def c2p_eval(U, Z, par=None):
    """One evaluation of the recovery residual at Z per state: dict of arrays
    ok, l2 (1 - v^2), iW (1/W), iZ, iZb (1/(Z + B^2)), fW (f/W), dfW (f'/W),
    rho, p."""
    U = _soa(U); n = U.shape[1]
    Z = np.ascontiguousarray(np.broadcast_to(Z, (n,)), dtype=np.float64)
    out = np.zeros((9, n))
    par = par or params()
    lib().or_c2p_eval(n, _dp(U), n, _dp(Z), C.byref(par), _dp(out))
    keys = ["ok", "l2", "iW", "iZ", "iZb", "fW", "dfW", "rho", "p"]
    return {k: out[i] for i, k in enumerate(keys)}


def pvm_face(VL, VR, tauL, tauR, d, par=None):
    VL = _soa(VL); VR = _soa(VR); n = VL.shape[1]
    assert VR.shape == VL.shape
    tauL = np.ascontiguousarray(np.broadcast_to(tauL, (n,)), dtype=np.float64)
    tauR = np.ascontiguousarray(np.broadcast_to(tauR, (n,)), dtype=np.float64)
    Fh = np.empty_like(VL)
    fb = np.zeros(n, np.int32); its = np.zeros(n, np.int32)
    par = par or params()
    lib().or_pvm_face(n, _dp(VL), _dp(VR), n, _dp(tauL), _dp(tauR), d, C.byref(par), _dp(Fh), n,
                      _dp(fb), _dp(its))
    return Fh, fb, its


def hll_face(VL, VR, tauL, tauR, d, par=None):
    """Rad-HLL face flux; returns (F^, Newton steps of the four quartic roots)."""
    VL = _soa(VL); VR = _soa(VR); n = VL.shape[1]
    assert VR.shape == VL.shape
    tauL = np.ascontiguousarray(np.broadcast_to(tauL, (n,)), dtype=np.float64)
    tauR = np.ascontiguousarray(np.broadcast_to(tauR, (n,)), dtype=np.float64)
    Fh = np.empty_like(VL)
    its = np.zeros(n, np.int32)
    par = par or params()
    lib().or_hll_face(n, _dp(VL), _dp(VR), n, _dp(tauL), _dp(tauR), d, C.byref(par), _dp(Fh), n, _dp(its))
    return Fh, its


def fast_speeds(V, d, par=None):
    """(lambda_min, lambda_max, Newton steps) of the magnetofluid block per state."""
    V = _soa(V); n = V.shape[1]
    lo = np.empty(n); hi = np.empty(n); its = np.zeros(n, np.int32)
    par = par or params()
    lib().or_fast_speeds(n, _dp(V), n, d, C.byref(par), _dp(lo), _dp(hi), _dp(its))
    return lo, hi, its


def jvp(U, w, d, par=None):
    """Exact A(U) w (forward mode through the recovery) per state; (Aw, status)."""
    U = _soa(U); w = _soa(w); n = U.shape[1]
    assert w.shape == U.shape
    Aw = np.empty_like(U); st = np.zeros(n, np.int32)
    par = par or params()
    lib().or_jvp(n, _dp(U), _dp(w), n, d, C.byref(par), _dp(Aw), n, _dp(st))
    return Aw, st


def quartic(V, d, lam, par=None):
    """(Q, Q', Q'') of the RMHD quartic of each state at lam (array [3, n])."""
    V = _soa(V); n = V.shape[1]
    lam = np.ascontiguousarray(np.broadcast_to(lam, (n,)), dtype=np.float64)
    out = np.empty((3, n))
    par = par or params()
    lib().or_quartic(n, _dp(V), n, d, C.byref(par), _dp(lam), _dp(out))
    return out


def rad_speeds(V, d):
    """(lambda_r1, lambda_r3) of the M1 radiation block per state."""
    V = _soa(V); n = V.shape[1]
    l1 = np.empty(n); l3 = np.empty(n)
    lib().or_rad_speeds(n, _dp(V), n, d, _dp(l1), _dp(l3))
    return l1, l3


def poly_coef(k):
    c = np.zeros(17)
    M = lib().or_poly_coef(k, _dp(c))
    return c[: M + 1].copy()


def implicit(Us, h, kap, sig, par=None):
    Us = _soa(Us); n = Us.shape[1]
    b = lambda x: np.ascontiguousarray(np.broadcast_to(x, (n,)), dtype=np.float64)
    h, kap, sig = b(h), b(kap), b(sig)
    Un = np.empty_like(Us)
    st = np.zeros(n, np.int32); it = np.zeros(n, np.int32)
    par = par or params()
    lib().or_implicit(n, _dp(Us), n, _dp(h), _dp(kap), _dp(sig), C.byref(par), _dp(Un), n,
                      _dp(st), _dp(it))
    return Un, st, it


def four_force(V, kap, sig, par=None):
    V = _soa(V); n = V.shape[1]
    b = lambda x: np.ascontiguousarray(np.broadcast_to(x, (n,)), dtype=np.float64)
    G = np.empty((4, n))
    par = par or params()
    lib().or_four_force(n, _dp(V), n, _dp(b(kap)), _dp(b(sig)), C.byref(par), _dp(G), n)
    return G


def cell_speed(V, d, par=None):
    V = _soa(V); n = V.shape[1]
    s = np.empty(n)
    par = par or params()
    lib().or_cell_speed(n, _dp(V), n, d, C.byref(par), _dp(s))
    return s


def make_grid(shape, dx, bc_lo=(1, 1, 1), bc_hi=(1, 1, 1), inflow_U=None, inflow_mask=None):
    """shape: interior cells per axis (x first). bc: 0 periodic, 1 outflow, 2 inflow."""
    g = OGrid()
    g.ndim = len(shape)
    n = list(shape) + [1] * (3 - len(shape))
    dxs = list(dx) + [1.0] * (3 - len(dx))
    for e in range(3):
        g.n[e] = n[e]; g.dx[e] = dxs[e]; g.bc_lo[e] = bc_lo[e]; g.bc_hi[e] = bc_hi[e]
    g.var_stride = int(np.prod(shape))
    g._keep = (inflow_U, inflow_mask)
    g.inflow_U = inflow_U.ctypes.data if inflow_U is not None else None
    g.inflow_mask = inflow_mask.ctypes.data if inflow_mask is not None else None
    return g


def _opac(kap, sig, ncell):
    ka = kap if isinstance(kap, np.ndarray) else None
    sa = sig if isinstance(sig, np.ndarray) else None
    k0 = 0.0 if ka is not None else float(kap)
    s0 = 0.0 if sa is not None else float(sig)
    if ka is not None:
        ka = np.ascontiguousarray(ka, dtype=np.float64).reshape(-1); assert ka.size == ncell
    if sa is not None:
        sa = np.ascontiguousarray(sa, dtype=np.float64).reshape(-1); assert sa.size == ncell
    return ka, sa, k0, s0


def step(grid, U, dt, kap, sig, par=None):
    """One IMEX step; U is [12, ncell] (x fastest; [12 + ndim, ncell] with
    constrained transport) and is not modified."""
    U = np.array(_state(U), copy=True)
    ncell = U.shape[1]
    assert ncell == grid.var_stride
    ka, sa, k0, s0 = _opac(kap, sig, ncell)
    rep = OReport()
    par = par or params()
    st = lib().or_step(C.byref(grid), C.byref(par), _dp(U), _dp(ka), _dp(sa), k0, s0, float(dt),
                       C.byref(rep))
    return U, st, rep


def max_speed(grid, U, par=None):
    U = _state(U)
    nf = C.c_longlong(0)
    par = par or params()
    s = lib().or_max_speed(C.byref(grid), C.byref(par), _dp(U), C.byref(nf))
    return s, nf.value


def face_fluxes(grid, U, kap, sig, par=None):
    U = _state(U)
    ncell = U.shape[1]
    ka, sa, k0, s0 = _opac(kap, sig, ncell)
    n = [grid.n[e] for e in range(3)]
    sizes = []
    for d in range(grid.ndim):
        m = list(n); m[d] += 1
        sizes.append(int(np.prod(m)))
    out = np.zeros(12 * sum(sizes))
    par = par or params()
    nfb = lib().or_face_fluxes(C.byref(grid), C.byref(par), _dp(U), _dp(ka), _dp(sa), k0, s0, _dp(out))
    res, off = [], 0
    for s in sizes:
        res.append(out[off: off + 12 * s].reshape(12, s)); off += 12 * s
    return res, nfb


def explicit_stage(grid, U0, Us, kap, sig, a0, a1, c, dt, par=None):
    """U* = a0 U0 + a1 Us - c dt sum_d dF^/dx_d (fluxes from Us)."""
    U0 = _soa(U0); Us = _soa(Us)
    ka, sa, k0, s0 = _opac(kap, sig, U0.shape[1])
    out = np.empty_like(U0)
    par = par or params()
    nbad = lib().or_explicit_stage(C.byref(grid), C.byref(par), _dp(U0), _dp(Us), _dp(ka), _dp(sa), k0, s0,
                                   float(a0), float(a1), float(c), float(dt), _dp(out))
    return out, nbad


def count_ops(fn, *args, **kw):
    """Run ``fn(lib_count, ...)`` and return (result, {add, mul, div, sqrt})."""
    L = lib(count=True)
    L.or_opcount_reset()
    r = fn(L, *args, **kw)
    out = (C.c_ulonglong * 4)()
    L.or_opcount_get(out)
    return r, dict(add=out[0], mul=out[1], div=out[2], sqrt=out[3])
