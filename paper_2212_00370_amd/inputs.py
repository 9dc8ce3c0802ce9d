"""Seeded synthetic inputs (primitive states, opacities, grid parameters).

This module holds no arithmetic of the method: it only draws initial states
with numpy's PCG64 generator and returns primitive arrays ``[12, ncell]``
(rho, v_x, v_y, v_z, p, B_x, B_y, B_z, E_r, F_x, F_y, F_z; x fastest), per-cell
opacities and the run parameters. Both the GPU path and the CPU oracle start
from these arrays, each converting primitives to conserved variables with its
own code.

Workloads (shapes and value ranges of the paper's test problems, Section 4):
  * ``riemann_1d``  -- seeded piecewise-constant RRMHD+M1 Riemann problems on
    [0, 1] (400 cells by default), outflow boundaries, gamma = 5/3.
  * ``blast_2d``    -- magnetised cylindrical blast (overpressure 1e3 inside
    r < 0.1) on [-1/2, 1/2]^2, smooth 1 % density perturbation, oblique
    B = 0.5, equilibrium radiation, opacity field spanning free streaming to
    diffusion, periodic boundaries, gamma = 4/3.
  * ``beam_3d``     -- relativistic magnetised beam (Lorentz factor 7) injected
    through a nozzle in the z = 0 face into an optically thick ambient medium,
    outflow elsewhere.
  * ``alfven_1d``   -- the large-amplitude circularly polarised Alfven wave of
    Section 4.1 (no radiation coupling), periodic on [0, 2 pi], gamma = 4/3.
  * ``serving_mix`` -- request mixes for the serving loop.
  * ``random_prims`` -- i.i.d. admissible states for unit-level checks.
  * ``alfven_2d``, ``field_loop_2d`` -- periodic 2D problems for constrained
    transport (staggered face fields in ``extra["bface"]``).

For constrained transport a problem also carries the staggered normal field
``extra["bface"]`` ``[ndim, ncell]``: row a holds b_a on the face on the lower
side of each cell along a, with the cell-centred B_a of ``V`` the mean of its
cell's two face values.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NV = 12
PERIODIC, OUTFLOW, INFLOW = 0, 1, 2


@dataclass
class Problem:
    name: str
    shape: tuple            # interior cells per axis, x first
    dx: tuple
    x0: tuple
    V: np.ndarray           # [12, ncell] primitives
    kappa: np.ndarray       # [ncell]
    sigma: np.ndarray       # [ncell]
    gamma: float
    a_rad: float
    t_coeff: float = 1.0
    bc_lo: tuple = (OUTFLOW, OUTFLOW, OUTFLOW)
    bc_hi: tuple = (OUTFLOW, OUTFLOW, OUTFLOW)
    cfl: float = 0.4
    t_end: float | None = None
    steps: int | None = None
    extra: dict = field(default_factory=dict)

    @property
    def ncell(self) -> int:
        return int(np.prod(self.shape))

    @property
    def ndim(self) -> int:
        return len(self.shape)


def _log_uniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def _unit_vectors(rng, n):
    v = rng.normal(size=(3, n))
    v /= np.linalg.norm(v, axis=0, keepdims=True)
    return v


def random_prims(seed: int, n: int, *, rho=(0.1, 10.0), p=(0.01, 10.0), vmax=0.9, bmax=2.0,
                 er=(1e-3, 10.0), fmax=1.0, zero_flux_frac=0.0) -> np.ndarray:
    """I.i.d. admissible primitive states: log-uniform rho, p, E_r; |v| < vmax
    in a uniform direction; |B| < bmax; F_r = f E_r m with f ~ U[0, fmax)."""
    rng = np.random.default_rng(seed)
    V = np.zeros((NV, n))
    V[0] = _log_uniform(rng, *rho, n)
    V[1:4] = _unit_vectors(rng, n) * rng.uniform(0.0, vmax, n)
    V[4] = _log_uniform(rng, *p, n)
    V[5:8] = _unit_vectors(rng, n) * rng.uniform(0.0, bmax, n)
    V[8] = _log_uniform(rng, *er, n)
    f = rng.uniform(0.0, fmax, n)
    if zero_flux_frac > 0:
        f[rng.uniform(size=n) < zero_flux_frac] = 0.0
    V[9:12] = _unit_vectors(rng, n) * (f * V[8])
    return V


def riemann_states(seed: int) -> dict:
    """Left/right states of one seeded 1D RRMHD+M1 Riemann problem."""
    rng = np.random.default_rng(seed)
    bx = rng.uniform(-1.0, 1.0)
    sides = {}
    for s in ("L", "R"):
        rho = _log_uniform(rng, 0.1, 10.0)
        p = _log_uniform(rng, 0.01, 10.0)
        n = _unit_vectors(rng, 1)[:, 0]
        v = n * rng.uniform(0.0, 0.9)
        while True:
            by, bz = rng.uniform(-1.7, 1.7, 2)
            if bx * bx + by * by + bz * bz < 4.0:
                break
        er = _log_uniform(rng, 1e-3, 10.0)
        m = _unit_vectors(rng, 1)[:, 0]
        fr = m * rng.uniform(0.0, 1.0) * er
        kap = _log_uniform(rng, 1e-2, 1e3)
        sig = _log_uniform(rng, 1e-2, 1e3)
        sides[s] = dict(rho=rho, v=v, p=p, B=np.array([bx, by, bz]), E=er, F=fr, kappa=kap, sigma=sig)
    TL = sides["L"]["p"] / sides["L"]["rho"]
    TR = sides["R"]["p"] / sides["R"]["rho"]
    a_rad = math.sqrt(sides["L"]["E"] * sides["R"]["E"]) / (TL * TR) ** 2
    return dict(sides=sides, a_rad=a_rad)


def riemann_1d(seed: int, n: int = 400) -> Problem:
    """Seeded 1D Riemann problem on [0, 1] with the jump at x = 1/2."""
    st = riemann_states(seed)
    dx = 1.0 / n
    x = (np.arange(n) + 0.5) * dx
    V = np.zeros((NV, n))
    kap = np.zeros(n)
    sig = np.zeros(n)
    for s, mask in (("L", x < 0.5), ("R", x >= 0.5)):
        d = st["sides"][s]
        V[0, mask] = d["rho"]
        V[1:4, mask] = d["v"][:, None]
        V[4, mask] = d["p"]
        V[5:8, mask] = d["B"][:, None]
        V[8, mask] = d["E"]
        V[9:12, mask] = d["F"][:, None]
        kap[mask] = d["kappa"]
        sig[mask] = d["sigma"]
    return Problem(name=f"riemann1d_s{seed}_n{n}", shape=(n,), dx=(dx,), x0=(0.0,), V=V, kappa=kap,
                   sigma=sig, gamma=5.0 / 3.0, a_rad=st["a_rad"], bc_lo=(OUTFLOW,) * 3,
                   bc_hi=(OUTFLOW,) * 3, cfl=0.4, t_end=0.4)


def alfven_1d(n: int) -> Problem:
    """Large-amplitude circularly polarised Alfven wave (Section 4.1, after
    Del Zanna et al.): rho_0 = 1, h_0 = 5 (p_0 = 1 for gamma = 4/3), B_0 = 1,
    amplitude A = sqrt(2 / (7 + 3 sqrt 5)), one wavelength on [0, 2 pi],
    v_y = -A cos x, v_z = -A sin x, B_y = -B_0 v_y / v_a, B_z = -B_0 v_z / v_a
    at cell centres, periodic. The paper's run: PVM-int-8, RK3, CFL 0.3, one
    period T = 2 pi / v_a (``t_end``). Radiation is a passive uniform field
    (E_r = 1e-8, F_r = 0, kappa = sigma = 0)."""
    gamma = 4.0 / 3.0
    rho0, h0, B0 = 1.0, 5.0, 1.0
    p0 = (h0 - 1.0) * rho0 * (gamma - 1.0) / gamma
    amp = math.sqrt(2.0 / (7.0 + 3.0 * math.sqrt(5.0)))
    va = math.sqrt(B0 ** 2 * (1.0 - amp ** 2) / (rho0 * h0 + B0 ** 2 * (1.0 - amp ** 2)))
    length = 2.0 * math.pi
    dx = length / n
    x = (np.arange(n) + 0.5) * dx
    V = np.zeros((NV, n))
    V[0] = rho0
    V[2] = -amp * np.cos(2.0 * math.pi * x / length)
    V[3] = -amp * np.sin(2.0 * math.pi * x / length)
    V[4] = p0
    V[5] = B0
    V[6] = -B0 * V[2] / va
    V[7] = -B0 * V[3] / va
    V[8] = 1e-8
    return Problem(name=f"alfven1d_n{n}", shape=(n,), dx=(dx,), x0=(0.0,), V=V, kappa=np.zeros(n),
                   sigma=np.zeros(n), gamma=gamma, a_rad=0.0, bc_lo=(PERIODIC,) * 3, bc_hi=(PERIODIC,) * 3,
                   cfl=0.3, t_end=length / va, extra={"v_a": va, "amplitude": amp})


def uniform_face_fields(P: Problem) -> np.ndarray:
    """Staggered normal fields of a problem whose in-plane field is uniform
    (the blast): every face of direction a carries the cell value B_a."""
    out = np.zeros((P.ndim, P.ncell))
    for a in range(P.ndim):
        assert np.all(P.V[5 + a] == P.V[5 + a][0]), "the in-plane field is not uniform"
        out[a] = P.V[5 + a]
    return out


def alfven_2d(n: int, ny: int = 2) -> Problem:
    """The Alfven wave of ``alfven_1d`` on an n x ny periodic grid, uniform in
    y (dy = dx). Face fields: b_x = B_0 on every x-face; b_y of a y-face is
    the B_y of the cells it separates (the field depends on x only)."""
    P1 = alfven_1d(n)
    dx = P1.dx[0]
    V = np.tile(P1.V, (1, ny))
    bface = np.zeros((2, n * ny))
    bface[0] = V[5]
    bface[1] = V[6]
    return Problem(name=f"alfven2d_n{n}x{ny}", shape=(n, ny), dx=(dx, dx), x0=(0.0, 0.0), V=V,
                   kappa=np.zeros(n * ny), sigma=np.zeros(n * ny), gamma=P1.gamma, a_rad=0.0,
                   bc_lo=(PERIODIC,) * 3, bc_hi=(PERIODIC,) * 3, cfl=P1.cfl, t_end=P1.t_end,
                   extra=dict(P1.extra, bface=bface))


def field_loop_2d(nx: int, ny: int | None = None, v0: float = 0.5, b0: float = 1e-3, radius: float = 0.3,
                  angle_deg: float | None = None) -> Problem:
    """Advection of a weak magnetic field loop (the constrained-transport test
    of Gardiner & Stone 2005) on [-1, 1] x [-1/2, 1/2], periodic: uniform
    rho = 1, p = 1, velocity v0 along the diagonal of the box, field from the
    vector potential A_z = b0 (R - r) for r < R (0 outside), gamma = 5/3;
    radiation passive (E_r = 1e-8, no opacity). The face fields are the
    differences of A_z at the cell corners (b_x = dA_z/dy, b_y = -dA_z/dx),
    so their discrete divergence is zero; the cell-centred field is the mean
    of each cell's two face values. One crossing of the box takes
    t = 2 / (v0 cos theta)."""
    ny = nx // 2 if ny is None else ny
    lx, ly = 2.0, 1.0
    dx, dy = lx / nx, ly / ny
    theta = math.atan2(ly, lx) if angle_deg is None else math.radians(angle_deg)
    xc = -1.0 + (np.arange(nx + 1)) * dx          # corners
    yc = -0.5 + (np.arange(ny + 1)) * dy
    Xc, Yc = np.meshgrid(xc, yc, indexing="xy")   # [ny + 1, nx + 1]
    r = np.sqrt(Xc * Xc + Yc * Yc)
    Az = np.where(r < radius, b0 * (radius - r), 0.0)
    bx = (Az[1:, :-1] - Az[:-1, :-1]) / dy        # x-face (i - 1/2, j): corners j-1/2 .. j+1/2
    by = -(Az[:-1, 1:] - Az[:-1, :-1]) / dx       # y-face (i, j - 1/2): corners i-1/2 .. i+1/2
    Bx = 0.5 * (bx + np.roll(bx, -1, axis=1))
    By = 0.5 * (by + np.roll(by, -1, axis=0))
    N = nx * ny
    V = np.zeros((NV, N))
    V[0] = 1.0
    V[1] = v0 * math.cos(theta)
    V[2] = v0 * math.sin(theta)
    V[4] = 1.0
    V[5] = Bx.reshape(-1)
    V[6] = By.reshape(-1)
    V[8] = 1e-8
    return Problem(name=f"fieldloop2d_{nx}x{ny}", shape=(nx, ny), dx=(dx, dy), x0=(-1.0, -0.5), V=V,
                   kappa=np.zeros(N), sigma=np.zeros(N), gamma=5.0 / 3.0, a_rad=0.0,
                   bc_lo=(PERIODIC,) * 3, bc_hi=(PERIODIC,) * 3, cfl=0.4,
                   t_end=lx / (v0 * math.cos(theta)),
                   extra={"bface": np.stack([bx.reshape(-1), by.reshape(-1)]), "b0": b0, "radius": radius})


def radiation_rp_1d(test: int, n: int = 256) -> Problem:
    """Optically thin radiation Riemann problems of Section 4.2 (after Melon
    Fuksman & Mignone): [-20, 20] with the jump at x = 0, outflow, t = 20.
    Test 1: (E_r, F_x, F_y) = (1, 0, 1/2) | (1, 0, 0); Test 2: (1/10, 1/10, 0)
    | (1, 0, 1). No matter-radiation coupling (kappa = sigma = 0): the fluid,
    which the paper does not specify, is a uniform unmagnetised gas at rest
    (rho = 1, p = 1). CFL 0.3 and RK3 as in the paper's other tests."""
    states = {1: ((1.0, 0.0, 0.5), (1.0, 0.0, 0.0)), 2: ((0.1, 0.1, 0.0), (1.0, 0.0, 1.0))}
    left, right = states[test]
    dx = 40.0 / n
    x = -20.0 + (np.arange(n) + 0.5) * dx
    V = np.zeros((NV, n))
    V[0] = 1.0
    V[4] = 1.0
    for q, (a, b) in zip((8, 9, 10), zip(left, right)):
        V[q] = np.where(x < 0.0, a, b)
    return Problem(name=f"radrp{test}_n{n}", shape=(n,), dx=(dx,), x0=(-20.0,), V=V, kappa=np.zeros(n),
                   sigma=np.zeros(n), gamma=4.0 / 3.0, a_rad=0.0, cfl=0.3, t_end=20.0)


def blast_2d(seed: int = 0, nx: int = 512, ny: int | None = None, steps: int = 200,
             e_bg: float = 0.0, p_in: float = 10.0) -> Problem:
    """Magnetised cylindrical blast on [-1/2, 1/2]^2 (periodic).

    Radiation starts in equilibrium with the gas, E_r = a_R T^4, plus an
    optional uniform isotropic background ``e_bg``; F_r = 0. ``p_in``: the
    pressure inside r < 0.1 (10: overpressure 1e3 over the ambient 0.01); the
    radiation constant stays 1e-3."""
    ny = nx if ny is None else ny
    rng = np.random.default_rng(seed)
    dx, dy = 1.0 / nx, 1.0 / ny
    x = -0.5 + (np.arange(nx) + 0.5) * dx
    y = -0.5 + (np.arange(ny) + 0.5) * dy
    X, Y = np.meshgrid(x, y, indexing="xy")      # [ny, nx], x fastest when flattened
    g = np.zeros_like(X)
    for _ in range(8):
        kx, ky = rng.integers(1, 5, 2)
        sx, sy = rng.choice([-1, 1], 2)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        g += np.cos(2.0 * math.pi * (sx * kx * X + sy * ky * Y) + ph)
    g /= np.max(np.abs(g))
    rho = 1.0 + 0.01 * g
    r = np.sqrt(X * X + Y * Y)
    p = np.where(r < 0.1, p_in, 0.01)
    T = p / rho
    a_rad = 10.0 / 10.0 ** 4          # p_in / T_in^4: radiation ~ gas pressure inside
    V = np.zeros((NV, ny * nx))
    V[0] = rho.reshape(-1)
    V[4] = p.reshape(-1)
    V[5] = 0.5 * math.cos(math.pi / 4)
    V[6] = 0.5 * math.sin(math.pi / 4)
    V[8] = (a_rad * T ** 4 + e_bg).reshape(-1)
    kap = (10.0 ** (-0.5 + 2.5 * np.sin(2.0 * math.pi * X)) / dx).reshape(-1)
    sig = (10.0 ** (-0.5 + 2.5 * np.sin(2.0 * math.pi * Y)) / 10.0 / dy).reshape(-1)
    return Problem(name=f"blast2d_s{seed}_{nx}x{ny}", shape=(nx, ny), dx=(dx, dy), x0=(-0.5, -0.5),
                   V=V, kappa=kap, sigma=sig, gamma=4.0 / 3.0, a_rad=a_rad,
                   bc_lo=(PERIODIC,) * 3, bc_hi=(PERIODIC,) * 3, cfl=0.4, steps=steps)


def serving_mix(seed: int, n: int, *, n1d=(256, 8192), n2d=(64, 512), t_end_1d: float = 0.05,
                steps_2d=(10, 50), mixed_frac: float = 0.5) -> list[dict]:
    """Request mix for the serving loop: half 1D Riemann problems with
    N ~ logU[256, 8192] run to t_end_1d, half 2D blasts with N^2 cells,
    N ~ logU[64, 512], run for a number of steps; FP64 / mixed precision
    50/50. Returns plain dicts (problem, precision flag, t_end or steps)."""
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        mixed = bool(rng.uniform() < mixed_frac)
        if rng.uniform() < 0.5:
            N = int(round(_log_uniform(rng, *n1d)))
            P = riemann_1d(int(rng.integers(0, 2**31 - 1)), n=N)
            out.append(dict(problem=P, mixed=mixed, t_end=t_end_1d, steps=None))
        else:
            N = int(round(_log_uniform(rng, *n2d)))
            P = blast_2d(int(rng.integers(0, 2**31 - 1)), N)
            out.append(dict(problem=P, mixed=mixed, t_end=None, steps=int(rng.integers(steps_2d[0], steps_2d[1] + 1))))
    return out


def poisson_arrivals(seed: int, n: int, rate: float) -> np.ndarray:
    """Arrival times (s) of a Poisson process with the given rate (1/s)."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate, n))


def beam_3d(seed: int = 0, nx: int = 512, ny: int | None = None, nz: int | None = None, steps: int = 50,
            r_noz: float = 0.05) -> Problem:
    """Cylindrical beam into an ambient medium on [-1/2,1/2]^2 x [0,1].

    Ambient: rho = 1 + 0.01 g (periodic Fourier modes), p = 0.01, v = 0,
    B = 0, radiation in equilibrium E_r = a_R T^4 (T = p/rho), F_r = 0.
    Beam (inflow cells below z = 0 inside r < r_noz): W = 7 along z,
    rho = 0.01, p = 0.01, B_phi = 0.3 r / r_noz, E_r = a_R (T = 1), F_r = 0.
    a_R = 0.01; kappa ~ logU[10, 1e3] i.i.d. per cell, sigma = 0.
    Returns the problem; the inflow primitives [12, nx*ny] and the mask are in
    ``extra`` (the caller converts them to conserved variables)."""
    ny = nx if ny is None else ny
    nz = nx if nz is None else nz
    rng = np.random.default_rng(seed)
    dx, dy, dz = 1.0 / nx, 1.0 / ny, 1.0 / nz
    x = -0.5 + (np.arange(nx) + 0.5) * dx
    y = -0.5 + (np.arange(ny) + 0.5) * dy
    z = (np.arange(nz) + 0.5) * dz
    a_rad = 0.01
    n = nx * ny * nz
    V = np.zeros((NV, n))
    # smooth density perturbation, built plane by plane (x fastest)
    Xp, Yp = np.meshgrid(x, y, indexing="xy")
    modes = [(rng.integers(1, 5, 3), rng.choice([-1, 1], 3), rng.uniform(0, 2 * math.pi)) for _ in range(8)]
    g = np.zeros((nz, ny, nx))
    for k, zz in enumerate(z):
        acc = np.zeros_like(Xp)
        for (kx, ky, kz), (sx, sy, sz), ph in modes:
            acc += np.cos(2 * math.pi * (sx * kx * Xp + sy * ky * Yp + sz * kz * zz) + ph)
        g[k] = acc
    g /= np.max(np.abs(g))
    rho = (1.0 + 0.01 * g).reshape(-1)
    V[0] = rho
    V[4] = 0.01
    V[8] = a_rad * (0.01 / rho) ** 4
    kap = _log_uniform(rng, 10.0, 1e3, n)
    sig = np.zeros(n)
    # inflow face (z = 0), transverse index i + nx j
    r = np.sqrt(Xp * Xp + Yp * Yp).reshape(-1)
    phi = np.arctan2(Yp, Xp).reshape(-1)
    mask = (r < r_noz).astype(np.uint8)
    Vin = np.zeros((NV, nx * ny))
    W = 7.0
    Vin[0] = 0.01
    Vin[3] = math.sqrt(1.0 - 1.0 / (W * W))
    Vin[4] = 0.01
    bphi = 0.3 * np.minimum(r / r_noz, 1.0)
    Vin[5] = -bphi * np.sin(phi)
    Vin[6] = bphi * np.cos(phi)
    Vin[8] = a_rad * 1.0
    return Problem(name=f"beam3d_s{seed}_{nx}x{ny}x{nz}", shape=(nx, ny, nz), dx=(dx, dy, dz), x0=(-0.5, -0.5, 0.0),
                   V=V, kappa=kap, sigma=sig, gamma=4.0 / 3.0, a_rad=a_rad,
                   bc_lo=(OUTFLOW, OUTFLOW, INFLOW), bc_hi=(OUTFLOW, OUTFLOW, OUTFLOW), cfl=0.3, steps=steps,
                   extra=dict(inflow_V=Vin, inflow_mask=mask))
