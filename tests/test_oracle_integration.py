"""Grid-level pins of the CPU oracle: conservation, dimensional reduction,
free streaming at c, diffusion, and the printed L1 errors of the Alfven wave
test (Section 4 of the paper)."""
import math
import os

import numpy as np
import pytest

from paper_2212_00370_amd import inputs as I


def run(oracle, grid, U, par, kap, sig, cfl, steps=None, t_end=None, dx=None):
    t = 0.0
    n = 0
    while True:
        if steps is not None and n >= steps:
            break
        if t_end is not None and t >= t_end * (1 - 1e-14):
            break
        s, nf = oracle.max_speed(grid, U, par)
        assert nf == 0
        dt = cfl * min(dx) / s
        if t_end is not None:
            dt = min(dt, t_end - t)
        U, st, rep = oracle.step(grid, U, dt, kap, sig, par)
        assert st == 0, (n, rep.c2p_fail, rep.imp_fail, rep.first_bad_cell)
        t += dt
        n += 1
    return U, t, n


def test_periodic_conservation(oracle):
    """Flux form with one numerical flux per face (eq. full) and the implicit
    step's conservation of tau + E_r and S + F_r: on a periodic grid the sums of
    D, B, tau + E_r and S + F_r are constant to rounding."""
    P = I.blast_2d(0, 48, 40)
    par = oracle.params(gamma=P.gamma, a_rad=P.a_rad, beta_mode=1)
    g = oracle.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    U0 = oracle.p2c(P.V, par)
    U, t, n = run(oracle, g, U0, par, P.kappa, P.sigma, P.cfl, steps=6, dx=P.dx)
    tot = lambda U: np.array([U[0].sum(), *(U[5:8].sum(axis=1)), (U[4] + U[8]).sum(),
                              *((U[1:4] + U[9:12]).sum(axis=1))])
    a, b = tot(U0), tot(U)
    scale = np.array([np.abs(U0[0]).sum(), *np.abs(U0[5:8]).sum(axis=1), np.abs(U0[4] + U0[8]).sum(),
                      *[np.abs(U0[4] + U0[8]).sum()] * 3])
    assert np.max(np.abs(b - a) / np.maximum(scale, 1.0)) < 1e-13
    assert not np.array_equal(U, U0)


def test_2d_uniform_in_y_equals_1d_bitwise(oracle):
    """A 2D state uniform in y evolves exactly like the 1D problem: the y-face
    fluxes between equal states are F(U) exactly, so their difference is 0."""
    P = I.riemann_1d(3, n=64)
    par = oracle.params(gamma=P.gamma, a_rad=P.a_rad, beta_mode=1)
    U1 = oracle.p2c(P.V, par)
    g1 = oracle.make_grid((64,), (1 / 64,))
    ny = 3
    U2 = np.tile(U1[:, None, :], (1, ny, 1)).reshape(12, -1)
    g2 = oracle.make_grid((64, ny), (1 / 64, 1 / 64), bc_lo=(1, 0, 1), bc_hi=(1, 0, 1))
    k2 = np.tile(P.kappa, ny); s2 = np.tile(P.sigma, ny)
    dt = 0.4 / 64 / 1.0
    for _ in range(3):
        U1, st1, _ = oracle.step(g1, U1, dt, P.kappa, P.sigma, par)
        U2, st2, _ = oracle.step(g2, U2, dt, k2, s2, par)
        assert st1 == 0 and st2 == 0
        for j in range(ny):
            assert np.array_equal(U2.reshape(12, ny, 64)[:, j, :], U1)


def test_free_streaming_pulse_moves_at_c(oracle):
    """f = 1 beam along +x in vacuum-like conditions (kappa = sigma = 0): the
    radiation flux equals the energy flux (eqs. xi, lam1-lam3 with f = 1), the
    first-order PVM face flux is upwind, and the pulse centroid moves at c = 1.
    The fluid is uniform and stays so (to finite-difference noise)."""
    n = 200
    dx = 1.0
    x = -100 + (np.arange(n) + 0.5) * dx
    Eb, A, w = 1e-6, 1e-3, 8.0
    V = np.zeros((12, n))
    V[0] = 1.0; V[4] = 1.0
    V[8] = Eb + A * np.exp(-((x + 40) / w) ** 2)
    V[9] = V[8]
    par = oracle.params(recon=0)
    g = oracle.make_grid((n,), (dx,))
    U0 = oracle.p2c(V, par)
    U, t, nst = run(oracle, g, U0, par, 0.0, 0.0, 0.4, t_end=50.0, dx=(dx,))
    c0 = np.sum(x * (U0[8] - Eb)) / np.sum(U0[8] - Eb)
    c1 = np.sum(x * (U[8] - Eb)) / np.sum(U[8] - Eb)
    assert (c1 - c0) / t == pytest.approx(1.0, abs=1e-6)
    assert np.max(np.abs(U[9] - U[8]) / U[8]) < 1e-6
    # The |F_r| <= E_r limit acts on finite-difference noise (F_x ~ E_r) and
    # hands that momentum to the gas, so the fluid moves only at noise level.
    assert np.max(np.abs(U[:8] - U0[:8])) < 1e-6


def heat_kernel(x, t, A, w, D):
    s2 = w * w + 4 * D * t
    return A * math.sqrt(w * w / s2) * np.exp(-x * x / s2)


def diffusion_run(oracle, sigma, beta_mode, t_end, solver=0):
    """Optically thick pulse (Section 4, radiation pulse): static uniform gas,
    kappa = 0, scattering sigma, Gaussian E_r; [-50, 50] with 100 zones."""
    n = 100
    dx = 1.0
    x = -50 + (np.arange(n) + 0.5) * dx
    A, w, Eb = 1e-6, 5.0, 1e-14
    V = np.zeros((12, n))
    V[0] = 1.0; V[4] = 1.0
    V[8] = Eb + A * np.exp(-(x / w) ** 2)
    par = oracle.params(gamma=5 / 3, beta_mode=beta_mode, solver=solver)
    g = oracle.make_grid((n,), (dx,))
    U0 = oracle.p2c(V, par)
    U, t, nst = run(oracle, g, U0, par, 0.0, sigma, 0.4, t_end=t_end, dx=(dx,))
    D = 1.0 / (3.0 * sigma)
    ex = Eb + heat_kernel(x, t, A, w, D)
    return np.sum(np.abs(U[8] - ex)) / np.sum(np.abs(ex - Eb)), U, ex


@pytest.mark.slow
@pytest.mark.parametrize("sigma", [100.0, 1000.0])
def test_diffusion_limit_matches_heat_kernel(oracle, sigma):
    """Diffusion limit: E_r follows the 1D heat kernel with D = 1/(3 rho (kappa +
    sigma)); the opacity-scaled viscosity (eq. beta) is far more accurate than
    beta = 1, which is catastrophically diffusive for tau >= 100."""
    t_end = 1875.0
    err, U, ex = diffusion_run(oracle, sigma, 1, t_end)
    err1, _, _ = diffusion_run(oracle, sigma, 2, t_end)
    assert err < 0.03
    assert err1 / err > 3.0


def _table4():
    """Section 4.1, Table 4 rows (tests/golden): N -> (Godunov, MinMod, MC, VanLeer)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "alfven_pvm_int8_table4.txt")
    rows = {}
    for ln in open(path):
        if ln.strip() and not ln.startswith("#"):
            n, *errs = ln.split()
            rows[int(n)] = tuple(float(e) for e in errs)
    return rows


# relative tolerance per reconstruction (Godunov, MinMod, MC, VanLeer): the
# paper's time-step sequence and last-step clipping are not printed, which
# moves the second-order rows by a few per cent
_TABLE4_REL = (1e-3, 3e-2, 5e-2, 5e-2)


@pytest.mark.parametrize("recon", [0, 1, 2, 3])
def test_alfven_wave_reproduces_table4(oracle, recon):
    """Section 4.1: the circularly polarised Alfven wave, PVM-int-8 with RK3
    and CFL 0.3, run for one period; L1(v_z) against the initial state must
    reproduce the printed Table 4 row of each reconstruction (Section 3.2:
    Godunov, MinMod, MC, VanLeer), with the observed orders ~1 and ~2. The
    PLM rows differ from one another by 30 % or more at N = 16..64, so a
    wrong limiter fails its row."""
    table = _table4()
    errs = {}
    for n in (16, 32, 64, 128):
        P = I.alfven_1d(n)
        par = oracle.params(gamma=P.gamma, a_rad=P.a_rad, rk_order=3, recon=recon, pvm_k=3)
        g = oracle.make_grid(P.shape, P.dx, bc_lo=P.bc_lo, bc_hi=P.bc_hi)
        U, t, _ = run(oracle, g, oracle.p2c(P.V, par), par, 0.0, 0.0, P.cfl, t_end=P.t_end, dx=P.dx)
        assert abs(t - P.t_end) <= 1e-12 * P.t_end
        V, _, st, _ = oracle.c2p(U, par)
        assert np.all(st == 0)
        errs[n] = float(np.mean(np.abs(V[3] - P.V[3])))
        printed = table[n][recon]
        assert errs[n] == pytest.approx(printed, rel=_TABLE4_REL[recon]), (n, errs[n], printed)
    orders = [math.log2(errs[n] / errs[2 * n]) for n in (32, 64)]
    if recon != 0:
        assert all(1.8 < o < 2.45 for o in orders), orders
    else:
        assert all(0.45 < o < 0.85 for o in orders), orders


def test_alfven_error_decreases_with_pvm_order(oracle):
    """eq. iterat: p_k approximates |x| from above and decreases with k, so the
    numerical viscosity, and the Alfven-wave error with it, falls with k; the
    degree-16 member stays close to PVM-int-8 (Section 5 reports the two alike)."""
    P = I.alfven_1d(64)
    errs = []
    for k in (1, 2, 3, 4):
        par = oracle.params(gamma=P.gamma, a_rad=P.a_rad, rk_order=3, recon=1, pvm_k=k)
        g = oracle.make_grid(P.shape, P.dx, bc_lo=P.bc_lo, bc_hi=P.bc_hi)
        U, _, _ = run(oracle, g, oracle.p2c(P.V, par), par, 0.0, 0.0, P.cfl, t_end=P.t_end, dx=P.dx)
        V, _, _, _ = oracle.c2p(U, par)
        errs.append(float(np.mean(np.abs(V[3] - P.V[3]))))
    assert all(a > b for a, b in zip(errs, errs[1:])), errs
    assert abs(errs[3] - errs[2]) < 0.1 * errs[2], errs


def _swap_xy(V, nx, ny):
    """[q, j nx + i] -> [q', i ny + j] with the x and y components exchanged."""
    W = V.reshape(V.shape[0], ny, nx).transpose(0, 2, 1).reshape(V.shape[0], -1)
    return np.ascontiguousarray(W[[0, 2, 1, 3, 4, 6, 5, 7, 8, 10, 9, 11]])


def test_xy_transpose_symmetry_bitwise(oracle):
    """Exchanging x and y (grid, cell sizes and vector components) commutes with
    the explicit scheme bit for bit: every sum over components is written as
    (x + y) + z and every per-direction operation is generic in d. A wrong
    direction index or a transposed operand breaks it. The opacities are zero
    here: the implicit 4x4 elimination of a coupled cell orders its rows
    E, F_x, F_y, F_z, which the exchange permutes."""
    P = I.blast_2d(0, 48, 40)
    nx, ny = P.shape
    par = oracle.params(gamma=P.gamma, a_rad=P.a_rad)
    g = oracle.make_grid((nx, ny), P.dx, P.bc_lo, P.bc_hi)
    gt = oracle.make_grid((ny, nx), (P.dx[1], P.dx[0]), P.bc_lo, P.bc_hi)
    U = oracle.p2c(P.V, par)
    Ut = oracle.p2c(_swap_xy(P.V, nx, ny), par)
    assert np.array_equal(Ut, _swap_xy(U, nx, ny))
    for _ in range(3):
        s, _ = oracle.max_speed(g, U, par)
        assert oracle.max_speed(gt, Ut, par)[0] == s
        dt = P.cfl * min(P.dx) / s
        U, st, _ = oracle.step(g, U, dt, 0.0, 0.0, par)
        Ut, st2, _ = oracle.step(gt, Ut, dt, 0.0, 0.0, par)
        assert st == 0 and st2 == 0
        assert np.array_equal(Ut, _swap_xy(U, nx, ny))
