"""Pins of the oracle's reconstruction fallback, of the cell optical depths that
enter a face, and of the post-solve radiation-flux limit.

Each test compares the oracle's full grid path (recovery, reconstruction, face
flux; or the implicit solve) with what the paper's definitions fix for a
specially built input, so that a plausible mistake in one of these steps
turns it red:
  * a cell whose reconstructed face velocity reaches |v|^2 >= 1 is zeroth
    order on both of its faces, in every variable (Section 3.2, reconstruction
    paragraph);
  * the face between cells i and i+1 takes the optical depths of exactly those
    two cells (eq. beta) ...
  * ... with tau = rho W (kappa + sigma) dx of the cell averages (eq. limits),
    for the PVM viscosity and for the Rad-HLL speed limit alike;
  * the implicit solve returns |F_r| <= E_r, keeping tau + E_r and S + F_r.
"""
import math

import numpy as np
import pytest

from paper_2212_00370_amd import inputs as I

SOLVERS = [0, 1, 2]          # PVM-int, Rad-HLL, exact-JVP PVM-int


def prim(rho, v, p, B=(0.3, -0.2, 0.1), E=1.0, F=(0.0, 0.0, 0.0)):
    V = np.zeros(12)
    V[0] = rho; V[1:4] = v; V[4] = p; V[5:8] = B; V[8] = E; V[9:12] = F
    return V


def permute_axes(V, d):
    """Rotate vector components so that the x-problem becomes a d-problem."""
    W = V.copy()
    for base in (1, 5, 9):
        comp = V[base:base + 3].copy()
        W[base:base + 3] = np.roll(comp, d, axis=0)
    return W


def grid_cells(oracle, cells, d, dx=0.1):
    """A grid of len(cells) cells along axis d (one cell across the others),
    outflow boundaries; returns (grid, U, face index of face i along d)."""
    n = len(cells)
    shape = [1, 1]
    shape[d] = n
    g = oracle.make_grid(tuple(shape), (dx, dx))
    V = np.stack([permute_axes(c, d) for c in cells], axis=1)
    return g, V


def face_state_flux(oracle, VL, VR, tl, tr, d, par):
    if par.solver == 1:
        F, _ = oracle.hll_face(VL[:, None], VR[:, None], tl, tr, d, par)
    else:
        F, fb, _ = oracle.pvm_face(VL[:, None], VR[:, None], tl, tr, d, par)
        assert fb[0] == 0
    return F[:, 0]


# ------------------------------------------------ reconstruction fallback ----
@pytest.mark.parametrize("solver", SOLVERS)
@pytest.mark.parametrize("recon", [1, 2, 3])
@pytest.mark.parametrize("d", [0, 1])
@pytest.mark.parametrize("mirror", [False, True])
def test_superluminal_face_value_reverts_cell_to_zeroth_order(oracle, solver, recon, d, mirror):
    """Cells A A X B B: the neighbours' slopes vanish (a uniform side), X's
    v_x slope is 0.2 (MinMod), 0.4 (MC) or 0.32 (VanLeer) and its v_y slope 0,
    so its upper face value (v_x + s/2, 0.99) has |v|^2 > 1 although every
    cell average has |v| < 1. X must then enter both of its faces with its
    cell average, in every variable (its density slope too): the two faces
    carry exactly the flux of the zeroth-order pairs (A, X) and (X, B).
    Mirrored (B B X A A with v_x negated) the superluminal value sits on X's
    lower face instead."""
    A = prim(1.0, (-0.1, 0.99, 0.0), 1.0)
    X = prim(2.0, (0.1, 0.99, 0.0), 1.0)
    Bc = prim(3.0, (0.9, 0.3, 0.0), 1.0)
    order = [A, A, X, Bc, Bc]
    if mirror:
        order = [c.copy() for c in order[::-1]]
        for c in order:
            c[1] = -c[1]
    for c in (A, X, Bc):
        assert c[1:4] @ c[1:4] < 1.0
    par = oracle.params(recon=recon, solver=solver)
    g, V = grid_cells(oracle, order, d)
    U = oracle.p2c(V, par)
    Vc, _, st, _ = oracle.c2p(U, par)
    assert np.all(st == 0)
    Fd, nfb = oracle.face_fluxes(g, U, 0.0, 0.0, par)
    assert nfb == 0
    F = Fd[d]                         # faces 0..5 along d (one row across)
    # face 2 sits between cells 1 (A) and 2 (X); face 3 between X and B
    exp2 = face_state_flux(oracle, Vc[:, 1], Vc[:, 2], 0.0, 0.0, d, par)
    exp3 = face_state_flux(oracle, Vc[:, 2], Vc[:, 3], 0.0, 0.0, d, par)
    assert np.array_equal(F[:, 2], exp2)
    assert np.array_equal(F[:, 3], exp3)


@pytest.mark.parametrize("solver", SOLVERS)
def test_subluminal_face_value_keeps_the_slope(oracle, solver):
    """Control for the test above: with v_y = 0.9 instead of 0.99 the upper face
    value stays below 1, X keeps its slopes, and its faces differ from the
    zeroth-order fluxes (the fallback above is what made them equal)."""
    A = prim(1.0, (-0.1, 0.9, 0.0), 1.0)
    X = prim(2.0, (0.1, 0.9, 0.0), 1.0)
    Bc = prim(3.0, (0.9, 0.3, 0.0), 1.0)
    par = oracle.params(recon=1, solver=solver)
    g, V = grid_cells(oracle, [A, A, X, Bc, Bc], 0)
    U = oracle.p2c(V, par)
    Vc, _, _, _ = oracle.c2p(U, par)
    Fd, _ = oracle.face_fluxes(g, U, 0.0, 0.0, par)
    exp2 = face_state_flux(oracle, Vc[:, 1], Vc[:, 2], 0.0, 0.0, 0, par)
    exp3 = face_state_flux(oracle, Vc[:, 2], Vc[:, 3], 0.0, 0.0, 0, par)
    assert np.max(np.abs(Fd[0][:, 2] - exp2)) > 1e-3
    assert np.max(np.abs(Fd[0][:, 3] - exp3)) > 1e-3


# ------------------------------------------------- optical depths at faces ----
def depth_case(seed, n, v, rho_jitter):
    """n cells of one moving gas (velocity v, so W > 1), the density optionally
    varying, a radiation field that changes from cell to cell (so every face
    has radiation viscosity), and kappa, sigma drawn per cell without order
    (so the two cells next to a face are distinguishable from their
    neighbours)."""
    rng = np.random.default_rng(seed)
    cells = []
    for i in range(n):
        rho = 1.3 * math.exp(rng.uniform(-rho_jitter, rho_jitter))
        E = math.exp(rng.uniform(-0.7, 0.7))
        m = rng.normal(size=3); m /= np.linalg.norm(m)
        cells.append(prim(rho, v, 0.7, B=(0.3, 0.1, 0.2), E=E, F=tuple(0.2 * E * m)))
    kap = np.exp(rng.uniform(math.log(10.0), math.log(400.0), n))
    sig = np.exp(rng.uniform(math.log(0.5), math.log(100.0), n))
    return cells, kap, sig


def depths(Vc, kap, sig, dx):
    """tau = rho W (kappa + sigma) dx of each cell average (eq. limits), from
    the recovered primitives: W from the velocity, 1/sqrt(1 - v^2)."""
    v2 = np.sum(Vc[1:4] ** 2, axis=0)
    W = 1.0 / np.sqrt(1.0 - v2)
    return Vc[0] * W * (kap + sig) * dx


@pytest.mark.parametrize("solver", SOLVERS)
def test_face_takes_the_depths_of_its_two_cells(oracle, solver):
    """Godunov faces of a moving gas (W = 3.0) over cells with unordered
    opacities: face i (cells i-1 | i) equals the face flux of those two cell
    states with exactly their depths tau_{i-1}, tau_i, where
    tau = rho W (kappa + sigma) dx (eqs. beta, limits). Optical depths
    2..4e3 keep beta = 1/max(tau_L, tau_R, 1) < 1 and the Rad-HLL limit
    4/(3 tau) active, so a depth taken from another cell, or without W, moves
    the radiation rows by O(1)."""
    n, dx = 14, 0.05
    v = (0.5, 0.8, 0.0)
    W = 1.0 / math.sqrt(1.0 - 0.89)
    assert W > 3.0
    cells, kap, sig = depth_case(40 + solver, n, v, 0.0)
    par = oracle.params(recon=0, solver=solver, beta_mode=1)
    g = oracle.make_grid((n,), (dx,))
    V = np.stack(cells, axis=1)
    U = oracle.p2c(V, par)
    Vc, _, st, _ = oracle.c2p(U, par)
    assert np.all(st == 0)
    tau = depths(Vc, kap, sig, dx)
    assert tau.min() > 1.0
    Fd, nfb = oracle.face_fluxes(g, U, kap, sig, par)
    assert nfb == 0
    F = Fd[0]
    for f in range(n + 1):
        l, r = max(f - 1, 0), min(f, n - 1)          # outflow: ghost = edge cell
        exp = face_state_flux(oracle, Vc[:, l], Vc[:, r], tau[l], tau[r], 0, par)
        scale = np.abs(exp) + 1e-12 * np.max(np.abs(exp))
        assert np.max(np.abs(F[:, f] - exp) / scale) < 1e-12, f


def minmod(a, b):
    return np.where(a * b > 0, np.where(np.abs(a) < np.abs(b), a, b), 0.0)


@pytest.mark.parametrize("solver", SOLVERS)
def test_face_depths_come_from_cell_averages(oracle, solver):
    """MinMod faces with the density varying from cell to cell: the face states
    are reconstructed (limited slopes of the primitives, V_i +- s_i/2), but
    the depths stay those of the two cell averages. The face states are built
    here from the cell averages (their fluxes checked against the oracle's
    face flux of those states), so a depth taken from a face state instead of
    the cell fails."""
    n, dx = 12, 0.05
    v = (0.6, -0.5, 0.3)
    cells, kap, sig = depth_case(50 + solver, n, v, 0.4)
    par = oracle.params(recon=1, solver=solver, beta_mode=1)
    g = oracle.make_grid((n,), (dx,))
    V = np.stack(cells, axis=1)
    U = oracle.p2c(V, par)
    Vc, _, st, _ = oracle.c2p(U, par)
    assert np.all(st == 0)
    tau = depths(Vc, kap, sig, dx)
    ext = np.concatenate([Vc[:, :1], Vc[:, :1], Vc, Vc[:, -1:], Vc[:, -1:]], axis=1)   # outflow ghosts
    s = minmod(ext[:, 1:-1] - ext[:, :-2], ext[:, 2:] - ext[:, 1:-1])                 # cells -1..n
    Fd, nfb = oracle.face_fluxes(g, U, kap, sig, par)
    assert nfb == 0
    for f in range(n + 1):
        # cells f-1 and f sit at columns f and f+1 of s (column 0 is cell -1)
        VL = ext[:, f + 1] + 0.5 * s[:, f]
        VR = ext[:, f + 2] - 0.5 * s[:, f + 1]
        assert np.all(np.sum(VL[9:12] ** 2) <= VL[8] ** 2) and np.sum(VR[9:12] ** 2) <= VR[8] ** 2
        l, r = max(f - 1, 0), min(f, n - 1)
        exp = face_state_flux(oracle, VL, VR, tau[l], tau[r], 0, par)
        scale = np.abs(exp) + 1e-12 * np.max(np.abs(exp))
        assert np.max(np.abs(Fd[0][:, f] - exp) / scale) < 1e-12, f


# --------------------------------------------- radiation limit after solve ----
def stiff_moving_cases(seed, n):
    """Admissible states (|v| < 0.99, f* = |F*|/E* in [0.9, 1)) with absorption
    and scattering up to 1e4 and steps h up to 1: the regime where the coupled
    system is stiffest."""
    rng = np.random.default_rng(seed)
    V = I.random_prims(seed, n, vmax=0.99)
    f = rng.uniform(0.9, 1.0, n)
    m = rng.normal(size=(3, n)); m /= np.linalg.norm(m, axis=0)
    V[9:12] = f * V[8] * m
    kap = np.exp(rng.uniform(math.log(1e-3), math.log(1e4), n))
    sig = np.exp(rng.uniform(math.log(1e-3), math.log(1e4), n)) * rng.integers(0, 2, n)
    h = np.exp(rng.uniform(math.log(1e-4), 0.0, n))
    a_rad = float(np.exp(rng.uniform(-8, 2)))
    return V, kap, sig, h, a_rad


def test_implicit_result_respects_the_flux_limit(oracle):
    """The backward-Euler system with the M1 closure has spurious roots with
    |F_r| > E_r: the closure's sqrt(4 - 3 f^2) is clamped at 0, and Newton can
    settle at f = 2/sqrt(3) on it. Starting from admissible states
    (|F*| < E*), every accepted result must satisfy |F_r| <= E_r (the upper
    limit of Section 3.2, kept after the solve) with tau + E_r and S + F_r
    unchanged (eqs. totale, totalm). Some results of this sample sit on the
    limit, i.e. the limit acted."""
    on_limit = 0
    for seed in (101, 102, 103):
        V, kap, sig, h, a_rad = stiff_moving_cases(seed, 20000)
        par = oracle.params(a_rad=a_rad)
        U = oracle.p2c(V, par)
        assert np.all(np.linalg.norm(U[9:12], axis=0) < U[8])
        Un, st, _ = oracle.implicit(U, h, kap, sig, par)
        ok = st == 0
        assert ok.mean() > 0.95
        fo = np.linalg.norm(Un[9:12], axis=0)[ok] / Un[8, ok]
        assert np.all(fo <= 1.0 + 1e-15), fo.max()
        on_limit += int(np.sum(fo > 1.0 - 1e-15))
        e0 = U[4] + U[8]; e1 = Un[4] + Un[8]
        assert np.max(np.abs(e1 - e0)[ok] / np.abs(e0[ok])) < 4e-16
        m0 = U[1:4] + U[9:12]; m1 = Un[1:4] + Un[9:12]
        assert np.max(np.abs(m1 - m0)[:, ok] / np.maximum(np.abs(m0[:, ok]).max(axis=0), 1e-300)) < 4e-16
    assert on_limit >= 5


def test_pvm_fallback_is_rusanov_whichever_step_fails(oracle):
    """A failed intermediate recovery drops the face to p_0 = 1 (Rusanov with
    lambda = 1) whichever Horner step it occurs in (Sec. 3.2, PVM algorithm;
    the chain's partial result is discarded). With a large difference step
    (pvm_eps = 0.5) some chains leave the admissible states in a later step:
    every face counted as a fallback equals the k = 0 flux bit for bit, and
    the others do not."""
    par = oracle.params(pvm_eps=0.5, beta_mode=0)
    par0 = oracle.params(pvm_k=0, beta_mode=0)
    VL = I.random_prims(31, 4000, vmax=0.9)
    VR = I.random_prims(32, 4000, vmax=0.9)
    Fh, fb, _ = oracle.pvm_face(VL, VR, 0.5, 0.5, 0, par)
    F0, _, _ = oracle.pvm_face(VL, VR, 0.5, 0.5, 0, par0)
    m = fb == 1
    assert 50 <= m.sum() <= 3950, m.sum()
    assert np.array_equal(Fh[:, m], F0[:, m])
    assert not np.any(np.all(Fh[:, ~m] == F0[:, ~m], axis=0))
