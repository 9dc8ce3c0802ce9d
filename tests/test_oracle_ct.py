"""Pins of the oracle's constrained transport: staggered normal field on the
faces, edge EMFs averaged by the CT-contact rule (the scheme the paper's
multidimensional runs use, Section 4 opening paragraph, after Gardiner &
Stone 2005).

  * the discrete divergence of the face field stays at round-off (it is the
    divergence of a discrete curl), where the cell-centred scheme lets it grow;
  * a problem uniform along y reduces to the 1D scheme (the contact-upwinded
    corner value of a y-uniform flow is exactly the x-face EMF), and one
    uniform along z to the 2D scheme;
  * the Alfven wave of Section 4.1 run in 2D with CT reproduces Table 4;
  * a weak field loop advected across the periodic box keeps a monotonically
    decaying magnetic energy and converges with resolution;
  * the totals D, tau + E_r, S + F_r and the face fields' sums are conserved.
"""
import math
import os

import numpy as np
import pytest

from paper_2212_00370_amd import inputs as I


def ct_state(oracle, P, par):
    return np.vstack([oracle.p2c(P.V, par), P.extra["bface"] if "bface" in P.extra else I.uniform_face_fields(P)])


def div_face(P, U):
    """Discrete divergence of the staggered field, per cell."""
    shape = P.shape[::-1]
    d = np.zeros(shape)
    for a in range(P.ndim):
        b = U[12 + a].reshape(shape)
        d += (np.roll(b, -1, axis=P.ndim - 1 - a) - b) / P.dx[a]
    return d


def run(oracle, P, par, U, steps=None, t_end=None, every=None):
    g = oracle.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    t, n = 0.0, 0
    while (steps is not None and n < steps) or (t_end is not None and t < t_end * (1 - 1e-14)):
        s, _ = oracle.max_speed(g, U, par)
        dt = P.cfl * min(P.dx) / s
        if t_end is not None:
            dt = min(dt, t_end - t)
        U, st, rep = oracle.step(g, U, dt, P.kappa, P.sigma, par)
        assert st == 0, (n, rep.c2p_fail, rep.imp_fail)
        t += dt
        n += 1
        if every is not None:
            every(n, U)
    return U, n


def test_ct_blast_divergence_stays_at_roundoff(oracle):
    """64x40 magnetised blast, 20 steps: max |div b| dx / max |b| < 1e-14 and
    the cell-centred field is the mean of the face values bit for bit; the
    cell-centred scheme's central-difference divergence grows to O(1e-2)."""
    oracle.threads(0)
    P = I.blast_2d(0, 64, 40)
    par = oracle.params(gamma=P.gamma, a_rad=P.a_rad, ct=1)
    U0 = ct_state(oracle, P, par)
    assert np.max(np.abs(div_face(P, U0))) == 0.0
    U, _ = run(oracle, P, par, U0, steps=20)
    bmax = np.max(np.abs(U[12:14]))
    assert np.max(np.abs(div_face(P, U))) * P.dx[0] / bmax < 1e-14
    nx, ny = P.shape
    for a, axis in ((0, 1), (1, 0)):
        b = U[12 + a].reshape(ny, nx)
        assert np.array_equal(U[5 + a].reshape(ny, nx), 0.5 * (b + np.roll(b, -1, axis=axis)))
    assert np.max(np.abs(U[12:14] - U0[12:14])) > 1e-3            # the field did evolve
    par0 = oracle.params(gamma=P.gamma, a_rad=P.a_rad)
    Uc, _ = run(oracle, P, par0, oracle.p2c(P.V, par0), steps=20)
    bx, by = Uc[5].reshape(ny, nx), Uc[6].reshape(ny, nx)
    dc = (np.roll(bx, -1, 1) - np.roll(bx, 1, 1)) / (2 * P.dx[0]) + (np.roll(by, -1, 0) - np.roll(by, 1, 0)) / (2 * P.dx[1])
    assert np.max(np.abs(dc)) * P.dx[0] / np.max(np.abs(Uc[5:7])) > 1e-3


@pytest.mark.parametrize("solver", [0, 1, 2])
def test_ct_face_states_take_the_face_normal_field(oracle, solver):
    """Both states of a d-face take the face's own b_d, so the normal field is
    continuous across it and the face flux of B_d is exactly zero (its
    physical flux v_d B_d - B_d v_d vanishes, and so does its jump). Checked
    on the field loop after 5 steps, where the reconstructed cell-centred
    normal field would jump; the same state's cell-centred face fluxes do
    carry B_d."""
    oracle.threads(0)
    P = I.field_loop_2d(48)
    par = oracle.params(gamma=P.gamma, a_rad=0.0, ct=1, solver=solver)
    U, _ = run(oracle, P, par, ct_state(oracle, P, par), steps=5)
    g = oracle.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    Fd, _ = oracle.face_fluxes(g, U, 0.0, 0.0, par)
    assert np.all(Fd[0][5] == 0.0) and np.all(Fd[1][6] == 0.0)
    par0 = oracle.params(gamma=P.gamma, a_rad=0.0, solver=solver)
    Fc, _ = oracle.face_fluxes(g, U[:12], 0.0, 0.0, par0)
    assert np.max(np.abs(Fc[0][5])) > 1e-8 and np.max(np.abs(Fc[1][6])) > 1e-8


def test_ct_conserves_totals(oracle):
    """Periodic blast with CT: sum D, sum (tau + E_r), sum (S + F_r) and the
    sums of each face field are conserved to round-off."""
    oracle.threads(0)
    P = I.blast_2d(1, 48, 40)
    par = oracle.params(gamma=P.gamma, a_rad=P.a_rad, ct=1)
    U0 = ct_state(oracle, P, par)
    U, _ = run(oracle, P, par, U0, steps=10)
    tot = lambda V: np.array([V[0].sum(), (V[4] + V[8]).sum(), (V[1] + V[9]).sum(), (V[2] + V[10]).sum(),
                              (V[3] + V[11]).sum(), V[12].sum(), V[13].sum(), V[7].sum()])
    mom = max(np.abs(U[1:4]).sum() + np.abs(U[9:12]).sum(), 1e-300)      # the gas starts at rest
    scale = np.array([np.abs(U0[0]).sum(), np.abs(U0[4] + U0[8]).sum()] + [mom] * 3
                     + [np.abs(U0[12]).sum(), np.abs(U0[13]).sum(), 1.0])
    assert np.all(np.abs(tot(U) - tot(U0)) / scale < 1e-13), np.abs(tot(U) - tot(U0)) / scale


@pytest.mark.parametrize("solver,tol", [(1, 1e-13), (2, 1e-13), (0, 1e-6)])
def test_ct_y_uniform_reduces_to_1d(oracle, solver, tol):
    """The Alfven wave on a 64x2 grid (uniform in y) with CT against the 1D
    run: 30 RK3 steps with the same dt. For a y-uniform flow the y-face EMFs
    equal the cell ones, the contact corrections cancel the cell EMFs, and the
    corner value is the x-face EMF, so the 1D scheme is recovered to rounding
    (amplified by 1/eps in the difference form of PVM-int-8)."""
    N = 64
    P1, P2 = I.alfven_1d(N), I.alfven_2d(N, 2)
    p1 = oracle.params(gamma=P1.gamma, a_rad=0.0, rk_order=3, solver=solver)
    p2 = oracle.params(gamma=P1.gamma, a_rad=0.0, rk_order=3, solver=solver, ct=1)
    g1 = oracle.make_grid(P1.shape, P1.dx, P1.bc_lo, P1.bc_hi)
    g2 = oracle.make_grid(P2.shape, P2.dx, P2.bc_lo, P2.bc_hi)
    U1, U2 = oracle.p2c(P1.V, p1), ct_state(oracle, P2, p2)
    for n in range(30):
        s1, _ = oracle.max_speed(g1, U1, p1)
        dt = P1.cfl * P1.dx[0] / s1
        U1, st1, _ = oracle.step(g1, U1, dt, 0.0, 0.0, p1)
        U2, st2, _ = oracle.step(g2, U2, dt, 0.0, 0.0, p2)
        assert st1 == 0 and st2 == 0
        assert np.array_equal(U2[:, :N], U2[:, N:])
        rel = np.abs(U2[:12, :N] - U1).max(axis=1) / np.maximum(np.abs(U1).max(axis=1), 1e-300)
        assert rel.max() < tol, (n, rel.max())
    assert np.all(U2[12] == 1.0)                                  # b_x stays B_0 on every face


def test_ct_alfven_wave_reproduces_table4(oracle):
    """Section 4.1 with CT: the Alfven wave on a 64x2 grid, PVM-int-8,
    PLM MinMod, RK3, CFL 0.3, one period: L1(v_z) within 3 % of the printed
    Table 4 MinMod value at N = 64."""
    P = I.alfven_2d(64, 2)
    par = oracle.params(gamma=P.gamma, a_rad=0.0, rk_order=3, ct=1)
    U, n = run(oracle, P, par, ct_state(oracle, P, par), t_end=P.t_end)
    V, _, st, _ = oracle.c2p(U[:12], par)
    l1 = float(np.mean(np.abs(V[3] - P.V[3])))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "alfven_pvm_int8_table4.txt")
    printed = {int(r.split()[0]): float(r.split()[2]) for r in open(path) if r.strip() and not r.startswith("#")}
    assert l1 == pytest.approx(printed[64], rel=0.03), (n, l1, printed[64])


def test_ct_field_loop_advection(oracle):
    """A weak field loop (b0 = 1e-3, R = 0.3) advected at v = 0.5 along the
    diagonal of the periodic [-1, 1] x [-1/2, 1/2] box for one crossing: the
    magnetic energy decays monotonically (no growth: the corner gradients are
    taken upwind of the contact), b_z stays 0, div b stays at round-off, and
    the loop's L1 error falls with resolution (64x32 -> 128x64)."""
    oracle.threads(0)
    errs = []
    for nx in (64, 128):
        P = I.field_loop_2d(nx)
        par = oracle.params(gamma=P.gamma, a_rad=0.0, ct=1)
        U0 = ct_state(oracle, P, par)
        eb0 = float(np.sum(U0[12] ** 2 + U0[13] ** 2))
        ebs = []
        U, n = run(oracle, P, par, U0, t_end=P.t_end,
                   every=lambda k, V: ebs.append(float(np.sum(V[12] ** 2 + V[13] ** 2)) / eb0))
        assert np.all(np.diff(ebs) <= 0.0), "magnetic energy grew"
        assert 0.2 < ebs[-1] < 1.0
        assert np.all(U[7] == 0.0)
        assert np.max(np.abs(div_face(P, U))) * P.dx[0] / P.extra["b0"] < 1e-13
        B0 = P.extra["bface"]
        errs.append(float(np.abs(U[12:14] - B0).sum() / np.abs(B0).sum()))
    assert errs[1] < 0.75 * errs[0], errs


def test_ct_z_uniform_3d_reduces_to_2d(oracle):
    """The field loop on a 32x16x2 periodic grid (uniform in z, v_z = b_z = 0)
    with CT in 3D against the 2D run, Rad-HLL: 20 steps with the same dt, equal
    to rounding; the z-faces and the x- and y-edge EMFs carry nothing."""
    P2 = I.field_loop_2d(32)
    nx, ny = P2.shape
    V3 = np.tile(P2.V, (1, 2))
    bf = P2.extra["bface"]
    b3 = np.vstack([np.tile(bf, (1, 2)), np.zeros((1, 2 * nx * ny))])
    P3 = I.Problem(name="loop3d", shape=(nx, ny, 2), dx=(P2.dx[0], P2.dx[1], P2.dx[0]), x0=(-1.0, -0.5, 0.0),
                   V=V3, kappa=np.zeros(V3.shape[1]), sigma=np.zeros(V3.shape[1]), gamma=P2.gamma, a_rad=0.0,
                   bc_lo=(0, 0, 0), bc_hi=(0, 0, 0), cfl=P2.cfl, extra={"bface": b3})
    p2 = oracle.params(gamma=P2.gamma, a_rad=0.0, ct=1, solver=1)
    g2 = oracle.make_grid(P2.shape, P2.dx, P2.bc_lo, P2.bc_hi)
    g3 = oracle.make_grid(P3.shape, P3.dx, P3.bc_lo, P3.bc_hi)
    U2, U3 = ct_state(oracle, P2, p2), ct_state(oracle, P3, p2)
    N = nx * ny
    for n in range(20):
        s2, _ = oracle.max_speed(g2, U2, p2)
        dt = P2.cfl * min(P2.dx) / s2
        U2, st2, _ = oracle.step(g2, U2, dt, 0.0, 0.0, p2)
        U3, st3, _ = oracle.step(g3, U3, dt, 0.0, 0.0, p2)
        assert st2 == 0 and st3 == 0
        assert np.array_equal(U3[:, :N], U3[:, N:])
        assert np.all(U3[14] == 0.0)
        rel = np.abs(U3[:14, :N] - U2).max(axis=1) / np.maximum(np.abs(U2).max(axis=1), 1e-300)
        assert rel.max() < 1e-13, (n, rel.max())
