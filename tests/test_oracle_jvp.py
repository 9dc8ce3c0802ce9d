"""Pins of the oracle's exact-JVP PVM variant: A(U) w computed in forward mode
through the recovery, and the PVM-int flux built on it.

A w is checked against fourth-order central differences of U -> F(V(U)), along
a contact (where F is affine in the density), and through the spectrum of the
Jacobian it assembles: the radiation block's eigenvalues are the M1 speeds of
eqs. lam1-lam3 and the magnetofluid block's extreme eigenvalues the roots of
the RMHD quartic. The flux built on it matches the eps-difference PVM-int-8
flux to the latter's O(eps) accuracy and reproduces Table 4.
"""
import math

import numpy as np
import pytest

from paper_2212_00370_amd import inputs as I
from test_oracle_integration import run

GAMMA = 4.0 / 3.0
JVP = 2


def test_jvp_equals_central_differences(oracle):
    par = oracle.params(gamma=GAMMA)
    tight = oracle.params(gamma=GAMMA, c2p_tol=1e-16, c2p_maxit=200)
    V = I.random_prims(5, 2000, vmax=0.9)
    U = oracle.p2c(V, par)
    rng = np.random.default_rng(1)
    w = rng.normal(size=U.shape) * (np.abs(U) + 1e-3 * np.abs(U).max(axis=0, keepdims=True))
    h = 1e-4
    for d in range(3):
        Aw, st = oracle.jvp(U, w, d, par)
        assert np.all(st == 0)

        def F(x):
            Vx, _, s, _ = oracle.c2p(x, tight)
            assert np.all(s == 0)
            return oracle.flux(Vx, d, tight)
        fd = (8 * (F(U + h * w) - F(U - h * w)) - (F(U + 2 * h * w) - F(U - 2 * h * w))) / (12 * h)
        err = np.abs(Aw - fd).max(axis=0) / np.abs(fd).max(axis=0)
        assert err.max() < 5e-9, (d, err.max())


def test_jvp_along_a_contact_is_advection(oracle):
    """Along a density change at fixed v, p, B the flux is v_x U plus terms
    that do not depend on rho, so A w = v_x w for w = dU/drho =
    (W, W^2 v, W^2 - W, 0, ...)."""
    par = oracle.params(gamma=GAMMA)
    V = I.random_prims(9, 500, vmax=0.9)
    U = oracle.p2c(V, par)
    W = 1 / np.sqrt(1 - (V[1:4] ** 2).sum(axis=0))
    w = np.zeros_like(U)
    w[0] = W
    w[1:4] = W ** 2 * V[1:4]
    w[4] = W ** 2 - W
    for d in range(3):
        Aw, st = oracle.jvp(U, w, d, par)
        assert np.all(st == 0)
        np.testing.assert_allclose(Aw, V[1 + d] * w, rtol=0, atol=1e-12 * np.abs(w).max())


def _jacobian(oracle, U1, d, par, rows):
    """Columns A e_k (k in rows) restricted to rows, for one state U1 [12]."""
    n = len(rows)
    Ub = np.repeat(U1[:, None], n, axis=1)
    E = np.zeros_like(Ub)
    for i, k in enumerate(rows):
        E[k, i] = 1.0
    Aw, st = oracle.jvp(Ub, E, d, par)
    assert np.all(st == 0)
    return Aw[rows][:, :]


def test_radiation_block_spectrum_is_the_m1_speeds(oracle):
    """eq. jacobian: the radiation block's eigenvalues are lambda_r1,
    lambda_r2 (twice, in 3D) and lambda_r3 of eqs. lam1-lam3."""
    par = oracle.params(gamma=GAMMA)
    V = I.random_prims(12, 40, fmax=0.95)
    U = oracle.p2c(V, par)
    for c in range(V.shape[1]):
        for d in range(3):
            J = _jacobian(oracle, U[:, c], d, par, [8, 9, 10, 11])
            ev = np.sort(np.linalg.eigvals(J).real)
            l1, l3 = oracle.rad_speeds(V[:, c:c + 1], d)
            E = V[8, c]
            F = V[9:12, c]
            f = np.linalg.norm(F) / E
            cth = F[d] / np.linalg.norm(F)
            xi = (3 + 4 * f * f) / (5 + 2 * math.sqrt(4 - 3 * f * f))
            l2 = cth * (3 * xi - 1) / (2 * f)
            np.testing.assert_allclose(ev, np.sort([l1[0], l2, l2, l3[0]]), rtol=0, atol=1e-9)


def test_magnetofluid_block_extreme_eigenvalues_are_the_quartic_roots(oracle):
    """The magnetofluid block (without the row of B_d, whose flux vanishes) has
    the fast magnetosonic speeds as its extreme eigenvalues: the roots of the
    RMHD quartic that Rad-HLL uses."""
    par = oracle.params(gamma=GAMMA)
    V = I.random_prims(13, 40, vmax=0.9)
    U = oracle.p2c(V, par)
    for c in range(V.shape[1]):
        for d in range(3):
            rows = [q for q in range(8) if q != 5 + d]
            J = _jacobian(oracle, U[:, c], d, par, rows)
            ev = np.linalg.eigvals(J).real
            lo, hi, _ = oracle.fast_speeds(V[:, c:c + 1], d, par)
            assert abs(ev.max() - hi[0]) < 1e-8 and abs(ev.min() - lo[0]) < 1e-8, (c, d, ev, lo, hi)


def test_jvp_flux_matches_the_difference_flux_and_is_consistent(oracle):
    """The exact-JVP face flux equals the eps = 1e-8 difference flux to the
    latter's O(eps) accuracy, and F^(U, U) = F(U) bit for bit."""
    par = oracle.params(gamma=GAMMA)
    parj = oracle.params(gamma=GAMMA, solver=JVP)
    rng = np.random.default_rng(2)
    VL = I.random_prims(5, 3000, vmax=0.9)
    VR = VL * (1 + 0.05 * rng.normal(size=VL.shape))
    VR[1:4] = 0.97 * VL[1:4]
    F1, fb1, _ = oracle.pvm_face(VL, VR, 0.5, 0.5, 0, par)
    F2, fb2, _ = oracle.pvm_face(VL, VR, 0.5, 0.5, 0, parj)
    assert np.all(fb1 == 0) and np.all(fb2 == 0)
    err = np.abs(F1 - F2).max(axis=0) / np.abs(F1).max(axis=0)
    assert err.max() < 2e-6 and np.median(err) < 1e-7, (err.max(), np.median(err))
    Fe, _, _ = oracle.pvm_face(VL, VL, 0.5, 0.5, 1, parj)
    assert np.array_equal(Fe, oracle.flux(VL, 1, par))


@pytest.mark.parametrize("beta_mode", [0, 1, 2])
def test_jvp_flux_scales_the_same_rows_as_the_difference_flux(oracle, beta_mode):
    """eq. beta at tau = 10 on both sides (beta = 0.1): the exact-JVP flux
    applies beta to the same rows as the difference flux (all rows, the
    radiation rows, none), so the two still agree to the difference flux's
    O(eps) accuracy, and the rows beta leaves alone equal those of beta = 1."""
    par = oracle.params(gamma=GAMMA, beta_mode=beta_mode)
    parj = oracle.params(gamma=GAMMA, solver=JVP, beta_mode=beta_mode)
    rng = np.random.default_rng(3)
    VL = I.random_prims(6, 2000, vmax=0.9)
    VR = VL * (1 + 0.05 * rng.normal(size=VL.shape))
    VR[1:4] = 0.97 * VL[1:4]
    F1, fb1, _ = oracle.pvm_face(VL, VR, 10.0, 10.0, 0, par)
    F2, fb2, _ = oracle.pvm_face(VL, VR, 10.0, 10.0, 0, parj)
    assert np.all(fb1 == 0) and np.all(fb2 == 0)
    err = np.abs(F1 - F2).max(axis=0) / np.abs(F1).max(axis=0)
    assert err.max() < 2e-6, err.max()
    F3, _, _ = oracle.pvm_face(VL, VR, 10.0, 10.0, 0, oracle.params(gamma=GAMMA, solver=JVP, beta_mode=2))
    rows = {0: [], 1: list(range(8)), 2: list(range(12))}[beta_mode]
    assert np.array_equal(F2[rows], F3[rows])


@pytest.mark.parametrize("recon", [0, 1, 2, 3])
def test_alfven_wave_with_jvp_reproduces_table4(oracle, recon):
    """Section 4.1, Table 4 with the exact-JVP flux: the same printed rows
    within the tolerances of the difference flux."""
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "alfven_pvm_int8_table4.txt")
    table = {int(r.split()[0]): [float(x) for x in r.split()[1:]] for r in open(path)
             if r.strip() and not r.startswith("#")}
    rel = (1e-3, 3e-2, 5e-2, 5e-2)[recon]
    for n in (16, 32, 64):
        P = I.alfven_1d(n)
        par = oracle.params(gamma=P.gamma, a_rad=P.a_rad, rk_order=3, recon=recon, solver=JVP)
        g = oracle.make_grid(P.shape, P.dx, bc_lo=P.bc_lo, bc_hi=P.bc_hi)
        U, t, _ = run(oracle, g, oracle.p2c(P.V, par), par, 0.0, 0.0, P.cfl, t_end=P.t_end, dx=P.dx)
        V, _, st, _ = oracle.c2p(U, par)
        err = float(np.mean(np.abs(V[3] - P.V[3])))
        assert err == pytest.approx(table[n][recon], rel=rel), (n, err)

