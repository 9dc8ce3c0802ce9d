"""Pins of the oracle's boundary handling (the Section 4 test setups use
periodic, outflow and inflow boundaries). At a boundary face whose two sides
reconstruct to the same state, the PVM flux reduces to the physical flux of
that state bit for bit (F^(U, U) = F(U)); the tests arrange exactly that and
check every boundary face, so a ghost cell mapped to the wrong interior cell,
the wrong transverse inflow state or an ignored inflow mask fails."""
import numpy as np

from paper_2212_00370_amd import inputs as I


def _flux(oracle, U, d, par):
    V, _, st, _ = oracle.c2p(U, par)
    assert np.all(st == 0)
    return oracle.flux(V, d, par)


def test_outflow_boundary_faces_carry_the_boundary_cell_flux(oracle):
    """Outflow = zero gradient: the ghosts copy the nearest interior cell, so
    the slopes vanish at the boundary and each boundary face carries the
    physical flux of its boundary cell, in both directions, on both sides."""
    nx, ny = 7, 5
    par = oracle.params(gamma=5 / 3)
    V = I.random_prims(31, nx * ny, vmax=0.5)
    U = oracle.p2c(V, par)
    g = oracle.make_grid((nx, ny), (0.1, 0.13))
    F = oracle.face_fluxes(g, U, 0.0, 0.0, par)[0]
    Fx, Fy = _flux(oracle, U, 0, par), _flux(oracle, U, 1, par)
    for j in range(ny):
        assert np.array_equal(F[0][:, (nx + 1) * j], Fx[:, nx * j])                    # x lo
        assert np.array_equal(F[0][:, (nx + 1) * j + nx], Fx[:, nx * j + nx - 1])      # x hi
    for i in range(nx):
        assert np.array_equal(F[1][:, i], Fy[:, i])                                    # y lo
        assert np.array_equal(F[1][:, nx * ny + i], Fy[:, nx * (ny - 1) + i])          # y hi


def test_inflow_mask_and_transverse_state(oracle):
    """Inflow on the lo side of the last axis: where the mask is set the ghosts
    hold that column's own inflow state, elsewhere they copy the boundary cell.
    Rows 0 and 1 of a masked column equal its inflow state, so its boundary
    face carries F(U_in[i]); unmasked columns carry F of their own cell."""
    nx, ny = 6, 5
    par = oracle.params(gamma=5 / 3)
    V = I.random_prims(32, nx * ny, vmax=0.5)
    Vin = I.random_prims(33, nx, vmax=0.5)
    mask = np.array([1, 0, 1, 1, 0, 1], dtype=np.uint8)
    for i in range(nx):
        if mask[i]:
            V[:, i] = Vin[:, i]
            V[:, nx + i] = Vin[:, i]
        else:
            V[:, nx + i] = V[:, i]
    U = oracle.p2c(V, par)
    Uin = np.ascontiguousarray(oracle.p2c(Vin, par))
    g = oracle.make_grid((nx, ny), (0.1, 0.13), bc_lo=(1, 2, 1), inflow_U=Uin, inflow_mask=mask)
    F = oracle.face_fluxes(g, U, 0.0, 0.0, par)[0]
    Fy_in, Fy = _flux(oracle, Uin, 1, par), _flux(oracle, U, 1, par)
    for i in range(nx):
        want = Fy_in[:, i] if mask[i] else Fy[:, i]
        assert np.array_equal(F[1][:, i], want), i


def test_inflow_ghost_takes_the_opacity_of_its_column(oracle):
    """The optical depth of an inflow ghost (eq. limits, tau = rho W (kappa +
    sigma) dx, entering beta at the inflow face) uses the inflow state's D and
    the opacities of the interior cell it borders, column by column: with
    Godunov states and opacities that vary along x, each masked column's
    boundary face equals the PVM face flux of (U_in, cell) with those two
    depths (to 1e-12: the face takes 1/W from the recovery)."""
    nx, ny = 6, 4
    dy = 0.13
    par = oracle.params(gamma=5 / 3, recon=0)
    V = I.random_prims(34, nx * ny, vmax=0.5)
    Vin = I.random_prims(35, nx, vmax=0.5)
    mask = np.array([1, 1, 0, 1, 1, 1], dtype=np.uint8)
    rng = np.random.default_rng(7)
    kap = 10.0 ** rng.uniform(0.5, 2.5, nx * ny)
    sig = 10.0 ** rng.uniform(0.0, 2.0, nx * ny)
    U = oracle.p2c(V, par)
    Uin = np.ascontiguousarray(oracle.p2c(Vin, par))
    g = oracle.make_grid((nx, ny), (0.1, dy), bc_lo=(1, 2, 1), inflow_U=Uin, inflow_mask=mask)
    F = oracle.face_fluxes(g, U, kap, sig, par)[0]
    Vc, _, st, _ = oracle.c2p(U, par)
    Vi, _, st2, _ = oracle.c2p(Uin, par)
    assert np.all(st == 0) and np.all(st2 == 0)
    for i in np.nonzero(mask)[0]:
        tl = Uin[0, i] * (kap[i] + sig[i]) * dy
        tr = U[0, i] * (kap[i] + sig[i]) * dy
        assert max(tl, tr) > 2.0                 # beta < 1 at this face
        want, _, _ = oracle.pvm_face(Vi[:, i:i + 1], Vc[:, i:i + 1], tl, tr, 1, par)
        scale = np.abs(want[:, 0]) + 1e-12 * np.max(np.abs(want))
        assert np.max(np.abs(F[1][:, i] - want[:, 0]) / scale) < 1e-12, i
