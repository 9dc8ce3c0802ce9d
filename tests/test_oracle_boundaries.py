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
