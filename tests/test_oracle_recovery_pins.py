"""Rounding-bound pins of the primitive recovery's evaluation of its residual.

The recovery (Newton on Z = rho h W^2 with a bracket; the paper leaves the
algorithm to the authors' RMHD code) evaluates, at each iterate Z,
  v^2(Z) = [S^2 + (S.B)^2 (2Z + B^2)/Z^2] / (Z + B^2)^2,
  1/W = sqrt(1 - v^2), rho = D/W, p = (gamma-1)/gamma (Z/W^2 - rho),
  f(Z) = Z + B^2 - p - B^2/(2 W^2) - (S.B)^2/(2 Z^2) - (tau + D)
(closed relations implied by eq. eqU). Three rearrangements of this
evaluation are made for speed, each the same quantity in exact arithmetic:
  (a) 1/Z and 1/(Z + B^2) are formed from one reciprocal of Z (Z + B^2);
  (b) f and f' are returned multiplied by 1/W (same signs, same Newton step);
  (c) a recovered state takes W from the final evaluation at the converged Z,
      not from its recovered velocity components.
Each test below compares the rearranged quantity with its plain form,
evaluated in 80-digit decimal arithmetic from the exact binary64 inputs, and
asserts a bound stated in units of the binary64 rounding unit u = 2^-53.
f' is compared with a central difference of the plain f in that precision,
so the derivative formula itself is pinned as well.
"""
from decimal import Decimal, getcontext

import numpy as np
import pytest

from paper_2212_00370_amd import inputs as I

U53 = 2.0 ** -53


def dec(x):
    return Decimal(float(x))


def plain_f(Z, D, S2, SB, B2, Et, g):
    """f(Z) and 1 - v^2(Z) in the plain form of the module docstring."""
    v2 = (S2 + SB * SB * (2 * Z + B2) / (Z * Z)) / ((Z + B2) ** 2)
    l2 = 1 - v2
    W = 1 / l2.sqrt()
    rho = D / W
    p = (g - 1) / g * (Z * l2 - rho)
    return Z + B2 - p - B2 * l2 / 2 - SB * SB / (2 * Z * Z) - Et, l2


@pytest.fixture(scope="module")
def evals(oracle):
    """Residual evaluations at the root and at Z up to 30 % away from it, over
    i.i.d. states up to |v| = 0.99 (W ~ 7)."""
    getcontext().prec = 80
    par = oracle.params(gamma=5.0 / 3.0)
    V = I.random_prims(7, 1500, vmax=0.99)
    U = oracle.p2c(V, par)
    _, Zr, st, _ = oracle.c2p(U, par)
    assert np.all(st == 0)
    rng = np.random.default_rng(1)
    Z = Zr * np.exp(rng.uniform(-0.3, 0.3, Zr.size))
    Z[:300] = Zr[:300]
    e = oracle.c2p_eval(U, Z, par)
    assert e["ok"].mean() > 0.7
    return U, Z, e


def test_one_reciprocal_gives_both_inverses(evals):
    """(a): 1/Z = (Z + B^2) * r and 1/(Z + B^2) = Z * r with r = 1/(Z (Z + B^2))
    are within 3 u (three roundings) and 4 u (plus the rounding of Z + B^2) of
    the exact inverses."""
    U, Z, e = evals
    B2 = (U[5] * U[5] + U[6] * U[6]) + U[7] * U[7]      # as binary64 forms it
    for c in range(U.shape[1]):
        z = dec(Z[c])
        assert abs(dec(e["iZ"][c]) * z - 1) <= Decimal(3 * U53), c
        assert abs(dec(e["iZb"][c]) * (z + dec(B2[c])) - 1) <= Decimal(4 * U53), c


def test_scaled_residual_and_slope_match_plain_forms(evals):
    """(b): f/W and f'/W as returned equal the plain f times 1/W, and the plain
    df/dZ (an 80-digit central difference of f) times 1/W, to
    16 u * (sum of |terms| of f) and 8 u W^2 * (sum of |terms| of f'); the
    W^2 is the conditioning of 1 - v^2 near v = 1."""
    U, Z, e = evals
    g = Decimal(5) / Decimal(3)
    nchk = 0
    for c in np.nonzero(e["ok"] == 1)[0]:
        z = dec(Z[c]); D = dec(U[0, c])
        S = [dec(U[1 + j, c]) for j in range(3)]; B = [dec(U[5 + j, c]) for j in range(3)]
        S2 = sum(s * s for s in S); SB = sum(s * b for s, b in zip(S, B)); B2 = sum(b * b for b in B)
        Et = dec(U[4, c]) + D
        f, l2 = plain_f(z, D, S2, SB, B2, Et, g)
        h = z * Decimal("1e-30")
        fp, l2p = plain_f(z + h, D, S2, SB, B2, Et, g)
        fm, l2m = plain_f(z - h, D, S2, SB, B2, Et, g)
        df = (fp - fm) / (2 * h)
        dv2 = -(l2p - l2m) / (2 * h)
        iW = l2.sqrt(); W = 1 / iW
        vB2 = SB * SB / (z * z)
        scale_f = z + B2 + abs(Et) + vB2
        scale_df = 1 + (g - 1) / g * (l2 + abs(dv2) * (D * W / 2 + z)) + B2 * abs(dv2) / 2 + vB2 / z
        assert abs(dec(e["fW"][c]) - f * iW) <= Decimal(16 * U53) * scale_f * iW, c
        assert abs(dec(e["dfW"][c]) - df * iW) <= Decimal(8 * U53) * W * W * scale_df * iW, c
        assert abs(dec(e["iW"][c]) - iW) <= Decimal(8 * U53) * W * W * iW, c
        nchk += 1
    assert nchk > 1000


def test_recovered_lorentz_factor_matches_recovered_velocity(oracle):
    """(c): the W a recovered state carries (from the final evaluation at the
    converged Z) equals 1/sqrt(1 - |v|^2) of its recovered velocity to
    8 u W^2 relative (1 - v^2 loses W^2 digits near v = 1), over states up to
    |v| = 0.99 and in the rest frame exactly."""
    getcontext().prec = 80
    par = oracle.params(gamma=4.0 / 3.0)
    V = I.random_prims(8, 3000, vmax=0.99)
    V[1:4, :50] = 0.0
    U = oracle.p2c(V, par)
    Vr, lw, st = oracle.c2p_lw(U, par)
    assert np.all(st == 0)
    for c in range(U.shape[1]):
        v = [dec(Vr[1 + j, c]) for j in range(3)]
        l2v = 1 - sum(x * x for x in v)
        Wv = 1 / l2v.sqrt()
        Wr = 1 / dec(lw[1, c])
        assert abs(Wr / Wv - 1) <= Decimal(8 * U53) * Wv * Wv, c
        assert abs(dec(lw[0, c]) - l2v) <= Decimal(8 * U53) * Wv * Wv * l2v, c
    assert np.all(lw[1, :50] == 1.0) and np.all(lw[0, :50] == 1.0)
