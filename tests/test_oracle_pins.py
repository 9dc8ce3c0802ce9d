"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these checks re-types the oracle's formulas: each compares it with a
value the paper prints, a closed form, an invariant, a special case that
reduces to a textbook result, or an independent computation (exact rational
arithmetic, a scalar bisection, numerical eigenvalues, the direct four-force
of eqs. g0/gi).
"""
from fractions import Fraction
import math
import os

import numpy as np
import pytest

from paper_2212_00370_amd import inputs as I


def rest_state(n, rho=1.0, p=1.0, B=(0, 0, 0), E=1.0, F=(0, 0, 0), v=(0, 0, 0)):
    V = np.zeros((12, n))
    V[0] = rho; V[1:4] = np.array(v, float)[:, None]; V[4] = p
    V[5:8] = np.array(B, float)[:, None]; V[8] = E; V[9:12] = np.array(F, float)[:, None]
    return V


# ---------------------------------------------------------------- closure ----
def xi_exact(f):
    """Eddington factor of eq. xi in exact-ish decimal arithmetic (mpmath-free)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    f = Decimal(float(f))
    return float((3 + 4 * f * f) / (5 + 2 * (4 - 3 * f * f).sqrt()))


def test_eddington_factor_limits(oracle):
    """Section 2.2: xi(0) = 1/3 (diffusion), xi(1) = 1 (free streaming); the
    flux row P_dd / E_r of a beam along d equals xi(f)."""
    par = oracle.params()
    fs = np.array([0.0, 1e-8, 0.1, 0.3, 0.5, 0.7, 0.9, 0.99, 1.0])
    V = rest_state(len(fs), E=2.0)
    V[9] = fs * 2.0
    F = oracle.flux(V, 0, par)
    xi = F[9] / 2.0
    assert xi[0] == pytest.approx(1.0 / 3.0, rel=2e-16, abs=0)
    assert xi[-1] == 1.0
    for f, x in zip(fs, xi):
        assert x == pytest.approx(xi_exact(f), rel=1e-15, abs=0)
    assert np.all(np.diff(xi) > -1e-16) and np.all(np.diff(xi[1:]) > 0)
    # small-f expansion xi ~ 1/3 + f^2/2
    assert xi[2] - 1.0 / 3.0 == pytest.approx(0.01 / 2.0, rel=2e-2)
    # transverse rows: (1 - xi)/2 E for n along d, zero off-diagonal
    Fy = oracle.flux(V, 1, par)
    assert np.allclose(Fy[10] / 2.0, (1 - xi) / 2, rtol=1e-14, atol=1e-16)
    assert np.all(Fy[9] == 0) and np.all(F[10] == 0) and np.all(F[11] == 0)


def test_closure_isotropic_when_no_flux(oracle):
    """F_r = 0: P_r = E_r / 3 delta (Eddington limit, Section 2.2)."""
    V = rest_state(3, E=3.0)
    for d in range(3):
        F = oracle.flux(V, d, oracle.params())
        row = F[9:12, 0]
        expect = np.zeros(3); expect[d] = 1.0
        assert np.allclose(row, expect, rtol=2e-16, atol=0)


# -------------------------------------------------------------- polynomial ----
def exact_internal_poly(k):
    """Expand eq. iterat in exact rationals; coefficients of x^(2m)."""
    p = [Fraction(1)]
    for _ in range(k):
        sq = [Fraction(0)] * (2 * len(p) - 1)
        for a, pa in enumerate(p):
            for b, pb in enumerate(p):
                sq[a + b] += pa * pb
        q = [Fraction(0)] * max(len(sq), 2)
        for m, pm in enumerate(p):
            q[m] += 2 * pm
        for m, s in enumerate(sq):
            q[m] -= s
        q[1] += 1
        while len(q) > 1 and q[-1] == 0:
            q.pop()
        p = [c / 2 for c in q]
    return p


def _printed_p3():
    """alpha_0..alpha_4 from tests/golden (Section 3.2, explicit form of p_3)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "pvm_int8_p3_coefficients.txt")
    vals = [Fraction(ln.strip()) for ln in open(path) if ln.strip() and not ln.startswith("#")]
    assert len(vals) == 5
    return vals


def test_pvm_int8_coefficients_match_paper(oracle):
    """Section 3.2: p_3(x) = x^2(x^2(x^2(a0 x^2 + a1) + a2) + a3) + a4 with the
    printed alpha_0..alpha_4; the oracle's coefficients of x^0 .. x^8 are
    alpha_4 .. alpha_0, and so is the exact expansion of eq. iterat."""
    printed = list(reversed(_printed_p3()))          # x^0 .. x^8
    c = oracle.poly_coef(3)
    assert [Fraction(x) for x in c] == printed
    assert [Fraction(x) for x in exact_internal_poly(3)] == printed


@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_internal_poly_properties(oracle, k):
    """deg p_k = 2^k, p_k(+-1) = 1, p_k(x) >= |x| on [-1, 1], p_k decreasing in k
    (internal approximation of |x| from above, eq. iterat)."""
    c = oracle.poly_coef(k)
    ex = exact_internal_poly(k)
    assert [Fraction(x) for x in c] == ex
    assert 2 * (len(c) - 1) == (0 if k == 0 else 2 ** k)
    x = np.linspace(-1, 1, 2001)
    p = sum(ci * x ** (2 * m) for m, ci in enumerate(c))
    assert sum(ex) == 1
    assert np.all(p >= np.abs(x) - 1e-15)
    if k > 0:
        cp = oracle.poly_coef(k - 1)
        pp = sum(ci * x ** (2 * m) for m, ci in enumerate(cp))
        assert np.all(p <= pp + 1e-15)


# --------------------------------------------------------- prim <-> cons ----
def test_prim_cons_round_trip(oracle):
    """eq. eqU and its inversion: c2p(p2c(V)) = V."""
    par = oracle.params()
    V = I.random_prims(11, 20000)
    U = oracle.p2c(V, par)
    V2, Z, st, it = oracle.c2p(U, par)
    assert np.all(st == 0)
    assert np.max(np.abs(V2[0] - V[0]) / V[0]) < 1e-12
    assert np.max(np.abs(V2[4] - V[4]) / V[4]) < 1e-10
    assert np.max(np.abs(V2[1:4] - V[1:4])) < 1e-12
    assert np.array_equal(V2[5:], V[5:])
    assert it.max() <= 20


def test_failed_recovery_takes_a_floored_state_at_rest(oracle):
    """A conserved state with no admissible primitives (total energy below the
    rest mass, or a non-positive D) fails its recovery and takes the finite
    state the failure reading fixes: rho = D (the density floor when D <= 0),
    v = 0, p = the pressure floor, with B, E_r and F_r passed through. The two
    floors are set to distinct values so that neither stands in for the
    other."""
    par = oracle.params(rho_floor=3e-11, p_floor=7e-10)
    U = np.zeros((12, 2))
    U[0] = [1.0, -1e-3]                      # D
    U[1:4, 0] = [0.3, -0.1, 0.05]            # S
    U[4] = [-0.5, 1.0]                       # tau: tau + D = 0.5 < D in the first
    U[5:8] = np.array([0.2, -0.1, 0.05])[:, None]
    U[8] = 0.4
    U[9:12] = np.array([0.1, 0.0, -0.05])[:, None]
    V, _, st, _ = oracle.c2p(U, par)
    assert np.all(st != 0)
    want = np.zeros((12, 2))
    want[0] = [1.0, 3e-11]
    want[4] = 7e-10
    want[5:] = U[5:]
    assert np.array_equal(V, want), V


def test_prim_cons_closed_forms(oracle):
    """Rest frame: D = rho, S = 0, tau = p/(gamma-1) + B^2/2; hydro (B = 0):
    S = rho h W^2 v, tau = rho h W^2 - p - rho W (eq. eqU)."""
    g = 5.0 / 3.0
    par = oracle.params(gamma=g)
    V = rest_state(1, rho=2.0, p=3.0, B=(0.3, -0.4, 1.2))
    U = oracle.p2c(V, par)[:, 0]
    assert U[0] == 2.0 and np.all(U[1:4] == 0)
    assert U[4] == pytest.approx(3.0 / (g - 1) + 0.5 * (0.09 + 0.16 + 1.44), rel=1e-15)
    v = np.array([0.3, -0.2, 0.5])
    V = rest_state(1, rho=1.5, p=0.7, v=v)
    U = oracle.p2c(V, par)[:, 0]
    W = 1 / math.sqrt(1 - v @ v)
    h = 1 + g / (g - 1) * 0.7 / 1.5
    assert np.allclose(U[1:4], 1.5 * h * W * W * v, rtol=1e-14)
    assert U[4] == pytest.approx(1.5 * h * W * W - 0.7 - 1.5 * W, rel=1e-14)


def test_c2p_warm_start(oracle):
    """Warm-started recovery near a known root needs at most 2 Newton steps and
    reaches the same state to rounding."""
    par = oracle.params()
    V = I.random_prims(12, 5000)
    U = oracle.p2c(V, par)
    _, Z, _, _ = oracle.c2p(U, par)
    Up = U.copy(); Up[:8] *= 1 + 1e-8
    Vc, _, st1, _ = oracle.c2p(Up, par)
    Vw, _, st2, itw = oracle.c2p(Up, par, Z_in=Z)
    assert np.all(st1 == 0) and np.all(st2 == 0)
    assert itw.max() <= 3
    assert np.max(np.abs(Vw[0] - Vc[0]) / Vc[0]) < 1e-13


# ---------------------------------------------------------------- PVM flux ----
def test_consistency_exact(oracle):
    """F^(U, U) = F(U) bit for bit: U_0 = 0 makes every Horner update exactly 0
    (eq. generalflux with U_R = U_L)."""
    par = oracle.params()
    V = I.random_prims(13, 3000)
    for d in range(3):
        F = oracle.flux(V, d, par)
        Fh, fb, _ = oracle.pvm_face(V, V, 2.0, 0.5, d, par)
        assert np.all(fb == 0)
        assert np.array_equal(Fh, F)


def test_k0_is_rusanov(oracle):
    """p_0 = 1: F^ = (F_L + F_R)/2 - beta (U_R - U_L)/2, i.e. Rusanov with
    lambda_max = 1 (eq. iterat with k = 0), bit for bit."""
    par = oracle.params(pvm_k=0, beta_mode=0)
    VL = I.random_prims(14, 2000); VR = I.random_prims(15, 2000)
    tl = np.random.default_rng(0).uniform(0, 5, 2000); tr = np.random.default_rng(1).uniform(0, 5, 2000)
    for d in range(3):
        Fh, fb, _ = oracle.pvm_face(VL, VR, tl, tr, d, par)
        UL, UR = oracle.p2c(VL, par), oracle.p2c(VR, par)
        FL, FR = oracle.flux(VL, d, par), oracle.flux(VR, d, par)
        beta = np.minimum(np.minimum(1 / np.maximum(tl, 1e-300), 1 / np.maximum(tr, 1e-300)), 1.0)
        ref = 0.5 * (FL + FR) - 0.5 * (beta * (UR - UL))
        assert np.array_equal(Fh, ref)


def test_contact_eigenvector(oracle):
    """Density jump with uniform v, p, B and radiation: F(U) = v_x U + const
    along the jump, so Q U_0 = p_3(v_x) U_0 (Section 3.2, PVM with
    lambda_max = 1)."""
    rng = np.random.default_rng(3)
    n = 200
    VL = I.random_prims(16, n, vmax=0.8)
    VR = VL.copy()
    VR[0] = VL[0] * np.exp(rng.uniform(-1.5, 1.5, n))
    par = oracle.params(beta_mode=2)
    d = 0
    Fh, fb, _ = oracle.pvm_face(VL, VR, 0.0, 0.0, d, par)
    assert np.all(fb == 0)
    UL, UR = oracle.p2c(VL, par), oracle.p2c(VR, par)
    FL, FR = oracle.flux(VL, d, par), oracle.flux(VR, d, par)
    U4 = (0.5 * (FL + FR) - Fh) * 2.0
    c = oracle.poly_coef(3)
    vx = VL[1]
    p3 = sum(ci * vx ** (2 * m) for m, ci in enumerate(c))
    U0 = UR - UL
    scale = np.abs(FL).max(axis=0) + np.abs(FR).max(axis=0)
    err = np.abs(U4 - p3 * U0).max(axis=0) / scale
    assert err.max() < 1e-6           # finite-difference noise ~ u / eps
    assert np.median(err) < 1e-7


def test_free_streaming_face_is_upwind(oracle):
    """f = 1 beam along +x (F_r = E_r e_x): the radiation flux is F = 1 * U on
    that family, p_3(1) = 1, so with beta = 1 the radiation rows of F^ are the
    upwind (left) state (Section 2.2 free-streaming limit, eqs. lam1-lam3)."""
    n = 50
    rng = np.random.default_rng(4)
    EL = np.exp(rng.uniform(-3, 2, n)); ER = np.exp(rng.uniform(-3, 2, n))
    VL = rest_state(n, rho=1.0, p=1.0); VR = VL.copy()
    VL[8] = EL; VL[9] = EL; VR[8] = ER; VR[9] = ER
    par = oracle.params()
    Fh, fb, _ = oracle.pvm_face(VL, VR, 0.0, 0.0, 0, par)
    # finite-difference noise of the eps = 1e-8 chain: ~ u / eps * max(E_L, E_R)
    scale = np.maximum(EL, ER)
    assert np.max(np.abs(Fh[8] - EL) / scale) < 1e-6
    assert np.max(np.abs(Fh[9] - EL) / scale) < 1e-6
    assert np.all(Fh[10:12] == 0)
    assert np.all(Fh[0] == 0)      # fluid at rest and uniform: no mass flux


def test_beta_limits(oracle):
    """eq. beta: beta = min(1/tau_L, 1/tau_R, 1) multiplies the viscous term."""
    par0 = oracle.params(pvm_k=0, beta_mode=0)
    VL = I.random_prims(17, 10); VR = I.random_prims(18, 10)
    UL, UR = oracle.p2c(VL, par0), oracle.p2c(VR, par0)
    FL, FR = oracle.flux(VL, 0, par0), oracle.flux(VR, 0, par0)
    for tl, tr, b in [(0.0, 0.0, 1.0), (0.5, 0.9, 1.0), (4.0, 2.0, 0.25), (3.0, 10.0, 0.1)]:
        Fh, _, _ = oracle.pvm_face(VL, VR, tl, tr, 0, par0)
        assert np.allclose(Fh, 0.5 * (FL + FR) - 0.5 * b * (UR - UL), rtol=1e-14, atol=1e-14)
    # radiation-only mode leaves the fluid rows unscaled
    par1 = oracle.params(pvm_k=0, beta_mode=1)
    Fh, _, _ = oracle.pvm_face(VL, VR, 10.0, 10.0, 0, par1)
    assert np.allclose(Fh[:8], 0.5 * (FL + FR)[:8] - 0.5 * (UR - UL)[:8], rtol=1e-14, atol=1e-14)
    assert np.allclose(Fh[8:], 0.5 * (FL + FR)[8:] - 0.05 * (UR - UL)[8:], rtol=1e-14, atol=1e-14)


# ----------------------------------------------------------------- speeds ----
def test_m1_speed_limits(oracle):
    """eqs. lam1-lam3: f -> 0 gives +-1/sqrt(3); f = 1 gives cos(theta);
    |lambda| <= 1."""
    par = oracle.params()
    V = rest_state(4, rho=1.0, p=1e-14, E=1.0)
    V[9:12, 1] = [1.0, 0, 0]
    V[9:12, 2] = [0.6, 0.8, 0]
    V[9:12, 3] = [0.3, 0.4, 0]
    sx = oracle.cell_speed(V, 0, par)
    sy = oracle.cell_speed(V, 1, par)
    assert sx[0] == pytest.approx(1 / math.sqrt(3), rel=1e-15)
    assert sx[1] == pytest.approx(1.0, rel=1e-15)
    assert sx[2] == pytest.approx(0.6, rel=1e-12)
    assert sy[2] == pytest.approx(0.8, rel=1e-12)
    assert sy[1] < 1e-6
    V2 = I.random_prims(19, 5000)
    for d in range(3):
        s = oracle.cell_speed(V2, d, par)
        assert np.all(s <= 1.0 + 1e-15) and np.all(s > 0)


def test_m1_speeds_are_jacobian_eigenvalues(oracle):
    """The radiation block's extreme eigenvalues (eqs. lam1, lam3) equal those of
    the numerically differentiated M1 flux (eq. jacobian)."""
    par = oracle.params()
    rng = np.random.default_rng(5)
    for _ in range(40):
        f = rng.uniform(0.05, 0.95)
        m = rng.normal(size=3); m /= np.linalg.norm(m)
        V0 = rest_state(1, rho=1.0, p=1e-14, E=1.0, F=tuple(f * m))
        J = np.zeros((4, 4))
        h = 1e-6
        for j in range(4):
            Vp = V0.copy(); Vm = V0.copy()
            Vp[8 + j] += h; Vm[8 + j] -= h
            Fp = oracle.flux(Vp, 0, par)[8:12, 0]; Fm = oracle.flux(Vm, 0, par)[8:12, 0]
            J[:, j] = (Fp - Fm) / (2 * h)
        ev = np.linalg.eigvals(J).real
        s = oracle.cell_speed(V0, 0, par)[0]
        assert s == pytest.approx(np.max(np.abs(ev)), abs=2e-7)


def test_fluid_speed_hydro_sound(oracle):
    """Fluid at rest, B = 0: the fast speed bound is the sound speed
    cs^2 = gamma p / (rho h); with radiation negligible (f = 0 gives 1/sqrt 3,
    so the check uses a hot gas with cs > 1/sqrt 3)."""
    g = 5.0 / 3.0
    par = oracle.params(gamma=g)
    V = rest_state(1, rho=1.0, p=100.0, E=1e-6)
    cs = math.sqrt(g * 100.0 / (1 + g / (g - 1) * 100.0))
    assert cs > 1 / math.sqrt(3)
    assert oracle.cell_speed(V, 0, par)[0] == pytest.approx(cs, rel=1e-14)


def test_fluid_speed_across_the_field_is_the_fast_speed(oracle):
    """Magnetised gas at rest with B perpendicular to d: the fluid part of the
    CFL speed (reading R19, the bound a^2 = c_s^2 + c_a^2 - c_s^2 c_a^2 with
    c_a^2 = b^2 / (rho h + b^2)) is the RMHD fast speed across the field, the
    extreme root of the quartic. A hot, strongly magnetised gas puts it above
    the radiation's 1/sqrt(3) and well above c_s alone."""
    g = 5.0 / 3.0
    par = oracle.params(gamma=g)
    rho, p, B = 1.0, 2.0, 3.0
    V = rest_state(1, rho=rho, p=p, B=(0.0, B, 0.0), E=1e-6)
    rhoh = rho + g / (g - 1) * p
    cs2 = g * p / rhoh
    ca2 = B * B / (rhoh + B * B)
    cf = math.sqrt(cs2 + ca2 - cs2 * ca2)
    assert cf > 1 / math.sqrt(3) and cf > 1.2 * math.sqrt(cs2)
    assert oracle.cell_speed(V, 0, par)[0] == pytest.approx(cf, rel=1e-14)
    lo, hi, _ = oracle.fast_speeds(V, 0, par)
    assert hi[0] == pytest.approx(cf, rel=1e-10) and lo[0] == pytest.approx(-cf, rel=1e-10)


def test_cfl_speed_takes_every_direction_of_the_grid(oracle):
    """The CFL rule's signal speed is the maximum over the cells and over all
    directions of the grid: a uniform hot gas (B = 0) moving along the last
    axis of a 2D or 3D grid has (v + c_s)/(1 + v c_s) there, above its speed
    along x, and no other value."""
    g = 5.0 / 3.0
    par = oracle.params(gamma=g)
    rho, p, v = 1.0, 3.0, 0.8
    rhoh = rho + g / (g - 1) * p
    cs = math.sqrt(g * p / rhoh)
    want = (v + cs) / (1 + v * cs)
    for shape in ((4, 3), (3, 2, 2)):
        n = int(np.prod(shape))
        vel = [0.0, 0.0, 0.0]
        vel[len(shape) - 1] = v
        U = oracle.p2c(rest_state(n, rho=rho, p=p, E=1e-6, v=vel), par)
        s, nf = oracle.max_speed(oracle.make_grid(shape, (0.1,) * len(shape)), U, par)
        assert nf == 0
        assert s == pytest.approx(want, rel=1e-12), (shape, s, want)


def test_fluid_speed_moving_gas_is_velocity_addition(oracle):
    """B = 0, gas moving along d with speed v: the fast-speed bound is the
    relativistic sum of v and the sound speed, (v + c_s)/(1 + v c_s) downstream
    and (v - c_s)/(1 - v c_s) upstream. A hot gas (c_s = 0.5..0.7) moving at
    v = 0.1..0.8 puts the larger of the two above the radiation's 1/sqrt(3)."""
    g = 5.0 / 3.0
    par = oracle.params(gamma=g)
    for d in range(3):
        for v in (0.1, 0.3, 0.5, 0.8):
            for p in (0.8, 3.0, 100.0):
                vel = [0.0, 0.0, 0.0]
                vel[d] = v
                V = rest_state(1, rho=1.0, p=p, E=1e-6, v=tuple(vel))
                h = 1 + g / (g - 1) * p
                cs = math.sqrt(g * p / h)
                lp = (v + cs) / (1 + v * cs)
                lm = (v - cs) / (1 - v * cs)
                expect = max(abs(lp), abs(lm), 1 / math.sqrt(3))
                assert max(abs(lp), abs(lm)) > 1 / math.sqrt(3) or p < 1.0
                assert oracle.cell_speed(V, d, par)[0] == pytest.approx(expect, rel=1e-13), (d, v, p)


# --------------------------------------------------------------- implicit ----
def static_solution(Estar, tau_t, rho, B2, h, kap, a_rad, g):
    """Static medium, no flux: E = (E* + h rho kappa a T^4)/(1 + h rho kappa)
    with p from p/(g-1) + B^2/2 + E(p) = tau_t (monotone in p: bisection)."""
    def E_of(p):
        T = p / rho
        return (Estar + h * rho * kap * a_rad * T ** 4) / (1 + h * rho * kap)

    lo, hi = 0.0, (g - 1) * (tau_t - 0.5 * B2)
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if mid / (g - 1) + 0.5 * B2 + E_of(mid) > tau_t:
            hi = mid
        else:
            lo = mid
    p = 0.5 * (lo + hi)
    return E_of(p), p


@pytest.mark.parametrize("method", [0, 1])
def test_implicit_static_closed_form(oracle, method):
    """Static limit of eqs. g0/gi (u = 0, F* = 0): scalar root, bisection."""
    g = 5.0 / 3.0
    rng = np.random.default_rng(6)
    for _ in range(20):
        rho = math.exp(rng.uniform(-2, 2)); p = math.exp(rng.uniform(-4, 2)); E = math.exp(rng.uniform(-6, 2))
        B = rng.uniform(-1, 1, 3)
        a = E / (p / rho) ** 4 * math.exp(rng.uniform(-3, 3))
        kap = math.exp(rng.uniform(-4, 7)); sig = math.exp(rng.uniform(-4, 5)); h = 1e-3
        par = oracle.params(gamma=g, a_rad=a, imp_method=method)
        V = rest_state(1, rho=rho, p=p, B=tuple(B), E=E)
        U = oracle.p2c(V, par)
        Un, st, it = oracle.implicit(U, h, kap, sig, par)
        assert st[0] == 0
        Eex, pex = static_solution(E, U[4, 0] + U[8, 0], rho, float(B @ B), h, kap, a, g)
        assert Un[8, 0] == pytest.approx(Eex, rel=1e-12)
        assert np.all(Un[9:12, 0] == 0) and np.all(Un[1:4, 0] == 0)
        Vn, _, _, _ = oracle.c2p(Un, par)
        assert Vn[4, 0] == pytest.approx(pex, rel=1e-10)


def test_implicit_energy_floor(oracle):
    """A non-positive explicit E_r fails the cell (status 1, state kept) unless
    e_floor > 0; then E* is raised to e_floor with tau + E_r kept, so the gas
    pays (counted): in the static limit the result is the scalar root of
    eqs. g0/gi with E* = e_floor and the original total tau_t."""
    g = 5.0 / 3.0
    rho, p, E, B = 1.0, 0.5, -0.01, (0.2, -0.1, 0.3)
    a, kap, h, floor = 0.3, 2.0, 1e-2, 0.05
    V = rest_state(1, rho=rho, p=p, B=B, E=E)
    par0 = oracle.params(gamma=g, a_rad=a)
    U = oracle.p2c(V, par0)
    Un, st, _ = oracle.implicit(U, h, kap, 0.0, par0)
    assert st[0] == 1 and np.array_equal(Un, U)
    par = oracle.params(gamma=g, a_rad=a, e_floor=floor)
    Un, st, _ = oracle.implicit(U, h, kap, 0.0, par)
    assert st[0] == 0
    tau_t = U[4, 0] + U[8, 0]
    assert Un[4, 0] + Un[8, 0] == pytest.approx(tau_t, rel=1e-14)
    Eex, pex = static_solution(floor, tau_t, rho, float(np.dot(B, B)), h, kap, a, g)
    assert Un[8, 0] == pytest.approx(Eex, rel=1e-12)
    Vn, _, _, _ = oracle.c2p(Un, par)
    assert Vn[4, 0] == pytest.approx(pex, rel=1e-10)


def test_implicit_stiff_limit(oracle):
    """h rho kappa -> infinity: radiation reaches equilibrium E = a_R T^4."""
    g = 5.0 / 3.0
    par = oracle.params(gamma=g, a_rad=0.5)
    V = rest_state(1, rho=1.0, p=1.0, E=0.2)
    U = oracle.p2c(V, par)
    Un, st, _ = oracle.implicit(U, 1.0, 1e12, 0.0, par)
    Vn, _, _, _ = oracle.c2p(Un, par)
    T = Vn[4, 0] / Vn[0, 0]
    assert st[0] == 0
    assert Un[8, 0] == pytest.approx(0.5 * T ** 4, rel=1e-10)


def implicit_cases(n, seed, kmax=1e3):
    rng = np.random.default_rng(seed)
    V = I.random_prims(seed, n, vmax=0.7)
    kap = np.exp(rng.uniform(math.log(1e-2), math.log(kmax), n))
    sig = np.exp(rng.uniform(math.log(1e-2), math.log(kmax), n))
    return V, kap, sig


def test_implicit_conserves_totals(oracle):
    """eqs. totale/totalm: tau + E_r and S + F_r are unchanged by the implicit
    step; D and B are untouched."""
    V, kap, sig = implicit_cases(2000, 20)
    par = oracle.params(a_rad=0.3)
    U = oracle.p2c(V, par)
    Un, st, _ = oracle.implicit(U, 2e-3, kap, sig, par)
    ok = st == 0
    assert ok.mean() > 0.99
    assert np.array_equal(Un[0, ok], U[0, ok]) and np.array_equal(Un[5:8][:, ok], U[5:8][:, ok])
    e0 = U[4] + U[8]; e1 = Un[4] + Un[8]
    assert np.max(np.abs(e1 - e0)[ok] / np.abs(e0[ok])) < 4e-16
    m0 = U[1:4] + U[9:12]; m1 = Un[1:4] + Un[9:12]
    assert np.max(np.abs(m1 - m0)[:, ok]) < 1e-15 * np.max(np.abs(m0))


def test_implicit_solves_backward_euler_with_direct_four_force(oracle):
    """The implicit result satisfies E = E* - h G^0, F = F* - h G^i with G from
    eqs. g0 and gi evaluated directly (independent of the matrix C; pins the
    sign of its C_{i+1,j+1} block)."""
    V, kap, sig = implicit_cases(1500, 21)
    par = oracle.params(a_rad=0.3)
    U = oracle.p2c(V, par)
    h = 2e-3
    Un, st, _ = oracle.implicit(U, h, kap, sig, par)
    ok = st == 0
    # Cells where the |F| <= E limit did not act on input or output.
    f_in = np.linalg.norm(U[9:12], axis=0) / U[8]
    f_out = np.linalg.norm(Un[9:12], axis=0) / Un[8]
    sel = ok & (f_in < 1) & (f_out < 0.999999)
    assert sel.mean() > 0.9
    Vn, _, _, _ = oracle.c2p(Un, par)
    G = oracle.four_force(Vn, kap, sig, par)
    resE = Un[8] - (U[8] - h * G[0])
    resF = Un[9:12] - (U[9:12] - h * G[1:4])
    scale = np.maximum(np.abs(U[8]), np.abs(Un[8])) + h * np.abs(G).max(axis=0)
    err = np.maximum(np.abs(resE), np.abs(resF).max(axis=0)) / scale
    assert np.max(err[sel]) < 1e-10


def test_picard_and_newton_reach_the_same_root(oracle):
    """Where the paper's lagged (Picard) iteration contracts, it and Newton find
    the same root of the backward-Euler system."""
    V, kap, sig = implicit_cases(1000, 22, kmax=10.0)
    parP = oracle.params(a_rad=0.01, imp_method=2, imp_maxit=200)
    parN = oracle.params(a_rad=0.01, imp_method=1)
    U = oracle.p2c(V, parP)
    UP, sP, _ = oracle.implicit(U, 1e-3, kap, sig, parP)
    UN, sN, _ = oracle.implicit(U, 1e-3, kap, sig, parN)
    ok = (sP == 0) & (sN == 0)
    assert ok.mean() > 0.95
    sc = np.abs(U[8]) + np.linalg.norm(U[9:12], axis=0)
    assert np.max(np.abs(UP[8] - UN[8])[ok] / sc[ok]) < 1e-12
    assert np.max(np.abs(UP[9:12] - UN[9:12])[:, ok] / sc[ok]) < 1e-12


def test_implicit_no_coupling_is_identity(oracle):
    """kappa = sigma = 0: no source, U unchanged."""
    V = I.random_prims(23, 500)
    par = oracle.params()
    U = oracle.p2c(V, par)
    Un, st, _ = oracle.implicit(U, 1e-2, 0.0, 0.0, par)
    assert np.all(st == 0)
    assert np.array_equal(Un[[0, 5, 6, 7]], U[[0, 5, 6, 7]])
    assert np.allclose(Un, U, rtol=1e-15, atol=1e-15)
