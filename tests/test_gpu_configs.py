"""GPU parity over whole runs of the benchmark configurations that the
per-step tests sample only briefly.

* The 1D Riemann problems (400 cells on [0, 1], seeded L/R states, PLM
  MinMod, PVM-int-8, IMEX RK2, CFL 0.4) run to t = 0.4, every step from the
  same input on both sides (the GPU state is handed to the oracle each step):
  the signal speed, the state and the failure counters must equal the
  oracle's bit for bit at every step, for all 32 seeds.
  Seeds 15 and 16 stop in their first step on the oracle as on the GPU (an
  inadmissible explicit fluid state at the contact, and a negative E_r in an
  optically thin cell next to a thick one); they are expected failures of the
  run to t = 0.4, and their first step, failures included, is compared
  separately.
* The 2D blast with beta scaling all twelve rows of the viscosity (the
  literal eq. beta), on a weaker blast that this form survives.
"""
import numpy as np
import pytest

from paper_2212_00370_amd import inputs as I

pytestmark = pytest.mark.gpu

TOL = 1e-12
FAILING_FIRST_STEP = {
    15: "the explicit fluid state right of the contact has no admissible primitive state (cold, fast shear)",
    16: "E_r < 0 after the explicit stage in the optically thin cell next to a thick one, and a failed implicit solve",
}


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2212_00370_amd import rrmhd
    return rrmhd


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def relerr(a, b):
    scale = np.maximum(np.abs(b), 1e-3 * np.max(np.abs(b), axis=1, keepdims=True))
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.abs(a - b) / scale))


def oracle_params(oracle, p):
    return oracle.params(gamma=p.gamma, a_rad=p.a_rad, t_coeff=p.t_coeff, pvm_eps=p.pvm_eps,
                         c2p_tol=p.c2p_tol, imp_tol=p.imp_tol, rho_floor=p.rho_floor, p_floor=p.p_floor,
                         pvm_k=p.pvm_k, beta_mode=p.beta_mode, recon=p.recon, rk_order=p.rk_order,
                         c2p_maxit=p.c2p_maxit, imp_maxit=p.imp_maxit, imp_picard_it=p.imp_picard_it,
                         imp_method=p.imp_method, e_floor=p.e_floor, solver=p.solver)


def run_compare(R, oracle, P, t_end=None, max_steps=None, **kw):
    """Step P on the GPU and the oracle from identical input each step until
    t_end (last step clipped) or max_steps; returns (steps, bitwise, reports
    of the failing step or None)."""
    import torch
    p = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad, **kw)
    op = oracle_params(oracle, p)
    g = R.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    og = oracle.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    s = R.Solver(g, p)
    opac = R.make_opacities(dev(torch, P.kappa), dev(torch, P.sigma))
    Uin = oracle.p2c(P.V, op)
    Ud = dev(torch, Uin)
    t, n, bit = 0.0, 0, True
    try:
        while True:
            if t_end is not None and t >= t_end * (1 - 1e-14):
                break
            if max_steps is not None and n >= max_steps:
                break
            sm_g = s.max_speed(Ud)
            sm_o, nf = oracle.max_speed(og, Uin, op)
            assert sm_g == sm_o, (n, sm_g, sm_o)
            h = P.cfl * min(P.dx) / sm_g
            if t_end is not None:
                h = min(h, t_end - t)
            s.step(Ud, h, opac)
            rep_g = s.report()
            Uo, st, rep_o = oracle.step(og, Uin, h, P.kappa, P.sigma, op)
            Ug = Ud.cpu().numpy()
            e = relerr(Ug, Uo)
            assert e <= TOL, (n, e)
            bit = bit and np.array_equal(Ug, Uo)
            assert rep_g["c2p_fail"] == rep_o.c2p_fail + nf, n
            assert rep_g["imp_fail"] == rep_o.imp_fail, n
            assert rep_g["pvm_fallback"] == rep_o.pvm_fallback, n
            assert rep_g["first_bad_cell"] == rep_o.first_bad_cell, n
            if st != 0:
                return n, bit, (rep_g, rep_o)
            Uin = Ug
            t += h
            n += 1
    finally:
        s.close()
    return n, bit, None


@pytest.mark.parametrize("seed", [
    pytest.param(s, marks=pytest.mark.xfail(strict=True, reason=FAILING_FIRST_STEP[s])) if s in FAILING_FIRST_STEP
    else s for s in range(32)])
def test_riemann_1d_to_t_end(R, oracle, seed):
    """All 32 seeded Riemann problems, 400 cells, to t = 0.4 (270-400 steps
    each), bitwise every step."""
    oracle.threads(0)
    P = I.riemann_1d(seed, 400)
    n, bit, fail = run_compare(R, oracle, P, t_end=P.t_end)
    print(f"riemann seed {seed}: {n} steps, bitwise {bit}", flush=True)
    assert fail is None, fail
    assert bit
    assert n > 200


@pytest.mark.parametrize("seed", sorted(FAILING_FIRST_STEP))
def test_riemann_1d_failing_first_step_matches_oracle(R, oracle, seed):
    """The first step of the two seeds that stop: the GPU's failure counters,
    first failing cell and state (failing cells keep their explicit state)
    equal the oracle's bit for bit."""
    P = I.riemann_1d(seed, 400)
    n, bit, fail = run_compare(R, oracle, P, max_steps=1)
    assert n == 0 and fail is not None and bit
    rep_g, rep_o = fail
    assert rep_o.imp_fail > 0 and rep_o.first_bad_cell in (199, 200)


@pytest.mark.parametrize("solver", [0, 2])
def test_literal_beta_2d_blast(R, oracle, solver):
    """beta on all twelve rows (eq. beta as printed) on the 64x40 magnetised
    blast with overpressure 10 (p_in = 0.1; the overpressure-1e3 blast fails
    at step 1 in this form), PVM-int-8 and its exact-JVP form: 12 steps,
    bitwise every step."""
    oracle.threads(0)
    P = I.blast_2d(0, 64, 40, p_in=0.1)
    n, bit, fail = run_compare(R, oracle, P, max_steps=12, beta_mode=0, solver=solver)
    assert fail is None, fail
    assert n == 12 and bit


def test_literal_beta_2d_blast_advance_256(R, oracle):
    """beta on all rows, 256^2 blast with overpressure 3 (p_in = 0.03), three
    steps with the time step formed on the device (rrmhd_advance) against the
    oracle's loop."""
    import torch
    oracle.threads(0)
    P = I.blast_2d(0, 256, p_in=0.03)
    p = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad, beta_mode=0)
    op = oracle_params(oracle, p)
    g = R.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    og = oracle.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    s = R.Solver(g, p)
    opac = R.make_opacities(dev(torch, P.kappa), dev(torch, P.sigma))
    U = oracle.p2c(P.V, op)
    Ud = dev(torch, U)
    dts = torch.zeros(3, dtype=torch.float64, device="cuda:0")
    s.advance(Ud, P.cfl, 3, opac, dts)
    rep = s.report()
    Ug, dtg = Ud.cpu().numpy(), dts.cpu().numpy()
    s.close()
    Uo = U
    for k in range(3):
        sm, _ = oracle.max_speed(og, Uo, op)
        h = P.cfl * min(P.dx) / sm
        assert dtg[k] == h
        Uo, st, rep_o = oracle.step(og, Uo, h, P.kappa, P.sigma, op)
        assert st == 0
    assert rep["c2p_fail"] == 0 and rep["imp_fail"] == 0
    assert np.array_equal(Ug, Uo), relerr(Ug, Uo)
