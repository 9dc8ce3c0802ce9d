"""GPU: the allocation-free advance (rrmhd_advance_noalloc, the library's
per-device scratch array as workspace) against rrmhd_advance with a caller
workspace, through the C ABI. Both run the same kernels, so the states, the
time steps and the failure counters must agree bit for bit; two calls in a
row, the second on a smaller grid, show that nothing of the first call's
scratch contents leaks into the second."""
import numpy as np
import pytest

from paper_2212_00370_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2212_00370_amd import rrmhd
    return rrmhd


def run_pair(R, P, nsteps, **kw):
    import torch
    p = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad, **kw)
    g = R.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")
    opac = R.make_opacities(dev(P.kappa), dev(P.sigma))
    s = R.Solver(g, p)
    U0 = s.prim_to_cons(dev(P.V))
    if kw.get("ct"):
        # constrained transport: the face-field planes follow the cell planes
        bface = P.extra["bface"] if "bface" in P.extra else I.uniform_face_fields(P)
        U0 = torch.cat([U0, dev(bface)]).contiguous()
    torch.cuda.synchronize()
    Ua = U0.clone()
    dta = torch.zeros(nsteps, dtype=torch.float64, device="cuda:0")
    s.advance(Ua, P.cfl, nsteps, opac, dta)
    rep_a = s.report()
    s.close()
    Ub = U0.clone()
    dtb = torch.zeros(nsteps, dtype=torch.float64, device="cuda:0")
    rep_dev = torch.zeros(64, dtype=torch.uint8, device="cuda:0")
    R.rrmhd_advance_noalloc(g, p, Ub, P.cfl, nsteps, opac, dtb, rep_dev)
    torch.cuda.synchronize()
    rep_b = R.report_from_bytes(bytes(rep_dev.cpu().numpy().tobytes()))
    return Ua.cpu().numpy(), Ub.cpu().numpy(), dta.cpu().numpy(), dtb.cpu().numpy(), rep_a, rep_b


def check(out):
    Ua, Ub, dta, dtb, rep_a, rep_b = out
    assert np.all(dta > 0)
    assert np.array_equal(dta, dtb)
    assert np.array_equal(Ua, Ub)
    assert rep_a == rep_b, (rep_a, rep_b)


def test_noalloc_equals_advance_two_calls_shrinking(R):
    """96x80 blast (3 steps), then a 48x40 blast (2 steps) reusing the scratch
    array the first call left behind."""
    for nx, ny, steps in ((96, 80, 3), (48, 40, 2)):
        print(f"noalloc vs advance: blast {nx}x{ny}, {steps} steps", flush=True)
        P = I.blast_2d(0, nx, ny)
        check(run_pair(R, P, steps))


def test_noalloc_equals_advance_1d_then_smaller_1d(R):
    """1D Riemann problem, 400 cells then 256 cells, mixed precision second."""
    P = I.riemann_1d(3, 400)
    print("noalloc vs advance: riemann seed 3, 400 cells", flush=True)
    check(run_pair(R, P, 4))
    P = I.riemann_1d(5, 256)
    print("noalloc vs advance: riemann seed 5, 256 cells, mixed", flush=True)
    check(run_pair(R, P, 3, precision=R.MIXED))


def test_noalloc_equals_advance_with_ct(R):
    """Constrained transport (one face-field plane per dimension after the 12
    cell planes): the 64x40 blast for 3 steps, then the smaller 48x24 field
    loop for 2 steps."""
    P = I.blast_2d(0, 64, 40)
    print("noalloc vs advance: CT blast 64x40, 3 steps", flush=True)
    check(run_pair(R, P, 3, ct=1))
    P = I.field_loop_2d(48)
    print("noalloc vs advance: CT field loop 48x24, 2 steps", flush=True)
    check(run_pair(R, P, 2, ct=1))


def test_noalloc_rejects_a_grid_beyond_the_scratch_array(R):
    import torch
    P = I.blast_2d(0, 512)
    p = R.rrmhd_default_params(gamma=P.gamma, a_rad=P.a_rad)
    g = R.make_grid(P.shape, P.dx, P.bc_lo, P.bc_hi)
    U = torch.zeros((12, 512 * 512), dtype=torch.float64, device="cuda:0")
    with pytest.raises(R.RRMHDError, match="workspace"):
        R.rrmhd_advance_noalloc(g, p, U, P.cfl, 1, R.make_opacities())
