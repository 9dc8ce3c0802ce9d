"""The C ABI without a GPU: the library loads, exports every entry point that
``include/rrmhd.h`` declares, the Python binding mirrors the header's structs
byte for byte, and the host-only entry points (defaults, workspace sizing,
argument validation, error strings) behave as documented. No call here
launches a kernel."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rrmhd.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", " ", src, flags=re.S)
    return set(re.findall(r"^\s*[A-Za-z_][\w\s\*]*?\b(rrmhd_\w+)\s*\(", src, flags=re.M))


@pytest.fixture(scope="module")
def R():
    from paper_2212_00370_amd import rrmhd
    return rrmhd


def test_every_declared_symbol_is_exported(R):
    names = _declared_functions()
    assert len(names) >= 15, names
    lib = C.CDLL(R.LIB_PATH)
    missing = [n for n in sorted(names) if not hasattr(lib, n)]
    assert not missing, missing
    # the binding covers exactly the declared entry points
    assert set(R.SIGNATURES) == names


def _c_layout(structs):
    """sizeof / offsetof of header structs, from a C program compiled with gcc."""
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "rrmhd.h"', "int main(void) {"]
    for sname, fields in structs.items():
        lines.append(f'  printf("{sname} size %zu\\n", sizeof({sname}));')
        for f in fields:
            lines.append(f'  printf("{sname} {f} %zu\\n", offsetof({sname}, {f}));')
    lines += ["  return 0;", "}"]
    wd = os.path.join(ROOT, "tests", "__pycache__")
    os.makedirs(wd, exist_ok=True)
    src = os.path.join(wd, "abi_layout.c")
    exe = os.path.join(wd, "abi_layout")
    with open(src, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-I", os.path.join(ROOT, "include"), src, "-o", exe], check=True)
    out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    res = {}
    for ln in out.splitlines():
        s, f, v = ln.split()
        res[(s, f)] = int(v)
    return res


def test_struct_layouts_match_header(R):
    structs = {"rrmhd_grid": R.rrmhd_grid, "rrmhd_params": R.rrmhd_params,
               "rrmhd_opacities": R.rrmhd_opacities, "rrmhd_report": R.rrmhd_report}
    lay = _c_layout({k: [f for f, _ in v._fields_] for k, v in structs.items()})
    for sname, cls in structs.items():
        assert lay[(sname, "size")] == C.sizeof(cls), sname
        for f, _ in cls._fields_:
            assert lay[(sname, f)] == getattr(cls, f).offset, (sname, f)


def test_default_params(R):
    p = R.rrmhd_params()
    R._lib.rrmhd_default_params(C.byref(p))
    assert p.pvm_eps == 1e-8 and p.pvm_k == 3          # PVM-int-8 with eps = 1e-8
    assert p.recon == R.RECON_MINMOD and p.rk_order == 2
    assert p.precision == R.FP64 and p.beta_mode == R.BETA_RAD_ONLY
    assert p.pvm_eps_mixed == 2.0 ** -12 and p.e_floor == 0.0
    assert p.gamma == 5.0 / 3.0
    assert p.solver == R.SOLVER_PVM


def _grid(R, n):
    return R.make_grid(tuple(n), tuple(1.0 / k for k in n), [R.BC_OUTFLOW] * 3, [R.BC_OUTFLOW] * 3)


def test_workspace_bytes(R):
    p = R.rrmhd_params()
    R._lib.rrmhd_default_params(C.byref(p))
    sizes = []
    for n in (16, 64, 256):
        g = _grid(R, (n, n))
        b = R._lib.rrmhd_workspace_bytes(C.byref(g), C.byref(p))
        N = n * n
        nf = 2 * (n + 1) * n
        # at least the stage state and primitives (12 planes each) and the face fluxes
        assert b >= 8 * (12 * N + 12 * N + 12 * nf), (n, b)
        assert b % 256 == 0
        sizes.append(b)
    assert sizes[0] < sizes[1] < sizes[2]
    bad = _grid(R, (16, 16))
    bad.dx[0] = 0.0
    assert R._lib.rrmhd_workspace_bytes(C.byref(bad), C.byref(p)) == 0
    # 2^31 cells: beyond the kernels' 32-bit index range
    big = _grid(R, (1 << 16, 1 << 15))
    assert R._lib.rrmhd_workspace_bytes(C.byref(big), C.byref(p)) == 0
    ok = _grid(R, (1 << 16, (1 << 15) - 1))
    assert R._lib.rrmhd_workspace_bytes(C.byref(ok), C.byref(p)) > 0
    bad = _grid(R, (16, 16))
    bad.bc_hi[0] = R.BC_INFLOW
    assert R._lib.rrmhd_workspace_bytes(C.byref(bad), C.byref(p)) == 0
    q = R.rrmhd_params()
    R._lib.rrmhd_default_params(C.byref(q))
    q.gamma = 0.5
    assert R._lib.rrmhd_workspace_bytes(C.byref(_grid(R, (16, 16))), C.byref(q)) == 0
    # every solver in both precisions; unknown solvers are refused
    R._lib.rrmhd_default_params(C.byref(q))
    q.solver = R.SOLVER_HLL
    assert R._lib.rrmhd_workspace_bytes(C.byref(_grid(R, (16, 16))), C.byref(q)) > 0
    q.precision = R.MIXED
    assert R._lib.rrmhd_workspace_bytes(C.byref(_grid(R, (16, 16))), C.byref(q)) > 0
    q.solver = R.SOLVER_PVM_JVP
    assert R._lib.rrmhd_workspace_bytes(C.byref(_grid(R, (16, 16))), C.byref(q)) > 0
    q.precision = R.FP64
    assert R._lib.rrmhd_workspace_bytes(C.byref(_grid(R, (16, 16))), C.byref(q)) > 0
    q.solver = 3
    assert R._lib.rrmhd_workspace_bytes(C.byref(_grid(R, (16, 16))), C.byref(q)) == 0
    assert R._lib.rrmhd_batch_workspace_bytes(0) == 0
    assert R._lib.rrmhd_batch_workspace_bytes(8) > 0


def test_argument_errors_need_no_device(R):
    p = R.rrmhd_params()
    R._lib.rrmhd_default_params(C.byref(p))
    g = _grid(R, (8, 8))
    ctx = C.c_void_p()
    # validation happens before any HIP call
    assert R._lib.rrmhd_init(None, C.byref(g), C.byref(p), None, 0, None) == R.RRMHD_E_INVALID
    assert R._lib.rrmhd_init(C.byref(ctx), C.byref(g), C.byref(p), None, 0, None) == R.RRMHD_E_WORKSPACE
    g2 = _grid(R, (8, 8))
    g2.ndim = 4
    assert R._lib.rrmhd_init(C.byref(ctx), C.byref(g2), C.byref(p), None, 0, None) == R.RRMHD_E_INVALID
    op = R.rrmhd_opacities()
    assert R._lib.rrmhd_step(None, None, C.byref(g), 1e-3, C.byref(op)) == R.RRMHD_E_INVALID
    assert R._lib.rrmhd_advance(None, None, C.byref(g), 0.4, 1, C.byref(op), None) == R.RRMHD_E_INVALID
    out = C.c_double()
    assert R._lib.rrmhd_max_speed(None, None, C.byref(g), C.byref(out)) == R.RRMHD_E_INVALID
    # the allocation-free advance validates before touching a device: a null
    # state, a bad cfl or step count, and a grid whose workspace exceeds the
    # 64 MiB scratch array are refused (the state pointer is never read)
    fake = C.c_void_p(0x1000)
    na = R._lib.rrmhd_advance_noalloc
    assert na(C.byref(g), C.byref(p), None, 0.4, 1, C.byref(op), None, None, None) == R.RRMHD_E_INVALID
    assert na(C.byref(g), C.byref(p), fake, 0.0, 1, C.byref(op), None, None, None) == R.RRMHD_E_INVALID
    assert na(C.byref(g), C.byref(p), fake, 0.4, -1, C.byref(op), None, None, None) == R.RRMHD_E_INVALID
    assert na(C.byref(g2), C.byref(p), fake, 0.4, 1, C.byref(op), None, None, None) == R.RRMHD_E_INVALID
    big = _grid(R, (512, 512))
    assert R._lib.rrmhd_workspace_bytes(C.byref(big), C.byref(p)) > (64 << 20)
    assert na(C.byref(big), C.byref(p), fake, 0.4, 1, C.byref(op), None, None, None) == R.RRMHD_E_WORKSPACE
    fits = _grid(R, (360, 360))
    assert R._lib.rrmhd_workspace_bytes(C.byref(fits), C.byref(p)) <= (64 << 20)


def test_error_strings(R):
    for st in (R.RRMHD_OK, R.RRMHD_E_INVALID, R.RRMHD_E_C2P, R.RRMHD_E_IMPLICIT, R.RRMHD_E_NONFINITE,
               R.RRMHD_E_DEVICE, R.RRMHD_E_WORKSPACE):
        s = R._lib.rrmhd_strerror(st)
        assert s and len(s.decode()) >= 2
    assert R._lib.rrmhd_strerror(-99)


def test_header_enums_match_binding(R):
    """Every enumerator of include/rrmhd.h has the same value in the binding
    (RRMHD_X -> X or RRMHD_X in paper_2212_00370_amd/rrmhd.py)."""
    import re
    hdr = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "rrmhd.h")).read()
    seen = 0
    for body in re.findall(r"enum\s*(?:\w+\s*)?\{([^}]*)\}", hdr):
        body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
        for name, val in re.findall(r"(RRMHD_\w+)\s*=\s*(-?\d+)", body):
            short = name[len("RRMHD_"):]
            py = getattr(R, short, getattr(R, name, None))
            assert py is not None, name
            assert py == int(val), (name, py, val)
            seen += 1
    assert seen >= 20


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus N with N > 1 exits with a message
    (before touching a device)."""
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
