"""CPU-side checks of librs: it loads, exports every symbol declared in
include/rs.h, and its host-only logic (parameter formulas, argument checks that
fail before any device work) behaves.  No kernel is launched here."""
import ctypes
import os
import re

import pytest

from oracle import ihs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rs.h")
LIB = os.path.join(ROOT, "paper_2006_05874_amd", "librs.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rs_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2006_05874_amd import build
        build.build(verbose=False)
    from paper_2006_05874_amd import rs
    return rs.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for want in ["rs_sketch_srht", "rs_sketch_gaussian", "rs_factor_woodbury", "rs_ihs_step",
                 "rs_adaptive_solve", "rs_factor_apply", "rs_gradient", "rs_params"]:
        assert want in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_declares_every_export():
    from paper_2006_05874_amd import rs
    assert set(declared_functions()) <= set(rs.EXPORTS)


def test_version_string(lib):
    assert b"gfx950" in lib.rs_version()


@pytest.mark.parametrize("kind,rho,eta", [("srht", 0.1, 0.01), ("srht", 0.37, 0.01),
                                          ("gaussian", 0.1, 0.01), ("gaussian", 0.18, 0.004),
                                          ("count", 0.1, 0.01)])
def test_params_match_oracle(lib, kind, rho, eta):
    from paper_2006_05874_amd import rs
    got = rs.rs_params(kind, rho, eta)
    want = ihs.params_for(kind, rho, eta)
    for k in ["mu_gd", "mu_p", "beta_p", "cbar_gd", "cbar_p"]:
        assert abs(got[k] - getattr(want, k)) < 1e-15 * max(1.0, abs(getattr(want, k)))


@pytest.mark.parametrize("kind,rho,eta", [("srht", 0.0, 0.01), ("srht", 1.0, 0.01),
                                          ("gaussian", 0.5, 0.01), ("gaussian", 0.1, 0.05)])
def test_params_reject_outside_domain(lib, kind, rho, eta):
    from paper_2006_05874_amd import rs
    with pytest.raises(rs.RsError) as e:
        rs.rs_params(kind, rho, eta)
    assert e.value.name == "arg"


def test_null_and_shape_errors_before_any_device_work(lib):
    vp = ctypes.c_void_p
    st = lib.rs_sketch_srht(vp(0), 1, 100, 10, 12, 4, 0, 0, vp(16), 1, 10, vp(0), vp(0), vp(0),
                            vp(0))
    assert st == 1 and b"null" in lib.rs_last_error()
    # lda not a multiple of 16 bytes
    st = lib.rs_gradient(vp(256), 1, 100, 10, 10, vp(256), 1.0, vp(256), 1, vp(256), vp(0))
    assert st == 1 and b"lda" in lib.rs_last_error()
    # misaligned A
    st = lib.rs_gradient(vp(260), 1, 100, 10, 12, vp(256), 1.0, vp(256), 1, vp(256), vp(0))
    assert st == 1 and b"aligned" in lib.rs_last_error()
    # k out of range
    st = lib.rs_gradient(vp(256), 1, 100, 10, 12, vp(256), 1.0, vp(256), 5, vp(256), vp(0))
    assert st == 1
    # m above the padded row count
    st = lib.rs_sketch_srht(vp(256), 1, 100, 10, 12, 129, 0, 0, vp(256), 1, 10, vp(0), vp(0),
                            vp(0), vp(0))
    assert st == 2
    # F64 A with F32 SA is not offered
    st = lib.rs_sketch_srht(vp(256), 0, 100, 10, 10, 4, 0, 0, vp(256), 1, 10, vp(0), vp(0),
                            vp(0), vp(0))
    assert st == 9


def test_solver_argument_errors(lib):
    from paper_2006_05874_amd import rs
    vp = ctypes.c_void_p
    o = rs.SolveOpts()
    lib.rs_solve_opts_default(ctypes.byref(o))
    assert o.rho == 0.1 and o.m_init == 1 and o.tol == 1e-7 and o.check_every == 4
    info = rs.SolveInfo()
    # n < d
    st = lib.rs_adaptive_solve(vp(256), 1, 8, 16, 16, vp(256), 0.1, ctypes.byref(o), vp(256),
                               ctypes.byref(info), vp(0))
    assert st == 2
    # nu^2 <= 0 is not positive definite
    st = lib.rs_adaptive_solve(vp(256), 1, 64, 16, 16, vp(256), 0.0, ctypes.byref(o), vp(256),
                               ctypes.byref(info), vp(0))
    assert st == 4
    # Gaussian rho outside Definition 3.1's domain
    o.kind, o.rho = 1, 0.5
    st = lib.rs_adaptive_solve(vp(256), 1, 64, 16, 16, vp(256), 0.1, ctypes.byref(o), vp(256),
                               ctypes.byref(info), vp(0))
    assert st == 1


def test_batch_and_grid_argument_errors_before_device_work(lib):
    from paper_2006_05874_amd import rs
    vp = ctypes.c_void_p
    opts = rs.SolveOpts()
    lib.rs_solve_opts_default(ctypes.byref(opts))
    infos = (rs.SolveInfo * 2)()
    # empty batch: nothing to do
    assert lib.rs_solve_batch((rs.Problem * 1)(), 0, ctypes.byref(opts), infos, 2, vp(0)) == 0
    # a problem with nu^2 <= 0 is rejected before any job starts
    P = (rs.Problem * 1)()
    P[0] = rs.Problem(vp(256), 1, 0, 100, 10, 12, vp(256), -1.0, vp(256))
    assert lib.rs_solve_batch(P, 1, ctypes.byref(opts), infos, 2, vp(0)) == 4
    # the learned batch needs a model
    assert lib.rs_learned_solve_batch(P, 1, ctypes.byref(opts), vp(0), vp(0), vp(0), infos,
                                      None, 2, vp(0)) == 1
    # nu grid: count, nu^2 and null checks
    nu = (ctypes.c_double * 2)(1e-2, 0.0)
    assert lib.rs_solve_nu_grid(vp(256), 1, 100, 10, 12, vp(256), nu, 0, ctypes.byref(opts),
                                vp(256), infos, vp(0)) == 1
    assert lib.rs_solve_nu_grid(vp(256), 1, 100, 10, 12, vp(256), nu, 2, ctypes.byref(opts),
                                vp(256), infos, vp(0)) == 4
    assert lib.rs_solve_nu_grid(vp(256), 1, 100, 10, 12, vp(256), None, 2, ctypes.byref(opts),
                                vp(256), infos, vp(0)) == 1
    # autotuner: k out of range, misaligned lda
    assert lib.rs_gradient_autotune(vp(256), 1, 100, 10, 12, vp(256), 5, None, vp(0)) == 1
    assert lib.rs_gradient_autotune(vp(256), 1, 100, 10, 10, vp(256), 2, None, vp(0)) == 1
    # plan query: bad shapes
    plan = (ctypes.c_int32 * 4)()
    assert lib.rs_gradient_plan(1, 100, 10, 0, ctypes.cast(plan, vp)) == 2
    assert lib.rs_gradient_plan(2, 100, 10, 1, ctypes.cast(plan, vp)) == 1


def test_next_forms_argument_errors_before_device_work(lib):
    from paper_2006_05874_amd import rs
    vp = ctypes.c_void_p
    o = rs.SolveOpts()
    lib.rs_solve_opts_default(ctypes.byref(o))
    infos = (rs.SolveInfo * 3)()
    info = rs.SolveInfo()
    # path: nu^2 increasing (arg), not positive (not_spd), empty (nothing to do)
    nu = (ctypes.c_double * 3)(1e-2, 1e-1, 1e-3)
    assert lib.rs_solve_path(vp(256), 1, 100, 10, 12, vp(256), nu, 3, ctypes.byref(o), vp(256),
                             infos, vp(0)) == 1
    nu = (ctypes.c_double * 3)(1e-2, -1.0, 1e-3)
    assert lib.rs_solve_path(vp(256), 1, 100, 10, 12, vp(256), nu, 3, ctypes.byref(o), vp(256),
                             infos, vp(0)) == 4
    assert lib.rs_solve_path(vp(256), 1, 100, 10, 12, vp(256), nu, 0, ctypes.byref(o), vp(256),
                             infos, vp(0)) == 0
    # dual: a tall matrix (shape), a null output (arg)
    assert lib.rs_adaptive_solve_dual(vp(256), 1, 100, 10, 12, vp(256), 0.1, ctypes.byref(o),
                                      vp(256), vp(256), ctypes.byref(info), vp(0)) == 2
    assert lib.rs_adaptive_solve_dual(vp(256), 1, 10, 100, 100, vp(256), 0.1, ctypes.byref(o),
                                      vp(256), None, ctypes.byref(info), vp(0)) == 1
    # CSR: the CountSketch is required (unsupported otherwise), d above 8192 (shape),
    # n < d (shape), null rowptr (arg), an FP8 CountSketch (unsupported)
    assert lib.rs_adaptive_solve_csr(vp(256), vp(256), vp(256), 1, 100, 10, 50, vp(256), 0.1,
                                     ctypes.byref(o), vp(256), ctypes.byref(info), vp(0)) == 9
    o.kind = 2
    assert lib.rs_adaptive_solve_csr(vp(256), vp(256), vp(256), 1, 100000, 9000, 50, vp(256), 0.1,
                                     ctypes.byref(o), vp(256), ctypes.byref(info), vp(0)) == 2
    assert lib.rs_adaptive_solve_csr(vp(256), vp(256), vp(256), 1, 10, 100, 50, vp(256), 0.1,
                                     ctypes.byref(o), vp(256), ctypes.byref(info), vp(0)) == 2
    assert lib.rs_adaptive_solve_csr(None, vp(256), vp(256), 1, 100, 10, 50, vp(256), 0.1,
                                     ctypes.byref(o), vp(256), ctypes.byref(info), vp(0)) == 1
    o.sketch_dtype = 3
    assert lib.rs_adaptive_solve_csr(vp(256), vp(256), vp(256), 1, 100, 10, 50, vp(256), 0.1,
                                     ctypes.byref(o), vp(256), ctypes.byref(info), vp(0)) == 9
    # the dense solvers refuse the CountSketch
    o.sketch_dtype = 1
    assert lib.rs_adaptive_solve(vp(256), 1, 64, 16, 16, vp(256), 0.1, ctypes.byref(o), vp(256),
                                 ctypes.byref(info), vp(0)) == 9
    # refreshed: nu^2 not positive, n < d
    lib.rs_solve_opts_default(ctypes.byref(o))
    rh = (ctypes.c_double * 8)()
    assert lib.rs_refreshed_ihs(vp(256), 1, 64, 16, 16, vp(256), 0.0, ctypes.byref(o), vp(256), rh,
                                ctypes.byref(info), vp(0)) == 4
    assert lib.rs_refreshed_ihs(vp(256), 1, 8, 16, 16, vp(256), 0.1, ctypes.byref(o), vp(256), rh,
                                ctypes.byref(info), vp(0)) == 2
    # rs_params: the CountSketch takes the SRHT's parameters
    assert rs.rs_params("count", 0.25, 0.01) == rs.rs_params("srht", 0.25, 0.01)


def test_binding_rejects_host_and_short_buffers():
    # the library reads n values of b, d of a start vector and nnz of val through raw
    # pointers: the binding refuses host tensors and buffers of the wrong size before
    # any call (a host pointer or a short buffer would be read out of bounds)
    import torch
    from paper_2006_05874_amd import rs
    A = torch.zeros(100, 12)
    with pytest.raises(ValueError, match="device tensor"):
        rs.rs_adaptive_solve(A, torch.zeros(100), 0.1)
    with pytest.raises(ValueError, match="b holds 99 values"):
        rs._rhs(torch.zeros(99), A, "w")
    with pytest.raises(ValueError, match="b must be a device tensor"):
        rs._rhs(torch.zeros(100), A, "w")
    z = rs._start(None, 12, "cpu", "w")
    assert z.dtype == torch.float64 and z.shape == (12,) and not z.any()
    with pytest.raises(ValueError, match="x0 holds 11 values, expected 12"):
        rs._start(torch.zeros(11), 12, "cpu", "w")
    with pytest.raises(ValueError, match="z0 must be a device tensor"):
        rs._start(torch.zeros(12), 12, "cpu", "w", "z0")
    rowptr = torch.tensor([0, 2, 3], dtype=torch.int64)
    col = torch.tensor([0, 4, 1], dtype=torch.int32)
    with pytest.raises(ValueError, match="one value per column index"):
        rs.rs_adaptive_solve_csr(rowptr, col, torch.zeros(2), 5, torch.zeros(2), 0.1)
    with pytest.raises(ValueError, match="n values of b"):
        rs.rs_adaptive_solve_csr(rowptr, col, torch.zeros(3), 5, torch.zeros(1), 0.1)
    with pytest.raises(ValueError, match="rowptr must be a device tensor"):
        rs.rs_adaptive_solve_csr(rowptr, col, torch.zeros(3), 5, torch.zeros(2), 0.1)


def test_missing_library_fails_loudly():
    # with no built library every entry point raises: there is no fallback path
    import subprocess
    import sys
    code = ("from paper_2006_05874_amd import rs\n"
            "rs.load.__defaults__ = ('/nonexistent/librs.so',)\n"
            "try:\n"
            "    rs.rs_params('srht', 0.1)\n"
            "except ImportError as e:\n"
            "    print('raised:', e)\n"
            "    raise SystemExit(3)\n")
    r = subprocess.run([sys.executable, "-c", code], cwd=ROOT, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode == 3, r.stdout + r.stderr
    assert "librs.so not built" in r.stdout


# ------------------------------------------------ Algorithm 1's tests as the kernels run them
def test_step_rule_accepts_as_algorithm1(lib):
    """The decision kernels' rule (host copy of the same source) against the tests
    of Algorithm 1 written out here: Polyak first, then the gradient candidate,
    ties accept, doubling otherwise, and the m_max reading."""
    from paper_2006_05874_amd import rs
    prm = ihs.params_for("srht", 0.1)
    cp, cg = prm.cbar_p, prm.cbar_gd
    r1, rt = 1.0, 0.5
    # (r_p / r_1)^(1/t) <= cbar_p at t = 2: r_p = cbar_p^2 r_1 ties, accepted
    assert rs.rs_step_rule(1, cp ** 2 * r1, 0.4, rt, r1, 2, 0, cp, cg) == "accept_polyak"
    # just above: the Polyak candidate fails, the gradient one passes
    assert rs.rs_step_rule(1, 1.01 * cp ** 2, cg * rt, rt, r1, 2, 0, cp, cg) == "accept_gd"
    # an off-by-one exponent would accept this one: (cp^1.5)^(1/2) > cp, but ^(1/3) < cp
    assert rs.rs_step_rule(1, cp ** 1.5, 0.9 * rt, rt, r1, 2, 0, cp, cg) == "double"
    assert rs.rs_step_rule(0, 0.0, 1.01 * cg * rt, rt, r1, 3, 0, cp, cg) == "double"
    # at m_max: any decrease is taken, else stuck
    assert rs.rs_step_rule(0, 0.0, 0.9 * rt, rt, r1, 3, 1, cp, cg) == "accept_gd"
    assert rs.rs_step_rule(0, 0.0, 1.1 * rt, rt, r1, 3, 1, cp, cg) == "stuck"
    assert rs.rs_step_rule(1, float("nan"), 0.1, rt, r1, 3, 0, cp, cg) == "nonfinite"


@pytest.mark.parametrize("polyak,r_p,r_gd", [(1, -1e-12, 1e-3), (1, 1e-3, -1e-12),
                                             (0, 0.0, -1e-12), (1, -5.0, -5.0)])
def test_step_rule_refuses_negative_decrements(lib, polyak, r_p, r_gd):
    """A negative decrement (an indefinite H_S^-1) passes no test: it asks for a
    larger sketch, and at m_max ends the run, instead of passing r/r_t <= cbar."""
    from paper_2006_05874_amd import rs
    prm = ihs.params_for("srht", 0.1)
    assert rs.rs_step_rule(polyak, r_p, r_gd, 0.5, 1.0, 2, 0, prm.cbar_p, prm.cbar_gd) == "double"
    assert rs.rs_step_rule(polyak, r_p, r_gd, 0.5, 1.0, 2, 1, prm.cbar_p,
                           prm.cbar_gd) == "indefinite"


def test_start_rule(lib):
    from paper_2006_05874_amd import rs
    assert rs.rs_start_rule(1.0, 2.0, 1e-7, 0) == "running"
    assert rs.rs_start_rule(1e-8, 1.0, 1e-7, 0) == "converged"
    assert rs.rs_start_rule(0.0, 0.0, 1e-7, 0) == "converged"
    assert rs.rs_start_rule(-1e-9, 1.0, 1e-7, 0) == "double"
    assert rs.rs_start_rule(1.0, -1.0, 1e-7, 0) == "double"
    assert rs.rs_start_rule(-1e-9, 1.0, 1e-7, 1) == "indefinite"
    assert rs.rs_start_rule(float("inf"), 1.0, 1e-7, 0) == "nonfinite"
