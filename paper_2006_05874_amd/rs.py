"""ctypes binding of librs (include/rs.h): argument marshalling only.

Every computation runs in the HIP library.  torch provides device memory and
the current HIP stream.  The binding checks what the C ABI cannot see: that each
buffer passed is device memory holding as many values as the call reads.  Loading fails loudly when librs.so is missing: there
is no CPU fallback.
"""
import ctypes
import math
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librs.so")

RS_OK, RS_ERR_ARG, RS_ERR_SHAPE, RS_ERR_NOT_POW2, RS_ERR_NOT_SPD = 0, 1, 2, 3, 4
RS_ERR_NONFINITE, RS_ERR_NO_CONVERGENCE, RS_ERR_OOM, RS_ERR_HIP, RS_ERR_UNSUPPORTED = 5, 6, 7, 8, 9
STATUS_NAMES = {0: "ok", 1: "arg", 2: "shape", 3: "not_pow2", 4: "not_spd", 5: "nonfinite",
                6: "no_convergence", 7: "oom", 8: "hip", 9: "unsupported"}

DTYPES = {"f64": 0, "f32": 1, "bf16": 2, "fp8": 3}
TORCH_DTYPES = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16,
                "fp8": torch.uint8}
SKETCH = {"srht": 0, "gaussian": 1, "count": 2}
RESAMPLE = {"fresh": 0, "nested": 1}
VARIANT = {"polyak": 0, "gd": 1}
EVENT_NAMES = {0: "polyak", 1: "gd", 2: "double"}
RS_MAX_EVENTS = 512


class RsError(RuntimeError):
    def __init__(self, status, where, msg):
        self.status = status
        self.name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{where}: {self.name}: {msg}")


class IhsParams(ctypes.Structure):
    _fields_ = [("mu_gd", ctypes.c_double), ("mu_p", ctypes.c_double),
                ("beta_p", ctypes.c_double), ("cbar_gd", ctypes.c_double),
                ("cbar_p", ctypes.c_double)]


class IhsState(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("x_prev", ctypes.c_void_p), ("g", ctypes.c_void_p),
                ("gtilde", ctypes.c_void_p), ("r_t", ctypes.c_double), ("r_1", ctypes.c_double),
                ("t", ctypes.c_int64)]


class StepResult(ctypes.Structure):
    _fields_ = [("accepted", ctypes.c_int32), ("r_p", ctypes.c_double), ("r_gd", ctypes.c_double)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("variant", ctypes.c_int), ("resample", ctypes.c_int),
                ("sketch_dtype", ctypes.c_int), ("rho", ctypes.c_double), ("eta", ctypes.c_double),
                ("m_init", ctypes.c_int64), ("m_max", ctypes.c_int64), ("tol", ctypes.c_double),
                ("max_iter", ctypes.c_int64), ("seed", ctypes.c_uint64),
                ("check_every", ctypes.c_int32), ("flags", ctypes.c_int32)]


RS_SOLVE_GRAPH_STEPS = 1
RS_SOLVE_REF_AT_ZERO = 2


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("reserved", ctypes.c_int32),
                ("m_final", ctypes.c_int64), ("doublings", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("grad_passes", ctypes.c_int64),
                ("applies", ctypes.c_int64), ("accepted_polyak", ctypes.c_int64),
                ("accepted_gd", ctypes.c_int64), ("r_final", ctypes.c_double),
                ("r_ref", ctypes.c_double), ("n_events", ctypes.c_int64),
                ("event_kind", ctypes.c_int32 * RS_MAX_EVENTS),
                ("event_t", ctypes.c_int32 * RS_MAX_EVENTS),
                ("event_m", ctypes.c_int64 * RS_MAX_EVENTS),
                ("ms_sketch", ctypes.c_double), ("ms_factor", ctypes.c_double),
                ("ms_iterate", ctypes.c_double)]


EXPORTS = ["rs_params", "rs_sketch_srht", "rs_sketch_gaussian", "rs_factor_woodbury",
           "rs_factor_apply", "rs_factor_destroy", "rs_gradient", "rs_ihs_step",
           "rs_solve_opts_default", "rs_adaptive_solve", "rs_last_error", "rs_version",
           "rs_profile_enable", "rs_profile_read", "rs_features", "rs_mlp_forward",
           "rs_mlp_backward", "rs_mlp_adam_step", "rs_learned_solve", "rs_solve_batch",
           "rs_solve_nu_grid", "rs_learned_solve_batch", "rs_gradient_autotune",
           "rs_gradient_plan", "rs_solve_path", "rs_adaptive_solve_dual", "rs_refreshed_ihs",
           "rs_adaptive_solve_csr", "rs_step_rule", "rs_start_rule", "rs_gradient_set_plan",
           "rs_gradient_noalloc", "rs_gradient_two"]
MLP_PARAMS = 18817
MLP_CACHE = 273
MLP_WORK = 257

_lib = None


class Problem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("a_t", ctypes.c_int), ("reserved", ctypes.c_int32),
                ("n", ctypes.c_int64), ("d", ctypes.c_int64), ("lda", ctypes.c_int64),
                ("b", ctypes.c_void_p), ("nu2", ctypes.c_double), ("x", ctypes.c_void_p)]


def load(path=LIB_PATH):
    """Load librs.so and declare its signatures (no GPU needed)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"librs.so not built at {path}; run paper_2006_05874_amd.build.build()")
    L = ctypes.CDLL(path)
    vp, i64, u64, u32, dbl = (ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_uint32,
                              ctypes.c_double)
    c_int = ctypes.c_int
    L.rs_params.argtypes = [c_int, dbl, dbl, ctypes.POINTER(IhsParams)]
    L.rs_sketch_srht.argtypes = [vp, c_int, i64, i64, i64, i64, u64, u32, vp, c_int, i64, vp, vp,
                                 vp, vp]
    L.rs_sketch_gaussian.argtypes = [vp, c_int, i64, i64, i64, i64, u64, u32, vp, c_int, i64, vp,
                                     vp]
    L.rs_factor_woodbury.argtypes = [vp, c_int, vp, i64, i64, i64, dbl, ctypes.POINTER(vp), vp]
    L.rs_factor_apply.argtypes = [vp, vp, vp, vp, i64, vp]
    L.rs_factor_destroy.argtypes = [vp]
    L.rs_factor_destroy.restype = None
    L.rs_gradient.argtypes = [vp, c_int, i64, i64, i64, vp, dbl, vp, i64, vp, vp]
    L.rs_gradient_noalloc.argtypes = [vp, c_int, i64, i64, i64, vp, dbl, vp, i64, vp, vp]
    L.rs_gradient_two.argtypes = [vp, i64, i64, i64, vp, vp, vp, vp, vp, vp, vp]
    L.rs_ihs_step.argtypes = [vp, c_int, i64, i64, i64, vp, dbl, vp, ctypes.POINTER(IhsParams),
                              c_int, ctypes.POINTER(IhsState), ctypes.POINTER(StepResult), vp]
    L.rs_solve_opts_default.argtypes = [ctypes.POINTER(SolveOpts)]
    L.rs_solve_opts_default.restype = None
    L.rs_adaptive_solve.argtypes = [vp, c_int, i64, i64, i64, vp, dbl, ctypes.POINTER(SolveOpts),
                                    vp, ctypes.POINTER(SolveInfo), vp]
    L.rs_profile_enable.argtypes = [c_int]
    L.rs_profile_read.argtypes = [ctypes.POINTER(i64), ctypes.POINTER(dbl)]
    L.rs_features.argtypes = [vp, c_int, i64, i64, i64, dbl, u64, vp, vp]
    L.rs_mlp_forward.argtypes = [vp, vp, i64, vp, vp, vp, vp, vp]
    L.rs_mlp_backward.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp]
    L.rs_mlp_adam_step.argtypes = [vp, vp, vp, vp, i64, i64, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float, ctypes.c_float, vp]
    L.rs_learned_solve.argtypes = [vp, c_int, i64, i64, i64, vp, dbl, ctypes.POINTER(SolveOpts),
                                   vp, vp, vp, vp, ctypes.POINTER(SolveInfo),
                                   ctypes.POINTER(i64), vp]
    L.rs_solve_batch.argtypes = [ctypes.POINTER(Problem), i64, ctypes.POINTER(SolveOpts),
                                 ctypes.POINTER(SolveInfo), ctypes.c_int32, vp]
    L.rs_solve_nu_grid.argtypes = [vp, c_int, i64, i64, i64, vp, ctypes.POINTER(dbl), i64,
                                   ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveInfo), vp]
    L.rs_adaptive_solve_dual.argtypes = [vp, c_int, i64, i64, i64, vp, dbl,
                                         ctypes.POINTER(SolveOpts), vp, vp,
                                         ctypes.POINTER(SolveInfo), vp]
    L.rs_refreshed_ihs.argtypes = [vp, c_int, i64, i64, i64, vp, dbl, ctypes.POINTER(SolveOpts),
                                   vp, ctypes.POINTER(dbl), ctypes.POINTER(SolveInfo), vp]
    L.rs_adaptive_solve_csr.argtypes = [vp, vp, vp, c_int, i64, i64, i64, vp, dbl,
                                        ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveInfo),
                                        vp]
    L.rs_solve_path.argtypes = [vp, c_int, i64, i64, i64, vp, ctypes.POINTER(dbl), i64,
                                ctypes.POINTER(SolveOpts), vp, ctypes.POINTER(SolveInfo), vp]
    L.rs_learned_solve_batch.argtypes = [ctypes.POINTER(Problem), i64, ctypes.POINTER(SolveOpts),
                                         vp, vp, vp, ctypes.POINTER(SolveInfo),
                                         ctypes.POINTER(i64), ctypes.c_int32, vp]
    L.rs_gradient_autotune.argtypes = [vp, c_int, i64, i64, i64, vp, i64, vp, vp]
    L.rs_gradient_plan.argtypes = [c_int, i64, i64, i64, vp]
    L.rs_gradient_set_plan.argtypes = [c_int, i64, i64, i64, vp]
    L.rs_step_rule.argtypes = [ctypes.c_int32, dbl, dbl, dbl, dbl, i64, ctypes.c_int32, dbl, dbl]
    L.rs_step_rule.restype = ctypes.c_int32
    L.rs_start_rule.argtypes = [dbl, dbl, dbl, ctypes.c_int32]
    L.rs_start_rule.restype = ctypes.c_int32
    L.rs_last_error.restype = ctypes.c_char_p
    L.rs_version.restype = ctypes.c_char_p
    for name in ["rs_params", "rs_sketch_srht", "rs_sketch_gaussian", "rs_factor_woodbury",
                 "rs_factor_apply", "rs_gradient", "rs_ihs_step", "rs_adaptive_solve",
                 "rs_profile_enable", "rs_profile_read", "rs_features", "rs_mlp_forward",
                 "rs_mlp_backward", "rs_mlp_adam_step", "rs_learned_solve", "rs_solve_batch",
                 "rs_solve_nu_grid", "rs_learned_solve_batch", "rs_gradient_autotune",
                 "rs_gradient_plan", "rs_solve_path", "rs_adaptive_solve_dual",
                 "rs_refreshed_ihs", "rs_adaptive_solve_csr", "rs_gradient_set_plan",
                 "rs_gradient_noalloc", "rs_gradient_two"]:
        getattr(L, name).restype = c_int
    _lib = L
    return L


RULES = {0: "accept_polyak", 1: "accept_gd", 2: "running", 3: "converged", 4: "double",
         5: "stuck", 6: "nonfinite", 7: "indefinite"}


def rs_step_rule(polyak, r_p, r_gd, r_t, r_1, t, at_cap, cbar_p, cbar_gd):
    """Outcome name of Algorithm 1's tests for one step (the kernels' rule)."""
    return RULES[load().rs_step_rule(int(bool(polyak)), r_p, r_gd, r_t, r_1, t, int(bool(at_cap)),
                                     cbar_p, cbar_gd)]


def rs_start_rule(r, r_ref, tol, at_cap):
    """Outcome name of the state check after a (re)factor (the kernels' rule)."""
    return RULES[load().rs_start_rule(r, r_ref, tol, int(bool(at_cap)))]


def _check(st, where):
    if st != RS_OK:
        raise RsError(st, where, load().rs_last_error().decode())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _mat(A, where):
    if not A.is_cuda:
        raise ValueError(f"{where}: A must be a device tensor")
    if A.dim() != 2 or A.stride(1) != 1:
        raise ValueError(f"{where}: A must be 2-D row-major (unit column stride)")
    if A.dtype == torch.float32:
        return 1
    if A.dtype == torch.float64:
        return 0
    raise ValueError(f"{where}: A must be float32 or float64")


def _dev(t, where, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise ValueError(f"{where}: {name} must be a device tensor")
    return t


def _rhs(b, A, where):
    """b as a contiguous device vector of A's dtype with at least A's n values (the
    library reads n of them: a shorter or host buffer would be read out of bounds)."""
    if b.numel() < A.shape[0]:
        raise ValueError(f"{where}: b holds {b.numel()} values, A has {A.shape[0]} rows")
    return _dev(b, where, "b").to(A.dtype).contiguous()


def _start(x0, length, device, where, name="x0"):
    """A private FP64 copy of a start vector of ``length`` values (zeros when None)."""
    if x0 is None:
        return torch.zeros(length, dtype=torch.float64, device=device)
    if x0.numel() != length:
        raise ValueError(f"{where}: {name} holds {x0.numel()} values, expected {length}")
    return _dev(x0, where, name).to(torch.float64).contiguous().clone()


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def padded(n, d, dtype=torch.float32, device="cuda"):
    """Row-major (n, d) tensor with a 16-byte-multiple leading dimension (view)."""
    es = torch.tensor([], dtype=dtype).element_size()
    vec = 16 // es
    ld = (d + vec - 1) // vec * vec
    return torch.zeros(n, ld, dtype=dtype, device=device)[:, :d]


# ------------------------------------------------------------------ entry points
def rs_params(kind="srht", rho=0.1, eta=0.01):
    p = IhsParams()
    _check(load().rs_params(SKETCH[kind], rho, eta, ctypes.byref(p)), "rs_params")
    return {k: getattr(p, k) for k, _ in IhsParams._fields_}


def rs_sketch_srht(A, m, seed=0, sketch_id=0, sa_dtype=None, rows=False, signs=False):
    """SA (m x d); for sa_dtype "fp8" returns (SA uint8 codes, column scales) in
    place of SA."""
    a_t = _mat(A, "rs_sketch_srht")
    n, d = A.shape
    sa_dtype = sa_dtype or ("f64" if a_t == 0 else "f32")
    SA = torch.empty(m, d, dtype=TORCH_DTYPES[sa_dtype], device=A.device)
    scale = torch.empty(d, dtype=torch.float32, device=A.device) if sa_dtype == "fp8" else None
    npad = 1 << max(0, math.ceil(math.log2(n)))
    R = torch.empty(m, dtype=torch.int64, device=A.device) if rows else None
    E = torch.empty(npad, dtype=torch.int8, device=A.device) if signs else None
    st = load().rs_sketch_srht(_ptr(A), a_t, n, d, A.stride(0), m, seed, sketch_id, _ptr(SA),
                               DTYPES[sa_dtype], SA.stride(0), _ptr(scale), _ptr(R), _ptr(E),
                               _stream())
    _check(st, "rs_sketch_srht")
    out = [(SA, scale) if scale is not None else SA]
    if rows:
        out.append(R)
    if signs:
        out.append(E)
    return out[0] if len(out) == 1 else tuple(out)


def rs_sketch_gaussian(A, m, seed=0, sketch_id=0, sa_dtype=None):
    a_t = _mat(A, "rs_sketch_gaussian")
    n, d = A.shape
    sa_dtype = sa_dtype or ("f64" if a_t == 0 else "f32")
    SA = torch.empty(m, d, dtype=TORCH_DTYPES[sa_dtype], device=A.device)
    scale = torch.empty(d, dtype=torch.float32, device=A.device) if sa_dtype == "fp8" else None
    st = load().rs_sketch_gaussian(_ptr(A), a_t, n, d, A.stride(0), m, seed, sketch_id, _ptr(SA),
                                   DTYPES[sa_dtype], SA.stride(0), _ptr(scale), _stream())
    _check(st, "rs_sketch_gaussian")
    return (SA, scale) if scale is not None else SA


class Factor:
    """Handle from rs_factor_woodbury; keeps SA alive while in use.  FP8 sketches
    are passed as (codes uint8, column scales float32)."""

    def __init__(self, SA, nu2):
        scale = None
        if isinstance(SA, tuple):
            SA, scale = SA
        if SA.dtype == torch.float32:
            sa_t = DTYPES["f32"]
        elif SA.dtype == torch.float64:
            sa_t = DTYPES["f64"]
        elif SA.dtype == torch.bfloat16:
            sa_t = DTYPES["bf16"]
        elif SA.dtype == torch.uint8:
            sa_t = DTYPES["fp8"]
        else:
            raise ValueError("SA dtype")
        self.SA, self.scale = SA, scale
        self.m, self.d = SA.shape
        h = ctypes.c_void_p()
        st = load().rs_factor_woodbury(_ptr(SA), sa_t, _ptr(scale), self.m, self.d, SA.stride(0),
                                       nu2, ctypes.byref(h), _stream())
        _check(st, "rs_factor_woodbury")
        self.handle = h

    def apply(self, G):
        """(H_S^-1 G, r) for G of shape (k, d) float64 (k right-hand sides)."""
        G = G.contiguous()
        k = G.shape[0]
        GT = torch.empty_like(G)
        r = torch.empty(k, dtype=torch.float64, device=G.device)
        _check(load().rs_factor_apply(self.handle, _ptr(G), _ptr(GT), _ptr(r), k, _stream()),
               "rs_factor_apply")
        return GT, r

    def close(self):
        if self.handle:
            torch.cuda.current_stream().synchronize()
            load().rs_factor_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def rs_factor_woodbury(SA, nu2):
    return Factor(SA, nu2)


def rs_factor_apply(F, G):
    return F.apply(G)


def rs_gradient(A, b, nu2, X):
    """G = A^T (A X - b) + nu2 X for X of shape (k, d) float64."""
    a_t = _mat(A, "rs_gradient")
    n, d = A.shape
    if X.dim() != 2 or X.shape[1] != d:
        raise ValueError(f"rs_gradient: X must be (k, {d})")
    X = _dev(X, "rs_gradient", "X").to(torch.float64).contiguous()
    G = torch.empty_like(X)
    bc = _rhs(b, A, "rs_gradient")
    st = load().rs_gradient(_ptr(A), a_t, n, d, A.stride(0), _ptr(bc), nu2, _ptr(X),
                            X.shape[0], _ptr(G), _stream())
    _check(st, "rs_gradient")
    return G


def rs_gradient_noalloc(A, b, nu2, X, G=None):
    """rs_gradient through the entry point that allocates no device memory (its
    partial sums live in the library's fixed device array).  X: (k, d) float64 on
    the device; G: None or a (k, d) float64 device tensor to write into."""
    a_t = _mat(A, "rs_gradient_noalloc")
    n, d = A.shape
    if X.dim() != 2 or X.shape[1] != d:
        raise ValueError(f"rs_gradient_noalloc: X must be (k, {d})")
    X = _dev(X, "rs_gradient_noalloc", "X")
    if X.dtype != torch.float64 or not X.is_contiguous():
        raise ValueError("rs_gradient_noalloc: X must be contiguous float64")
    if G is None:
        G = torch.empty_like(X)
    elif G.shape != X.shape or G.dtype != torch.float64 or not G.is_contiguous():
        raise ValueError("rs_gradient_noalloc: G must be a contiguous float64 tensor shaped as X")
    G = _dev(G, "rs_gradient_noalloc", "G")
    bc = _rhs(b, A, "rs_gradient_noalloc")
    st = load().rs_gradient_noalloc(_ptr(A), a_t, n, d, A.stride(0), _ptr(bc), nu2, _ptr(X),
                                    X.shape[0], _ptr(G), _stream())
    _check(st, "rs_gradient_noalloc")
    return G


def rs_ihs_step(A, b, nu2, F, params, variant, state):
    """One step; ``state`` is a dict with device tensors x, x_prev, g, gtilde and
    host values r_t, r_1, t (updated in place)."""
    a_t = _mat(A, "rs_ihs_step")
    n, d = A.shape
    p = IhsParams(**{k: params[k] for k, _ in IhsParams._fields_})
    s = IhsState(_ptr(state["x"]), _ptr(state["x_prev"]), _ptr(state["g"]), _ptr(state["gtilde"]),
                 state["r_t"], state["r_1"], state["t"])
    out = StepResult()
    st = load().rs_ihs_step(_ptr(A), a_t, n, d, A.stride(0), _ptr(b), nu2, F.handle,
                            ctypes.byref(p), VARIANT[variant], ctypes.byref(s), ctypes.byref(out),
                            _stream())
    _check(st, "rs_ihs_step")
    state["r_t"], state["t"] = s.r_t, s.t
    return {"accepted": out.accepted, "r_p": out.r_p, "r_gd": out.r_gd}


RS_SOLVE_TIMING = 4
_TIMING = [False]


def set_phase_timing(on=True):
    """Solves started after this call time their phases (RS_SOLVE_TIMING): their
    info dicts carry ms_sketch, ms_factor and ms_iterate."""
    _TIMING[0] = bool(on)


def _opts(a_t, kind, variant, resample, sketch_dtype, rho, eta, m_init, m_max, tol, max_iter,
          seed, check_every):
    o = SolveOpts()
    load().rs_solve_opts_default(ctypes.byref(o))
    o.kind, o.variant, o.resample = SKETCH[kind], VARIANT[variant], RESAMPLE[resample]
    o.sketch_dtype = DTYPES[sketch_dtype or ("f64" if a_t == 0 else "f32")]
    o.rho, o.eta, o.m_init, o.m_max, o.tol = rho, eta, m_init, m_max, tol
    o.max_iter, o.seed, o.check_every = max_iter, seed, check_every
    if _TIMING[0]:
        o.flags |= RS_SOLVE_TIMING
    return o


def rs_adaptive_solve(A, b, nu2, kind="srht", variant="polyak", resample="fresh",
                      sketch_dtype=None, rho=0.1, eta=0.01, m_init=1, m_max=0, tol=1e-7,
                      max_iter=200, seed=0, check_every=4, x0=None, raise_on_error=True,
                      ref_at_zero=False):
    """Algorithm 1 end to end.  Returns (x float64 tensor, info dict).  ref_at_zero
    takes the stop test's reference decrement at the origin."""
    a_t = _mat(A, "rs_adaptive_solve")
    n, d = A.shape
    o = _opts(a_t, kind, variant, resample, sketch_dtype, rho, eta, m_init, m_max, tol, max_iter,
              seed, check_every)
    o.flags |= RS_SOLVE_REF_AT_ZERO if ref_at_zero else 0
    x = _start(x0, d, A.device, "rs_adaptive_solve")
    bc = _rhs(b, A, "rs_adaptive_solve")
    info = SolveInfo()
    st = load().rs_adaptive_solve(_ptr(A), a_t, n, d, A.stride(0), _ptr(bc), nu2,
                                  ctypes.byref(o), _ptr(x), ctypes.byref(info), _stream())
    return x, _info(info, st, raise_on_error, "rs_adaptive_solve")


def _batch_problems(problems, where):
    a_ts = [_mat(A, where) for A, _, _ in problems]
    P = (Problem * len(problems))()
    xs, bs = [], []
    # one zeroed allocation for every solution (views of it, 16-byte aligned)
    offs, tot = [], 0
    for A, _, _ in problems:
        offs.append(tot)
        tot += (A.shape[1] + 1) // 2 * 2
    X = torch.zeros(max(tot, 1), dtype=torch.float64, device=problems[0][0].device)
    for i, (A, b, nu2) in enumerate(problems):
        n, d = A.shape
        x = X[offs[i]:offs[i] + d]
        bc = _rhs(b, A, where)
        xs.append(x)
        bs.append(bc)
        P[i] = Problem(_ptr(A), a_ts[i], 0, n, d, A.stride(0), _ptr(bc), float(nu2), _ptr(x))
    return a_ts, P, xs, bs


def rs_solve_batch(problems, kind="srht", variant="polyak", resample="fresh",
                   sketch_dtype=None, rho=0.1, eta=0.01, m_init=1, m_max=0, tol=1e-7,
                   max_iter=200, seed=0, check_every=4, workers=8, graph_steps=False,
                   raise_on_error=True):
    """Solve a list of (A, b, nu2) problems with one option set.  Returns a list of
    (x, info) pairs in the input order.  ``graph_steps`` replays each job's queued
    steps from HIP graphs."""
    if not problems:
        return []
    a_ts, P, xs, bs = _batch_problems(problems, "rs_solve_batch")
    o = _opts(a_ts[0], kind, variant, resample, sketch_dtype, rho, eta, m_init, m_max, tol,
              max_iter, seed, check_every)
    o.flags |= RS_SOLVE_GRAPH_STEPS if graph_steps else 0
    infos = (SolveInfo * len(problems))()
    st = load().rs_solve_batch(P, len(problems), ctypes.byref(o), infos, workers, _stream())
    if st != RS_OK and raise_on_error and st != RS_ERR_NO_CONVERGENCE:
        _check(st, "rs_solve_batch")
    return [(xs[i], _info(infos[i], infos[i].status, False, "rs_solve_batch"))
            for i in range(len(problems))]


def rs_learned_solve_batch(problems, params, mu, sd, kind="srht", variant="polyak",
                           resample="fresh", sketch_dtype=None, rho=0.1, eta=0.01, m_max=0,
                           tol=1e-7, max_iter=200, seed=0, check_every=4, workers=8,
                           graph_steps=False, raise_on_error=True):
    """Learned starting m for every problem, then the batched solve.  Returns a list
    of (x, info) pairs; info["m_init"] is the starting m used."""
    if not problems:
        return []
    a_ts, P, xs, bs = _batch_problems(problems, "rs_learned_solve_batch")
    o = _opts(a_ts[0], kind, variant, resample, sketch_dtype, rho, eta, 1, m_max, tol,
              max_iter, seed, check_every)
    o.flags |= RS_SOLVE_GRAPH_STEPS if graph_steps else 0
    infos = (SolveInfo * len(problems))()
    used = (ctypes.c_int64 * len(problems))()
    st = load().rs_learned_solve_batch(P, len(problems), ctypes.byref(o), _ptr(params), _ptr(mu),
                                       _ptr(sd), infos, used, workers, _stream())
    if st != RS_OK and raise_on_error and st != RS_ERR_NO_CONVERGENCE:
        _check(st, "rs_learned_solve_batch")
    out = []
    for i in range(len(problems)):
        inf = _info(infos[i], infos[i].status, False, "rs_learned_solve_batch")
        inf["m_init"] = int(used[i])
        out.append((xs[i], inf))
    return out


RS_SOLVE_PERSISTENT = 8


def rs_solve_nu_grid(A, b, nu2s, kind="srht", variant="polyak", resample="fresh",
                     sketch_dtype=None, rho=0.1, eta=0.01, m_init=1, m_max=0, tol=1e-7,
                     max_iter=200, seed=0, check_every=4, X0=None, raise_on_error=True,
                     persistent=False):
    """Solve for every nu^2 in ``nu2s`` on one (A, b).  Returns (X, infos) with X
    a (len(nu2s), d) float64 tensor of solutions.  ``persistent`` runs each window
    of check_every steps as one cooperative launch (RS_SOLVE_PERSISTENT)."""
    a_t = _mat(A, "rs_solve_nu_grid")
    n, d = A.shape
    k = len(nu2s)
    o = _opts(a_t, kind, variant, resample, sketch_dtype, rho, eta, m_init, m_max, tol, max_iter,
              seed, check_every)
    o.flags |= RS_SOLVE_PERSISTENT if persistent else 0
    if X0 is not None and tuple(X0.shape) != (k, d):
        raise ValueError(f"rs_solve_nu_grid: X0 must be ({k}, {d})")
    X = (torch.zeros(k, d, dtype=torch.float64, device=A.device) if X0 is None
         else _dev(X0, "rs_solve_nu_grid", "X0").to(torch.float64).contiguous().clone())
    bc = _rhs(b, A, "rs_solve_nu_grid")
    nu = (ctypes.c_double * k)(*[float(v) for v in nu2s])
    infos = (SolveInfo * k)()
    st = load().rs_solve_nu_grid(_ptr(A), a_t, n, d, A.stride(0), _ptr(bc), nu, k,
                                 ctypes.byref(o), _ptr(X), infos, _stream())
    if st != RS_OK and raise_on_error and st != RS_ERR_NO_CONVERGENCE:
        _check(st, "rs_solve_nu_grid")
    return X, [_info(infos[i], infos[i].status, False, "rs_solve_nu_grid") for i in range(k)]


def rs_adaptive_solve_dual(A, b, nu2, kind="srht", variant="polyak", resample="fresh",
                           sketch_dtype=None, rho=0.1, eta=0.01, m_init=1, m_max=0, tol=1e-7,
                           max_iter=200, seed=0, check_every=4, z0=None, raise_on_error=True,
                           ref_at_zero=False):
    """The underdetermined case (n <= d) through the dual problem.  Returns
    (x, z, info): x = A^T z the primal solution (d), z the dual one (n), both
    float64 tensors."""
    a_t = _mat(A, "rs_adaptive_solve_dual")
    n, d = A.shape
    o = _opts(a_t, kind, variant, resample, sketch_dtype, rho, eta, m_init, m_max, tol, max_iter,
              seed, check_every)
    o.flags |= RS_SOLVE_REF_AT_ZERO if ref_at_zero else 0
    z = _start(z0, n, A.device, "rs_adaptive_solve_dual", "z0")
    bc = _rhs(b, A, "rs_adaptive_solve_dual")
    x = torch.zeros(d, dtype=torch.float64, device=A.device)
    info = SolveInfo()
    st = load().rs_adaptive_solve_dual(_ptr(A), a_t, n, d, A.stride(0), _ptr(bc), nu2,
                                       ctypes.byref(o), _ptr(z), _ptr(x), ctypes.byref(info),
                                       _stream())
    return x, z, _info(info, st, raise_on_error, "rs_adaptive_solve_dual")


def rs_adaptive_solve_csr(rowptr, col, val, d, b, nu2, variant="polyak", resample="fresh",
                          sketch_dtype=None, rho=0.1, m_init=1, m_max=0, tol=1e-7, max_iter=200,
                          seed=0, check_every=4, x0=None, raise_on_error=True):
    """Algorithm 1 with the CountSketch for a sparse A given as device CSR tensors
    (rowptr int64 n + 1, col int32 nnz, val float32/float64 nnz).  Returns (x, info)."""
    if rowptr.dtype != torch.int64 or col.dtype != torch.int32:
        raise RsError(1, "rs_adaptive_solve_csr", "rowptr must be int64 and col int32")
    if val.dtype not in (torch.float32, torch.float64) or b.dtype != val.dtype:
        raise RsError(1, "rs_adaptive_solve_csr", "val and b must share float32 or float64")
    a_t = 0 if val.dtype == torch.float64 else 1
    n = rowptr.numel() - 1
    if n < 1 or val.numel() != col.numel() or b.numel() < n:
        raise ValueError("rs_adaptive_solve_csr: needs n >= 1 rows, one value per column "
                         "index and n values of b")
    for t, name in ((rowptr, "rowptr"), (col, "col"), (val, "val"), (b, "b")):
        _dev(t, "rs_adaptive_solve_csr", name)
    o = _opts(a_t, "count", variant, resample, sketch_dtype, rho, 0.01, m_init, m_max, tol,
              max_iter, seed, check_every)
    x = _start(x0, d, val.device, "rs_adaptive_solve_csr")
    info = SolveInfo()
    st = load().rs_adaptive_solve_csr(_ptr(rowptr.contiguous()), _ptr(col.contiguous()),
                                      _ptr(val.contiguous()), a_t, n, d, col.numel(),
                                      _ptr(b.contiguous()), nu2, ctypes.byref(o), _ptr(x),
                                      ctypes.byref(info), _stream())
    return x, _info(info, st, raise_on_error, "rs_adaptive_solve_csr")


def rs_refreshed_ihs(A, b, nu2, m, kind="srht", variant="gd", sketch_dtype=None, rho=0.1,
                     eta=0.01, tol=1e-7, max_iter=200, seed=0, x0=None, raise_on_error=True):
    """IHS with a new sketch of size m at every step (the refreshed-embedding
    ablation).  Returns (x, r_history list, info dict)."""
    a_t = _mat(A, "rs_refreshed_ihs")
    n, d = A.shape
    o = _opts(a_t, kind, variant, "fresh", sketch_dtype, rho, eta, m, 0, tol, max_iter, seed, 1)
    x = _start(x0, d, A.device, "rs_refreshed_ihs")
    bc = _rhs(b, A, "rs_refreshed_ihs")
    rh = (ctypes.c_double * (max_iter + 1))()
    info = SolveInfo()
    st = load().rs_refreshed_ihs(_ptr(A), a_t, n, d, A.stride(0), _ptr(bc), nu2,
                                 ctypes.byref(o), _ptr(x), rh, ctypes.byref(info), _stream())
    res = _info(info, st, raise_on_error, "rs_refreshed_ihs")
    return x, [rh[i] for i in range(min(info.grad_passes, max_iter + 1))], res


def rs_solve_path(A, b, nu2s, kind="srht", variant="polyak", sketch_dtype=None, rho=0.1,
                  eta=0.01, m_init=1, m_max=0, tol=1e-7, max_iter=200, seed=0, check_every=4,
                  x0=None, raise_on_error=True):
    """Regularization path over the non-increasing ``nu2s`` with warm starts and
    nested sketches.  Returns (X, infos) with X a (len(nu2s), d) float64 tensor of
    solutions; x0 is the first start (zeros when None)."""
    a_t = _mat(A, "rs_solve_path")
    n, d = A.shape
    k = len(nu2s)
    o = _opts(a_t, kind, variant, "nested", sketch_dtype, rho, eta, m_init, m_max, tol, max_iter,
              seed, check_every)
    X = torch.zeros(max(k, 1), d, dtype=torch.float64, device=A.device)
    if x0 is not None:
        X[0] = _start(x0, d, A.device, "rs_solve_path")
    bc = _rhs(b, A, "rs_solve_path")
    nu = (ctypes.c_double * max(k, 1))(*[float(v) for v in nu2s])
    infos = (SolveInfo * max(k, 1))()
    st = load().rs_solve_path(_ptr(A), a_t, n, d, A.stride(0), _ptr(bc), nu, k,
                              ctypes.byref(o), _ptr(X), infos, _stream())
    if st != RS_OK and raise_on_error and st != RS_ERR_NO_CONVERGENCE:
        _check(st, "rs_solve_path")
    return X[:k], [_info(infos[i], infos[i].status, False, "rs_solve_path") for i in range(k)]


def _info(info, st, raise_on_error, where):
    res = {
        "status": STATUS_NAMES.get(info.status, str(info.status)),
        "m_final": info.m_final, "doublings": info.doublings, "steps": info.steps,
        "grad_passes": info.grad_passes, "applies": info.applies,
        "accepted_polyak": info.accepted_polyak, "accepted_gd": info.accepted_gd,
        "r_final": info.r_final, "r_ref": info.r_ref,
        "ms_sketch": info.ms_sketch, "ms_factor": info.ms_factor,
        "ms_iterate": info.ms_iterate,
        "events": [(int(info.event_t[i]), EVENT_NAMES[int(info.event_kind[i])],
                    int(info.event_m[i])) for i in range(info.n_events)],
    }
    if st != RS_OK and raise_on_error and st != RS_ERR_NO_CONVERGENCE:
        _check(st, where)
    res["status_code"] = st
    return res


def rs_features(A, nu2, seed=0):
    """16 FP32 features of (A, nu2) on the device."""
    a_t = _mat(A, "rs_features")
    n, d = A.shape
    f = torch.empty(16, dtype=torch.float32, device=A.device)
    _check(load().rs_features(_ptr(A), a_t, n, d, A.stride(0), nu2, seed, _ptr(f), _stream()),
           "rs_features")
    return f


def rs_mlp_forward(params, X, mu, sd, cache=False):
    X = X.contiguous()
    B = X.shape[0]
    y = torch.empty(B, dtype=torch.float32, device=X.device)
    C = torch.empty(B, MLP_CACHE, dtype=torch.float32, device=X.device) if cache else None
    _check(load().rs_mlp_forward(_ptr(params), _ptr(X), B, _ptr(mu), _ptr(sd), _ptr(y), _ptr(C),
                                 _stream()), "rs_mlp_forward")
    return (y, C) if cache else y


def rs_mlp_backward(params, cache, t):
    B = t.shape[0]
    G = torch.empty(MLP_PARAMS, dtype=torch.float32, device=t.device)
    loss = torch.empty(1, dtype=torch.float32, device=t.device)
    work = torch.empty(B, MLP_WORK, dtype=torch.float32, device=t.device)
    _check(load().rs_mlp_backward(_ptr(params), _ptr(cache), _ptr(t.contiguous()), B, _ptr(G),
                                  _ptr(loss), _ptr(work), _stream()), "rs_mlp_backward")
    return G, loss


def rs_mlp_adam_step(params, grad, m, v, step, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    _check(load().rs_mlp_adam_step(_ptr(params), _ptr(grad), _ptr(m), _ptr(v), params.numel(),
                                   step, lr, b1, b2, eps, _stream()), "rs_mlp_adam_step")


def rs_learned_solve(A, b, nu2, params, mu, sd, kind="srht", variant="polyak", resample="fresh",
                     sketch_dtype=None, rho=0.1, eta=0.01, m_max=0, tol=1e-7, max_iter=200,
                     seed=0, check_every=4, x0=None, raise_on_error=True):
    """Learned starting m, then Algorithm 1.  Returns (x, info) with info["m_init"]."""
    a_t = _mat(A, "rs_learned_solve")
    n, d = A.shape
    o = _opts(a_t, kind, variant, resample, sketch_dtype, rho, eta, 1, m_max, tol, max_iter,
              seed, check_every)
    x = _start(x0, d, A.device, "rs_learned_solve")
    bc = _rhs(b, A, "rs_learned_solve")
    info = SolveInfo()
    used = ctypes.c_int64(0)
    st = load().rs_learned_solve(_ptr(A), a_t, n, d, A.stride(0), _ptr(bc), nu2,
                                 ctypes.byref(o), _ptr(params), _ptr(mu), _ptr(sd), _ptr(x),
                                 ctypes.byref(info), ctypes.byref(used), _stream())
    res = _info(info, st, raise_on_error, "rs_learned_solve")
    res["m_init"] = used.value
    return x, res


def rs_gradient_two(A, b, nu2s, X0, X1):
    """(G0, G1) for two problems sharing FP32 A and b, X_j of shape (2, d) float64, in
    one read of A; each equals rs_gradient(A, b, nu2s[j], X_j)."""
    if _mat(A, "rs_gradient_two") != DTYPES["f32"]:
        raise ValueError("rs_gradient_two: A must be float32")
    n, d = A.shape
    Xs = []
    for X in (X0, X1):
        if X.dim() != 2 or tuple(X.shape) != (2, d):
            raise ValueError(f"rs_gradient_two: X must be (2, {d})")
        Xs.append(_dev(X, "rs_gradient_two", "X").to(torch.float64).contiguous())
    G0, G1 = torch.empty_like(Xs[0]), torch.empty_like(Xs[1])
    bc = _rhs(b, A, "rs_gradient_two")
    nu = (ctypes.c_double * 2)(float(nu2s[0]), float(nu2s[1]))
    st = load().rs_gradient_two(_ptr(A), n, d, A.stride(0), _ptr(bc),
                                ctypes.cast(nu, ctypes.c_void_p), _ptr(Xs[0]), _ptr(Xs[1]),
                                _ptr(G0), _ptr(G1), _stream())
    _check(st, "rs_gradient_two")
    return G0, G1


def rs_gradient_autotune(A, b, k=2):
    """Tune the gradient pass for this problem and k; returns the chosen plan
    (threads per row, vectors per thread, blocks, rows per group and step)."""
    a_t = _mat(A, "rs_gradient_autotune")
    n, d = A.shape
    plan = (ctypes.c_int32 * 4)()
    bc = _rhs(b, A, "rs_gradient_autotune")
    _check(load().rs_gradient_autotune(_ptr(A), a_t, n, d, A.stride(0), _ptr(bc), k,
                                       ctypes.cast(plan, ctypes.c_void_p), _stream()),
           "rs_gradient_autotune")
    return tuple(plan)


def rs_gradient_plan(dtype, n, d, k):
    plan = (ctypes.c_int32 * 4)()
    _check(load().rs_gradient_plan(DTYPES[dtype], n, d, k, ctypes.cast(plan, ctypes.c_void_p)),
           "rs_gradient_plan")
    return tuple(plan)


def rs_gradient_set_plan(dtype, n, d, k, plan):
    """Fix the gradient plan (threads per row, vectors, grid, rows per step) of a key."""
    arr = (ctypes.c_int32 * 4)(*[int(v) for v in plan])
    _check(load().rs_gradient_set_plan(DTYPES[dtype], n, d, k, ctypes.cast(arr, ctypes.c_void_p)),
           "rs_gradient_set_plan")


def rs_profile_enable(on=True):
    _check(load().rs_profile_enable(1 if on else 0), "rs_profile_enable")


def rs_profile_read():
    """(launches, total_ms) of the bracketed gradient partial-sum launches."""
    n = ctypes.c_int64()
    ms = ctypes.c_double()
    _check(load().rs_profile_read(ctypes.byref(n), ctypes.byref(ms)), "rs_profile_read")
    return n.value, ms.value


def version():
    return load().rs_version().decode()
