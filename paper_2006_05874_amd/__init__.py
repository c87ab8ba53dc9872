"""MI355X (gfx950) adaptive Hessian-sketch ridge solver.

The compute path is librs.so (HIP kernels behind the C ABI in include/rs.h);
this package holds its ctypes binding (``rs``) and its build script.
"""
from .rs import (RsError, Factor, load, padded, rs_adaptive_solve, rs_factor_apply,
                 rs_factor_woodbury, rs_gradient, rs_ihs_step, rs_params, rs_sketch_gaussian,
                 rs_sketch_srht, version)

__all__ = ["RsError", "Factor", "load", "padded", "rs_adaptive_solve", "rs_factor_apply",
           "rs_factor_woodbury", "rs_gradient", "rs_ihs_step", "rs_params", "rs_sketch_gaussian",
           "rs_sketch_srht", "version"]
