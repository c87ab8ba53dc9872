"""Seeded synthetic ridge problems shared by the tests, the smoke run and the bench.

This module holds no arithmetic of the solver: it only draws inputs.  Shapes and
spectra follow the paper's synthetic experiments (Appendix A.1: exponential and
polynomial singular-value decays): A = G diag(sigma) V^T with G i.i.d.
N(0, 1/n) and V Haar-distributed, b = A x_pl + c * xi.
"""
from .problems import (Problem, make_problem, spectrum, config_c1, config_c2,
                       config_c4b_specs, make_c4b_problem, make_problem_torch,
                       config_c4a_nu2, make_c4a_problem, config_path_nu2,
                       make_path_problem, make_wide_problem_torch, make_dual_problem,
                       make_sparse_problem, config_sparse)

__all__ = ["Problem", "make_problem", "spectrum", "config_c1", "config_c2",
           "config_c4b_specs", "make_c4b_problem", "make_problem_torch",
           "config_c4a_nu2", "make_c4a_problem", "config_path_nu2", "make_path_problem",
           "make_wide_problem_torch", "make_dual_problem", "make_sparse_problem",
           "config_sparse"]
