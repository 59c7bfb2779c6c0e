"""MI355X (gfx950) implementation of CPAA, the Chebyshev Polynomial Approximation
Algorithm for PageRank on undirected graphs (arXiv 2112.01743).

The computation lives in the HIP library ``libcpaa.so`` (C ABI in
``include/cpaa.h``); this package holds its sources (``csrc/``), the build
script and a ctypes binding.  Nothing here falls back to a CPU path: if the
library is missing, ``binding.lib()`` raises.
"""
from .binding import (CpaaError, Plan, cpaa_default_opts, cpaa_last_error, cpaa_plan,  # noqa: F401
                      cpaa_plan_destroy, cpaa_plan_info_get, cpaa_solve, cpaa_solve_batched,
                      cpaa_solve_graphs, cpaa_solve_power, cpaa_solve_power_batched, lib)

__all__ = ["Plan", "CpaaError", "lib", "cpaa_default_opts", "cpaa_last_error", "cpaa_plan",
           "cpaa_plan_destroy", "cpaa_plan_info_get", "cpaa_solve", "cpaa_solve_batched",
           "cpaa_solve_graphs", "cpaa_solve_power", "cpaa_solve_power_batched"]
