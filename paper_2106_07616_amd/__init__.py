"""MI355X (gfx950) implementation of the data-parallel hot path of the
semi-implicit PHS-RBF meshless solver of Shahane & Vanka (arXiv 2106.07616).

The computation lives in librbffd.so (HIP kernels behind the C ABI of
include/rbffd.h); this package holds the ctypes binding and the host-side time
loop (Sec. 3.2: outer tolerance min(1e-4, dt * eps_s); Sec. 4.1: steady error).
"""
from __future__ import annotations

from .binding import (BDF1, BDF2, RBFFD_FP32_IR, RBFFD_FP32_MATRIX, RBFFD_FP64, RBFFD_PREC_BLOCK64, RBFFD_PREC_JACOBI,
                      Context, DeviceCloud, Operators, RbffdError, Server, lib, poisson_solve, poisson_solve_batched,
                      poisson_solve_noalloc, rbffd_autotune_krylov, rbffd_krylov_kernel_times,
                      rbffd_assemble, rbffd_build_stencils, rbffd_build_stencils_batched, rbffd_convdiff_lambda, rbffd_cylinder_forces, rbffd_interpolate,
                      rbffd_stencil_sizes, simple_step, simple_step_batched)
from .driver import Solver, outer_tolerance

__all__ = ["BDF1", "BDF2", "RBFFD_FP32_IR", "RBFFD_FP32_MATRIX", "RBFFD_FP64", "RBFFD_PREC_BLOCK64", "RBFFD_PREC_JACOBI",
           "Context", "DeviceCloud", "Operators", "RbffdError", "Server", "lib", "poisson_solve", "poisson_solve_batched",
           "poisson_solve_noalloc", "rbffd_autotune_krylov", "rbffd_krylov_kernel_times",
           "rbffd_assemble", "rbffd_build_stencils", "rbffd_build_stencils_batched", "rbffd_convdiff_lambda", "rbffd_cylinder_forces", "rbffd_interpolate",
           "rbffd_stencil_sizes", "simple_step", "simple_step_batched", "Solver", "outer_tolerance"]
