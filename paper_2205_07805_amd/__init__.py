"""MI355X-native iterated Gauss-Seidel GMRES (one global reduction per Arnoldi step).

The solver is the C-ABI library ``libigs.so`` (HIP kernels for gfx950, see
``include/igs.h``); ``igs`` is its ctypes binding and ``Solver`` a small
convenience wrapper that keeps device buffers in torch tensors.
"""
from . import igs
from .igs import (IgsError, IgsInfo, IgsOpts, IgsRequest, igs_create, igs_create_dense,
                  igs_debug_copy_H, igs_debug_copy_V, igs_destroy, igs_kernel_reduce, igs_kernel_spmv,
                  igs_kernel_update, igs_last_error, igs_profile_get, igs_profile_reset,
                  igs_serve, igs_serve_batched, igs_solve, igs_solve_batch, igs_solve_opts,
                  igs_tune, igs_tune_reset, load_library)
from .serving import serve
from .solver import Solver, solve_batch

__all__ = [
    "igs", "IgsError", "IgsInfo", "IgsOpts", "IgsRequest", "Solver", "load_library", "serve",
    "igs_create", "igs_create_dense", "igs_solve", "igs_solve_opts", "igs_destroy",
    "igs_last_error", "igs_debug_copy_H", "igs_debug_copy_V", "igs_kernel_spmv",
    "igs_kernel_reduce", "igs_kernel_update", "igs_profile_get", "igs_profile_reset",
    "igs_serve", "igs_solve_batch", "igs_serve_batched", "solve_batch", "igs_tune",
    "igs_tune_reset",
]
