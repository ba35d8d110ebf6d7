"""Plain FP64 CPU oracle for iterated Gauss-Seidel GMRES -- TEST INFRASTRUCTURE ONLY.

This package is the slow, obviously-correct reference the HIP path is checked
against.  It is written from the paper's definitions and algorithms (GMRES as
the Arnoldi-QR factorisation with a Givens least-squares solve; Gram-Schmidt
projection as Gauss-Seidel / Jacobi sweeps on the normal equations; the
two-reduce Algorithm 4.1 and the one-reduce Algorithm 4.2) in numpy float64,
with plain loops and no blocking, fusion or reordering beyond what those
definitions state.

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import it.  The product path (the C-ABI library and its Python
binding) never imports, links or calls anything here, and nothing here imports
the product path.  Inputs come from the separate ``workloads`` module.

Parity status of each function is listed in its module docstring; a function
whose result is pinned by no test says "parity unpinned" there.
"""
from .operators import CsrOperator, DenseOperator, as_operator
from .projector import forward_subst_unit_lower, gs_project, strictly_lower_gram
from .lsq import GivensLS, back_substitution
from .arnoldi import (CycleResult, StopRule, cycle_mgs, cycle_householder,
                      cycle_igs_2r, cycle_igs_1r, householder_arnoldi, canonical_signs)
from .gmres import SolveResult, gmres
from . import diagnostics

__all__ = [
    "CsrOperator", "DenseOperator", "as_operator",
    "forward_subst_unit_lower", "gs_project", "strictly_lower_gram",
    "GivensLS", "back_substitution",
    "CycleResult", "StopRule", "cycle_mgs", "cycle_householder", "cycle_igs_2r",
    "cycle_igs_1r", "householder_arnoldi", "canonical_signs",
    "SolveResult", "gmres", "diagnostics",
]
