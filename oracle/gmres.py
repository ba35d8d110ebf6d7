"""Restarted GMRES(m) driver around the Arnoldi cycles (Section 1, Section 4).

The paper gives one cycle (Algorithms 4.1/4.2 followed by the least-squares
solve and ``x = x0 + V y``); restarts and stopping are not specified there and
are read as follows.  Each cycle starts from the explicit residual
``r = b - A x``; the solve is converged when ``||r|| <= tol ||b||`` at the start
of a cycle.  Inside a cycle the Arnoldi residual ``|g_J| <= tol ||b||`` ends the
cycle early, after which ``x += V_J y`` and the next cycle re-checks the true
residual.  The iteration count is the sum of finished columns ``J`` over all
cycles; ``maxit`` (default ``20 n``) bounds it.

Pinned by: tests/test_oracle_gmres.py -- full GMRES (m = n) against a dense
LU solve, the minimal-residual property against a brute-force least-squares
minimiser over the Krylov space, the closed-form bound for Embree's
bidiagonal matrix, backward error at machine precision, restart semantics.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

from .arnoldi import StopRule, cycle_householder, cycle_igs_1r, cycle_igs_2r, cycle_mgs
from .operators import as_operator

VARIANTS = ("igs1r", "igs2r", "mgs", "householder")


@dataclass
class SolveResult:
    x: np.ndarray
    iters: int
    cycles: int
    converged: bool
    relres_true: float            # ||b - A x|| / ||b|| at the last check
    status: str
    first_cycle: object = None    # CycleResult of cycle 0 (V, H, L ...)
    cycle_J: list = field(default_factory=list)
    res_hist: list = field(default_factory=list)   # Arnoldi residual / ||b|| per iteration
    lagnorm_fallbacks: int = 0
    breakdowns: int = 0


def run_cycle(op, r0, m, stop, variant, gs_iters, jacobi=False):
    if variant == "igs1r":
        if gs_iters != 2:
            raise ValueError("the one-reduce variant applies two Gauss-Seidel sweeps")
        return cycle_igs_1r(op, r0, m, stop, jacobi=jacobi)
    if variant == "igs2r":
        return cycle_igs_2r(op, r0, m, stop, gs_iters=gs_iters)
    if variant == "mgs":
        return cycle_mgs(op, r0, m, stop)
    if variant == "householder":
        return cycle_householder(op, r0, m, stop)
    raise ValueError(f"unknown variant {variant!r}")


def gmres(a, b, x0=None, restart: int = 50, tol: float = 1e-12, variant: str = "igs1r",
          gs_iters: int = 2, maxit: int | None = None, jacobi: bool = False,
          lagnorm_tau: float = 1e-4, max_cycles: int | None = None) -> SolveResult:
    """Solve A x = b with restarted GMRES built on the chosen Arnoldi variant."""
    op = as_operator(a)
    b = np.asarray(b, dtype=np.float64)
    n = b.size
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    m = min(int(restart), n)
    if m < 1:
        raise ValueError("restart must be >= 1")
    if tol < 0:
        raise ValueError("tol must be >= 0")
    maxit = 20 * n if maxit is None else int(maxit)
    nb = math.sqrt(b @ b)
    tol_abs = tol * nb
    its = cycles = fallbacks = breakdowns = 0
    first = None
    cycle_J, hist = [], []
    status = "maxit"
    converged = False
    while True:
        r = b - op.matvec(x)
        rho = math.sqrt(r @ r)
        relres = rho / nb if nb > 0 else rho
        if rho <= tol_abs:
            converged, status = True, "converged"
            break
        if its >= maxit or (max_cycles is not None and cycles >= max_cycles):
            break
        stop = StopRule(tol_abs=tol_abs, its_left=maxit - its, lagnorm_tau=lagnorm_tau)
        cyc = run_cycle(op, r, m, stop, variant, gs_iters, jacobi)
        if first is None:
            first = cyc
        x = x + cyc.V[:, : cyc.J] @ cyc.y
        its += cyc.J
        cycles += 1
        cycle_J.append(cyc.J)
        hist.extend((cyc.res_hist / nb).tolist() if nb > 0 else cyc.res_hist.tolist())
        fallbacks += cyc.lagnorm_fallbacks
        breakdowns += cyc.status == "breakdown"
    return SolveResult(x=x, iters=its, cycles=cycles, converged=converged,
                       relres_true=relres, status=status, first_cycle=first,
                       cycle_J=cycle_J, res_hist=hist, lagnorm_fallbacks=fallbacks,
                       breakdowns=breakdowns)
