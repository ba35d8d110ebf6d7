"""Pins for the oracle's restarted GMRES: exact solves, minimal residual,
closed-form convergence, backward error, restart and stopping semantics."""
import math

import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import diagnostics as D

ALL = [("igs1r", 2), ("igs2r", 2), ("igs2r", 1), ("mgs", 1), ("householder", 1)]


@pytest.mark.parametrize("variant,gs", ALL)
@pytest.mark.parametrize("case", ["rand8", "rand16", "rand32", "walker10", "convdiff4"])
def test_full_gmres_matches_lu(case, variant, gs):
    """With m = n GMRES is exact: x equals a dense LU solve to O(eps kappa)."""
    if case.startswith("rand"):
        n = int(case[4:])
        a = W.random_wellcond(n, n)
        b = W.rhs_normal(n, n + 1)
    elif case == "walker10":
        a, b = W.walker(10, 2000.0), np.ones(10)
    else:
        a = W.convdiff2d(4, 10.0).to_dense()
        b = W.rhs_normal(16, 2)
    n = b.size
    res = O.gmres(a, b, restart=n, tol=1e-15, variant=variant, gs_iters=gs, maxit=4 * n)
    x_lu = np.linalg.solve(a, b)
    kappa = np.linalg.cond(a)
    err = np.linalg.norm(res.x - x_lu) / np.linalg.norm(x_lu)
    assert err <= 1e2 * n * np.finfo(float).eps * kappa, (err, kappa)
    anorm = np.linalg.norm(a, 2)
    assert D.backward_error(O.as_operator(a), b, res.x, anorm) <= 1e-14


def _krylov_minimiser(a, b, x0, k):
    r0 = b - a @ x0
    K = np.empty((b.size, k))
    v = r0.copy()
    for i in range(k):
        K[:, i] = v
        v = a @ v
    Q, _ = np.linalg.qr(K)                   # orthonormal basis of K_k(A, r0)
    y = np.linalg.lstsq(a @ Q, r0, rcond=None)[0]
    return x0 + Q @ y


@pytest.mark.parametrize("variant,gs", ALL)
def test_minimal_residual_property(variant, gs):
    """x_k minimises ||b - A x|| over x0 + K_k(A, r0) (eq:llse) -- brute force on tiny n."""
    a = W.random_wellcond(12, 21)
    b = W.rhs_normal(12, 22)
    x0 = W.rhs_normal(12, 23) * 0.1
    for k in range(1, 8):
        res = O.gmres(a, b, x0=x0, restart=k, tol=0.0, variant=variant, gs_iters=gs, max_cycles=1)
        xb = _krylov_minimiser(a, b, x0, k)
        r_o = np.linalg.norm(b - a @ res.x)
        r_b = np.linalg.norm(b - a @ xb)
        assert r_o == pytest.approx(r_b, rel=1e-10), (k, r_o, r_b)
        assert np.allclose(res.x, xb, rtol=1e-9, atol=1e-12)


@pytest.mark.parametrize("variant", ["igs1r", "igs2r"])
def test_embree_closed_form_bound(variant):
    """A = I + delta S: GMRES residual obeys ||r_k|| <= delta^k ||r_0||."""
    delta = 0.1
    a = W.embree_bidiag(100, delta)
    b = W.rhs_normal(100, 3)
    c = O.gmres(a, b, restart=20, tol=0.0, variant=variant, gs_iters=2, max_cycles=1).first_cycle
    rho = c.rho
    for k, g in enumerate(c.res_hist, start=1):
        assert g <= delta ** k * rho * (1 + 1e-9) + 1e-15 * rho, (k, g / rho)


@pytest.mark.parametrize("tol,beta_max", [(1e-12, 1e-12), (1e-13, 1e-14)])
def test_convdiff2d_backward_error_and_counts(tol, beta_max):
    """All variants take the same number of iterations and reach the backward-error target."""
    a, b = W.make_convdiff2d_32()
    op = O.as_operator(a)
    anorm = D.norm2(op)
    counts = {}
    for variant, gs in ALL[:4]:
        res = O.gmres(a, b, restart=50, tol=tol, variant=variant, gs_iters=gs)
        assert res.converged
        assert res.relres_true <= tol
        assert D.backward_error(op, b, res.x, anorm) <= beta_max
        counts[(variant, gs)] = res.iters
    assert max(counts.values()) - min(counts.values()) <= 2, counts


def test_restart_semantics():
    a = W.convdiff2d(12, 20.0)
    b = W.rhs_normal(a.n, 9)
    res = O.gmres(a, b, restart=7, tol=1e-10, variant="igs1r")
    assert res.converged and res.iters == sum(res.cycle_J)
    assert all(J == 7 for J in res.cycle_J[:-1])
    assert res.cycles == len(res.cycle_J)
    # the budget is honoured exactly and reported as not converged
    cut = O.gmres(a, b, restart=7, tol=1e-10, variant="igs1r", maxit=17)
    assert not cut.converged and cut.iters == 17
    # restarting from the returned x continues the solve (x is the whole state)
    cont = O.gmres(a, b, x0=cut.x, restart=7, tol=1e-10, variant="igs1r")
    assert cont.converged


def test_happy_breakdown():
    """b in a 2-D invariant subspace: the cycle breaks down at j = 2 with the exact solution."""
    n = 30
    a = np.diag(np.arange(1.0, n + 1))
    b = np.zeros(n)
    b[0] = b[1] = 1.0
    for variant, gs in ALL[:4]:
        res = O.gmres(a, b, restart=10, tol=1e-14, variant=variant, gs_iters=gs)
        assert res.first_cycle.status == "breakdown" and res.first_cycle.J == 2
        assert res.converged and res.iters == 2
        assert np.allclose(res.x, np.linalg.solve(a, b), atol=1e-14)


def test_lagnorm_guard_forced():
    """Forcing the lagged-norm guard ends every cycle after the explicit-norm column."""
    a = W.embree_bidiag(60, 0.3)
    b = W.rhs_normal(60, 1)
    res = O.gmres(a, b, restart=10, tol=1e-12, variant="igs1r", lagnorm_tau=2.0)
    assert res.converged
    assert res.lagnorm_fallbacks == res.cycles
    assert all(J == 1 for J in res.cycle_J)
    # the explicit norm keeps the Arnoldi relation exact on the finished column
    c = res.first_cycle
    anorm = np.linalg.norm(a, 2)
    assert D.arnoldi_relation_residual(O.as_operator(a), c.V, c.H, anorm) < 1e-14


def test_zero_rhs_and_exact_initial_guess():
    a = W.random_wellcond(10, 1)
    res = O.gmres(a, np.zeros(10), restart=5, tol=1e-12)
    assert res.converged and res.iters == 0 and np.all(res.x == 0)
    b = W.rhs_normal(10, 2)
    x = np.linalg.solve(a, b)
    res = O.gmres(a, b, x0=x, restart=5, tol=1e-12)
    assert res.converged and res.iters == 0


def test_input_validation():
    a = W.random_wellcond(5, 1)
    b = np.ones(5)
    with pytest.raises(ValueError):
        O.gmres(a, b, restart=0)
    with pytest.raises(ValueError):
        O.gmres(a, b, tol=-1.0)
    with pytest.raises(ValueError):
        O.gmres(a, b, variant="igs1r", gs_iters=1)
    with pytest.raises(ValueError):
        O.gmres(a, b, variant="nope")
