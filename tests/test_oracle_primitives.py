"""Pins for the oracle's building blocks: operators, triangular solves, Givens LS,
the Gauss-Seidel projector identities and the diagnostics."""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import diagnostics as D


def test_csr_matvec_matches_dense():
    rng = np.random.default_rng(0)
    for a in (W.convdiff2d(9, 7.0), W.convdiff3d(5, 50.0)):
        d = a.to_dense()
        op = O.as_operator(a)
        x = rng.standard_normal(a.n)
        assert np.allclose(op.matvec(x), d @ x, rtol=1e-14, atol=1e-13)
        assert np.allclose(op.rmatvec(x), d.T @ x, rtol=1e-14, atol=1e-13)


def test_csr_matvec_empty_rows_and_random_pattern():
    rng = np.random.default_rng(1)
    d = rng.standard_normal((40, 40)) * (rng.random((40, 40)) < 0.1)
    d[7, :] = 0.0          # an empty row
    a = W.csr_from_dense(d)
    x = rng.standard_normal(40)
    assert np.allclose(O.as_operator(a).matvec(x), d @ x, atol=1e-14)


def test_forward_substitution_against_library_solve():
    rng = np.random.default_rng(2)
    for k in (1, 2, 7, 40):
        L = np.tril(rng.standard_normal((k, k)) * 0.3, -1)
        r = rng.standard_normal(k)
        x = O.forward_subst_unit_lower(L, r)
        assert np.allclose(x, np.linalg.solve(np.eye(k) + L, r), rtol=1e-12, atol=1e-12)


def test_givens_ls_against_lstsq():
    rng = np.random.default_rng(3)
    m = 12
    H = np.triu(rng.standard_normal((m + 1, m)), -1)
    rho = 2.5
    gls = O.GivensLS(m, rho)
    e1 = np.zeros(m + 1)
    e1[0] = rho
    for c in range(m):
        gres = gls.add_column(c, H[: c + 2, c])
        k = c + 1
        y_ref = np.linalg.lstsq(H[: k + 1, :k], e1[: k + 1], rcond=None)[0]
        y = gls.solve(k)
        assert np.allclose(y, y_ref, rtol=1e-11, atol=1e-12)
        assert gres == pytest.approx(np.linalg.norm(e1[: k + 1] - H[: k + 1, :k] @ y), rel=1e-10)


def test_back_substitution_against_library_solve():
    rng = np.random.default_rng(4)
    R = np.triu(rng.standard_normal((9, 9))) + 5 * np.eye(9)
    g = rng.standard_normal(9)
    assert np.allclose(O.back_substitution(R, g), np.linalg.solve(R, g), rtol=1e-13)


def _near_orthogonal(n, k, noise, seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.standard_normal((n, k)))
    q = q + noise * rng.standard_normal((n, k))
    return q / np.linalg.norm(q, axis=0)      # unit columns: Q^T Q = I + L + L^T


def test_projector_identities_exact_algebra():
    """Q^T u = N M^{-1} Q^T a and Q^T w = (N M^{-1})^2 Q^T a (Section 2)."""
    n, k = 200, 12
    Q = _near_orthogonal(n, k, 1e-3, 5)
    a = np.random.default_rng(6).standard_normal(n)
    L = O.strictly_lower_gram(Q)
    assert np.allclose(Q.T @ Q, np.eye(k) + L + L.T, atol=1e-14)
    M = np.eye(k) + L
    N = -L.T
    NMinv = N @ np.linalg.inv(M)
    u, r1 = O.gs_project(Q, L, a, sweeps=1)
    w, r13 = O.gs_project(Q, L, a, sweeps=2)
    qa = Q.T @ a
    lhs_u, rhs_u = Q.T @ u, NMinv @ qa
    lhs_w, rhs_w = Q.T @ w, NMinv @ NMinv @ qa
    assert np.linalg.norm(lhs_u - rhs_u) <= 1e-9 * np.linalg.norm(rhs_u)
    assert np.linalg.norm(lhs_w - rhs_w) <= 1e-6 * np.linalg.norm(rhs_w) + 1e-15 * np.linalg.norm(a)
    # the second sweep shrinks the component in range(Q) by another factor ~ ||N M^{-1}||
    assert np.linalg.norm(Q.T @ w) < 1e-2 * np.linalg.norm(Q.T @ u)
    # accumulated coefficient: r1 + r3 = (I + M^{-1} N) r1  (eq:recur)
    assert np.allclose(r13, (np.eye(k) + np.linalg.solve(M, N)) @ r1, rtol=1e-12, atol=1e-14)
    # one sweep is the inverse compact WY projector I - Q (I+L)^{-1} Q^T (eq:correct)
    assert np.allclose(u, a - Q @ np.linalg.solve(M, qa), atol=1e-13)


def test_projector_two_sweeps_matches_T2():
    """T2 = T1 - T1 L^T T1 is the two-sweep correction matrix (Section 2)."""
    n, k = 150, 9
    Q = _near_orthogonal(n, k, 1e-3, 7)
    a = np.random.default_rng(8).standard_normal(n)
    L = O.strictly_lower_gram(Q)
    T1 = np.linalg.inv(np.eye(k) + L)
    T2 = T1 - T1 @ L.T @ T1
    w, r = O.gs_project(Q, L, a, sweeps=2)
    assert np.allclose(r, T2 @ (Q.T @ a), rtol=1e-11, atol=1e-14)
    assert np.allclose(w, a - Q @ T2 @ Q.T @ a, atol=1e-13)
    # T2 is symmetric to first order: its antisymmetric part is O(||L||^2)
    assert np.linalg.norm(T2 - T2.T) < 10 * np.linalg.norm(L) ** 2


def test_departure_from_normality_identity():
    """dep^2(I + L) = ||L||_F^2 (eq:LOO)."""
    rng = np.random.default_rng(9)
    L = np.tril(rng.standard_normal((15, 15)) * 0.01, -1)
    assert D.departure_from_normality(np.eye(15) + L) == pytest.approx(np.linalg.norm(L, "fro"), rel=1e-6)


def test_paige_S_identity():
    """I - S = (I + L^T)^{-1} with S = (I + L^T)^{-1} L^T (Section 1)."""
    V = _near_orthogonal(80, 10, 1e-2, 10)
    L = np.tril(V.T @ V, -1)
    S = D.paige_S(V)
    assert np.allclose(np.eye(10) - S, np.linalg.inv(np.eye(10) + L.T), atol=1e-13)


def test_norm2_estimate_and_backward_error():
    a = W.convdiff2d(12, 5.0)
    op = O.as_operator(a)
    exact = D.norm2(op)
    est = D.norm2_estimate(op, a.n, iters=400)
    assert est <= exact * (1 + 1e-12)
    assert est == pytest.approx(exact, rel=1e-3)
    d = a.to_dense()
    b = W.rhs_normal(a.n, 1)
    x = np.linalg.solve(d, b)
    assert D.backward_error(op, b, x, exact) < 1e-15


# ---- normwise backward error (Section 1, eq:nrbe) --------------------------

def _rigal_gaches_perturbation(A, b, x, beta, anorm):
    """The perturbations that attain beta: dA = beta ||A|| (r/||r||)(x/||x||)^T,
    db = -beta ||b|| r/||r||, with r = b - A x (Rigal and Gaches)."""
    r = b - A @ x
    rn, xn, bn = np.linalg.norm(r), np.linalg.norm(x), np.linalg.norm(b)
    dA = beta * anorm * np.outer(r / rn, x / xn)
    db = -beta * bn * r / rn
    return dA, db


def _backward_error_cases():
    rng = np.random.default_rng(21)
    out = []
    a = W.convdiff2d(7, 3.0)
    out.append(a.to_dense())
    out.append(rng.standard_normal((9, 9)) + 4 * np.eye(9))
    out.append(W.walker(10, 2000.0))
    cases = []
    for A in out:
        n = A.shape[0]
        b = rng.standard_normal(n)
        # an approximate solution with a residual well above rounding
        x = np.linalg.solve(A, b) + 1e-3 * rng.standard_normal(n)
        cases.append((A, b, x))
    return cases


@pytest.mark.parametrize("case", range(3))
def test_backward_error_rigal_gaches_construction(case):
    """beta is attained: (A + dA) x = b + db with ||dA||_2 = beta ||A||_2 and
    ||db|| = beta ||b|| (the optimal perturbations of Rigal and Gaches)."""
    A, b, x = _backward_error_cases()[case]
    op = O.DenseOperator(A)
    anorm = float(np.linalg.norm(A, 2))
    beta = D.backward_error(op, b, x, anorm)
    assert beta > 1e-8                       # far from rounding: the test can see the formula
    dA, db = _rigal_gaches_perturbation(A, b, x, beta, anorm)
    scale = anorm * np.linalg.norm(x) + np.linalg.norm(b)
    assert np.linalg.norm((A + dA) @ x - (b + db)) <= 1e-14 * scale
    assert np.linalg.norm(dA, 2) == pytest.approx(beta * anorm, rel=1e-12)
    assert np.linalg.norm(db) == pytest.approx(beta * np.linalg.norm(b), rel=1e-12)
    # no smaller perturbation solves the system: for any (E, f) with
    # (A + E) x = b + f, max(||E||/||A||, ||f||/||b||) >= beta
    rng = np.random.default_rng(case)
    for _ in range(20):
        E = rng.standard_normal(A.shape) * beta * anorm * rng.uniform(0.1, 2.0)
        f = (A + E) @ x - b
        assert max(np.linalg.norm(E, 2) / anorm, np.linalg.norm(f) / np.linalg.norm(b)) >= beta * (1 - 1e-12)


def test_backward_error_hand_computed_2x2():
    """A = diag(2, 1), b = (3, 4), x = (1.5, 2): A x = (3, 2), r = (0, 2),
    ||r|| = 2, ||b|| = 5, ||A||_2 = 2, ||x|| = 2.5, so beta = 2 / (5 + 2 * 2.5) = 0.2."""
    A = np.diag([2.0, 1.0])
    b = np.array([3.0, 4.0])
    x = np.array([1.5, 2.0])
    assert D.backward_error(O.DenseOperator(A), b, x, 2.0) == pytest.approx(0.2, rel=1e-15)
    # the attaining perturbation by hand: dA = 0.4 e2 (0.6, 0.8), db = (0, -1)
    dA, db = _rigal_gaches_perturbation(A, b, x, 0.2, 2.0)
    assert np.allclose(dA, [[0.0, 0.0], [0.24, 0.32]], atol=1e-15)
    assert np.allclose(db, [0.0, -1.0], atol=1e-15)
    assert np.allclose((A + dA) @ x, b + db, atol=1e-15)


# ---- Gauss-Seidel iteration matrix M^{-1} N (Section 2) ---------------------

def test_gs_spectral_radius_closed_form_2x2():
    """L = [[0, 0], [l, 0]]: -(I + L)^{-1} L^T = [[0, -l], [0, l^2]], eigenvalues 0 and l^2."""
    for ell in (0.0, 1e-8, 0.3, -0.7, 0.999):
        L = np.array([[0.0, 0.0], [ell, 0.0]])
        assert D.gs_spectral_radius(L) == pytest.approx(ell * ell, rel=1e-14, abs=1e-300)


def test_gs_spectral_radius_young_tridiagonal():
    """For a consistently ordered (tridiagonal) I + L + L^T, the Gauss-Seidel
    radius is the square of the Jacobi radius, rho(L + L^T)^2 (Young)."""
    rng = np.random.default_rng(22)
    for k in (3, 6, 11):
        L = np.diag(rng.uniform(-0.45, 0.45, k - 1), -1)
        rho_j = float(np.max(np.abs(np.linalg.eigvalsh(L + L.T))))
        assert D.gs_spectral_radius(L) == pytest.approx(rho_j ** 2, rel=1e-10)
        assert D.gs_spectral_radius(L) < 1.0          # I + L + L^T is positive definite here


def test_gs_spectral_radius_small_for_near_orthogonal_basis():
    """V^T V = I + L + L^T with ||L|| small: the radius is below ||L||_2 ||L^T||_2 / (1 - ||L||)
    (a norm bound on ||(I + L)^{-1} L^T||) and far below 1."""
    V = _near_orthogonal(100, 8, 1e-3, 23)
    L = np.tril(V.T @ V, -1)
    nl = np.linalg.norm(L, 2)
    rho = D.gs_spectral_radius(L)
    assert rho <= nl / (1 - nl) * (1 + 1e-12)
    assert rho < 1e-2


def test_gs_spectral_radius_is_the_sweep_contraction_rate():
    """The radius is the asymptotic error contraction per Gauss-Seidel sweep on
    (I + L + L^T) y = c, y <- (I + L)^{-1} (c - L^T y), measured by running the
    sweeps (a dense, non-tridiagonal L)."""
    V = _near_orthogonal(12, 10, 0.12, 24)
    L = np.tril(V.T @ V, -1)
    k = L.shape[0]
    A = np.eye(k) + L + L.T
    c = np.random.default_rng(25).standard_normal(k)
    y_star = np.linalg.solve(A, c)
    y = np.zeros(k)
    errs = []
    for _ in range(40):
        y = np.linalg.solve(np.eye(k) + L, c - L.T @ y)
        errs.append(np.linalg.norm(y - y_star))
    k0, k1 = 8, 38          # before the error reaches rounding level (rho^38 ~ 1e-10)
    rate = (errs[k1] / errs[k0]) ** (1.0 / (k1 - k0))
    rho = D.gs_spectral_radius(L)
    assert 0.05 < rho < 0.9
    assert rate == pytest.approx(rho, rel=2e-2)
