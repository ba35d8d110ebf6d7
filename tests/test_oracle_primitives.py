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
