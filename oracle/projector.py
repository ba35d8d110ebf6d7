"""Gram-Schmidt projection as relaxation on the normal equations (Section 2).

The projection of ``a`` onto the orthogonal complement of range(Q) needs the
solution ``r`` of the normal equations ``Q^T Q r = Q^T a`` (eq:normal).  With
the splitting ``Q^T Q = M - N``, ``M = I + L``, ``N = -L^T`` and ``L`` the
strictly lower part of ``Q^T Q``, one Gauss-Seidel sweep from the zero guess
gives ``r1 = M^{-1} Q^T a`` (the inverse compact WY correction
``T1 = (I + L)^{-1}``, eq:correct) and the projected vector ``u = a - Q r1``
(eq:proj).  A second sweep on the residual equation gives
``r3 = M^{-1} Q^T u`` and ``w = u - Q r3``, with coefficient ``r1 + r3``
(Algorithm 2.1 / eq:recur, eq:proj1).

Pinned by: tests/test_oracle_primitives.py -- forward substitution against a
dense library solve; the exact-algebra identities ``Q^T u = N M^{-1} Q^T a``
and ``Q^T w = (N M^{-1})^2 Q^T a``; ``r1 + r3 = (I + M^{-1} N) r1``.
"""
from __future__ import annotations

import numpy as np


def forward_subst_unit_lower(L: np.ndarray, r: np.ndarray) -> np.ndarray:
    """Solve (I + L) x = r for strictly lower triangular L, row by row."""
    k = r.shape[0]
    x = np.array(r, dtype=np.float64, copy=True)
    for i in range(k):
        x[i] = r[i] - L[i, :i] @ x[:i]
    return x


def strictly_lower_gram(Q: np.ndarray) -> np.ndarray:
    """L with Q^T Q = I + L + L^T (strictly lower part of Q^T Q)."""
    return np.tril(Q.T @ Q, -1)


def gs_project(Q: np.ndarray, L: np.ndarray, a: np.ndarray, sweeps: int):
    """Project ``a`` against the columns of ``Q`` with ``sweeps`` Gauss-Seidel sweeps.

    Returns ``(w, r)`` where ``w`` is the projected vector and ``r`` the
    accumulated coefficient vector (``r1`` or ``r1 + r3``).
    """
    r0 = Q.T @ a
    r1 = forward_subst_unit_lower(L, r0)
    u = a - Q @ r1
    if sweeps == 1:
        return u, r1
    if sweeps != 2:
        raise ValueError("sweeps must be 1 or 2")
    r2 = Q.T @ u
    r3 = forward_subst_unit_lower(L, r2)
    w = u - Q @ r3
    return w, r1 + r3
