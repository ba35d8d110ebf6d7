"""Quality measures the paper reports (Sections 1, 4 and 5).

* ``backward_error``: the norm-wise relative backward error (eq:nrbe).
* ``orthogonality_loss``: ``||I - V^T V||_F``.
* ``arnoldi_relation_residual``: ``||A V_J - V_{J+1} H||_F / ||A||_2``.
* ``departure_from_normality``: Henrici's ``sqrt(||X||_F^2 - sum |lambda|^2)``;
  for ``I + L`` it equals ``||L||_F`` (eq:LOO).
* ``paige_S``: ``S = (I + L^T)^{-1} L^T`` with ``L`` the strictly lower part
  of ``V^T V``; stagnation of MGS-GMRES goes with ``||S||_2 -> 1``.
* ``gs_spectral_radius``: spectral radius of ``M^{-1} N = -(I + L)^{-1} L^T``.
* ``norm2_estimate``: power iteration on ``A^T A`` (a lower bound on ||A||_2)
  for operators too large for a dense SVD.

Pinned by tests/test_oracle_primitives.py:

* departure identity against the eigenvalue definition;
* power estimate against the exact 2-norm;
* backward error: the perturbations of Rigal and Gaches built from the
  returned value solve (A + dA) x = b + db exactly with ||dA|| = beta ||A||
  and ||db|| = beta ||b||, no random perturbation that solves it is smaller,
  and a hand-computed 2 x 2 case (beta = 0.2);
* Gauss-Seidel radius: the 2 x 2 closed form l^2, Young's relation
  rho_GS = rho_Jacobi^2 for tridiagonal L, and the measured contraction rate
  of the sweeps on a dense L.

tests/test_oracle_mutations.py plants wrong denominators and wrong iteration
matrices and checks that these pins catch each one.
"""
from __future__ import annotations

import math

import numpy as np


def backward_error(op, b: np.ndarray, x: np.ndarray, anorm: float) -> float:
    r = b - op.matvec(x)
    return math.sqrt(r @ r) / (math.sqrt(b @ b) + anorm * math.sqrt(x @ x))


def orthogonality_loss(V: np.ndarray) -> float:
    k = V.shape[1]
    return float(np.linalg.norm(np.eye(k) - V.T @ V, "fro"))


def arnoldi_relation_residual(op, V: np.ndarray, H: np.ndarray, anorm: float) -> float:
    J = H.shape[1]
    AV = np.stack([op.matvec(V[:, c]) for c in range(J)], axis=1)
    return float(np.linalg.norm(AV - V[:, : J + 1] @ H, "fro")) / anorm


def departure_from_normality(X: np.ndarray) -> float:
    lam = np.linalg.eigvals(X)
    val = np.linalg.norm(X, "fro") ** 2 - float(np.sum(np.abs(lam) ** 2))
    return math.sqrt(max(val, 0.0))


def paige_S(V: np.ndarray) -> np.ndarray:
    L = np.tril(V.T @ V, -1)
    k = L.shape[0]
    return np.linalg.solve(np.eye(k) + L.T, L.T)


def gs_spectral_radius(L: np.ndarray) -> float:
    k = L.shape[0]
    it = -np.linalg.solve(np.eye(k) + L, L.T)
    return float(np.max(np.abs(np.linalg.eigvals(it)))) if k else 0.0


def norm2_estimate(op, n: int, iters: int = 200, seed: int = 12345) -> float:
    x = np.random.default_rng(seed).standard_normal(n)
    x /= math.sqrt(x @ x)
    est = 0.0
    for _ in range(iters):
        y = op.rmatvec(op.matvec(x))
        ny = math.sqrt(y @ y)
        if ny == 0.0:
            return 0.0
        est = math.sqrt(ny)
        x = y / ny
    return est


def norm2(op) -> float:
    """Exact ||A||_2 for small dense-able operators."""
    return float(np.linalg.norm(op.to_dense(), 2))
