"""The GMRES least-squares problem min_y || rho e1 - H y || (eq:llse).

The Hessenberg matrix is reduced column by column with Givens rotations (the
paper does not fix a method; this is the standard one).  For a finished
column ``h`` (rows 0..c+1) the stored rotations ``i < c`` are applied in order
as ``[h_i; h_{i+1}] <- [cs_i h_i + sn_i h_{i+1}; -sn_i h_i + cs_i h_{i+1}]``,
then a new rotation ``d = hypot(h_c, h_{c+1})``, ``cs = h_c/d``,
``sn = h_{c+1}/d`` zeroes the subdiagonal and updates the rotated right-hand
side ``g``: ``g_{c+1} = -sn g_c``, ``g_c = cs g_c``.  ``|g_{c+1}|`` is the
Arnoldi residual norm after ``c+1`` steps.  ``y`` solves the upper triangular
``R y = g`` by back substitution.

Pinned by: tests/test_oracle_primitives.py -- ``y`` against numpy's lstsq of
the unrotated ``H``; ``|g_{k}|`` against the explicit ``||rho e1 - H y||``.
"""
from __future__ import annotations

import math

import numpy as np


class GivensLS:
    """Incremental Givens QR of H_{k+1,k} with right-hand side rho e1."""

    def __init__(self, m: int, rho: float):
        self.R = np.zeros((m + 1, m))
        self.cs = np.zeros(m)
        self.sn = np.zeros(m)
        self.g = np.zeros(m + 1)
        self.g[0] = rho
        self.ncols = 0

    def add_column(self, c: int, h: np.ndarray) -> float:
        """Rotate finished column ``c`` (entries 0..c+1); return |g_{c+1}|."""
        if c != self.ncols:
            raise ValueError("columns must be added in order")
        col = np.array(h[: c + 2], dtype=np.float64, copy=True)
        for i in range(c):
            a, b = col[i], col[i + 1]
            col[i] = self.cs[i] * a + self.sn[i] * b
            col[i + 1] = -self.sn[i] * a + self.cs[i] * b
        d = math.hypot(col[c], col[c + 1])
        if d == 0.0:
            cs, sn = 1.0, 0.0
        else:
            cs, sn = col[c] / d, col[c + 1] / d
        self.cs[c], self.sn[c] = cs, sn
        col[c], col[c + 1] = d, 0.0
        self.R[: c + 2, c] = col
        self.g[c + 1] = -sn * self.g[c]
        self.g[c] = cs * self.g[c]
        self.ncols = c + 1
        return abs(self.g[c + 1])

    def solve(self, k: int) -> np.ndarray:
        """y minimising the first k columns' least-squares problem."""
        return back_substitution(self.R[:k, :k], self.g[:k])


def back_substitution(R: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Solve R y = g for upper triangular R, last row first."""
    k = g.shape[0]
    y = np.zeros(k)
    for i in range(k - 1, -1, -1):
        y[i] = (g[i] - R[i, i + 1:k] @ y[i + 1:k]) / R[i, i]
    return y
