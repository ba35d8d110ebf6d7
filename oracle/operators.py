"""The operator ``A`` of ``Ax = b`` (Section 1: a real n x n matrix).

CsrOperator.matvec is the plain definition ``y_i = sum_k vals[k] * x[col[k]]``
over the entries ``k`` of row ``i``, summed in storage order.  DenseOperator
uses numpy's matrix-vector product (a library primitive).

Pinned by: tests/test_oracle_primitives.py (CSR product against the dense
product of the same matrix; transpose product against the dense transpose).
"""
from __future__ import annotations

import numpy as np


class CsrOperator:
    """y = A x for A in CSR form (int32 indices, float64 values)."""

    def __init__(self, row_ptr, col_idx, vals):
        self.row_ptr = np.asarray(row_ptr)
        self.col_idx = np.asarray(col_idx)
        self.vals = np.asarray(vals, dtype=np.float64)
        self.n = self.row_ptr.size - 1
        # row index of every stored entry, in storage order
        self._rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))

    @property
    def shape(self):
        return (self.n, self.n)

    def matvec(self, x: np.ndarray) -> np.ndarray:
        prod = self.vals * x[self.col_idx]
        return np.bincount(self._rows, weights=prod, minlength=self.n)

    def rmatvec(self, x: np.ndarray) -> np.ndarray:
        """y = A^T x (used only by the power-iteration norm estimate)."""
        prod = self.vals * x[self._rows]
        return np.bincount(self.col_idx, weights=prod, minlength=self.n)

    def to_dense(self) -> np.ndarray:
        a = np.zeros((self.n, self.n))
        a[self._rows, self.col_idx] = self.vals
        return a


class DenseOperator:
    """y = A x for a dense float64 matrix."""

    def __init__(self, a):
        self.a = np.asarray(a, dtype=np.float64)
        self.n = self.a.shape[0]

    @property
    def shape(self):
        return self.a.shape

    def matvec(self, x: np.ndarray) -> np.ndarray:
        return self.a @ x

    def rmatvec(self, x: np.ndarray) -> np.ndarray:
        return self.a.T @ x

    def to_dense(self) -> np.ndarray:
        return self.a


def as_operator(a):
    """Wrap a dense array, a workloads.Csr, or an operator."""
    if hasattr(a, "matvec"):
        return a
    if hasattr(a, "row_ptr"):
        return CsrOperator(a.row_ptr, a.col_idx, a.vals)
    return DenseOperator(a)
