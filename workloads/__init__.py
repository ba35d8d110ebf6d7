"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the bench.

This module builds matrices and right-hand sides only.  It holds none of the
solver's arithmetic (no Arnoldi step, no projection, no least squares), so both
the CPU oracle and the HIP path can draw their inputs from it without sharing
any part of the method.

Matrices come in two forms:

* ``Csr`` -- compressed sparse rows with int32 ``row_ptr``/``col_idx`` and
  float64 ``vals``; columns are sorted ascending inside each row.
* dense float64 arrays in C (row-major) order.

Generators
----------
convdiff2d / convdiff3d
    Steady convection-diffusion ``-lap(u) + Pe * w . grad(u)`` on the unit
    square / cube, zero Dirichlet boundary eliminated, ``N`` interior points
    per side, ``h = 1/(N+1)``, lexicographic numbering ``i + N*j (+ N*N*k)``,
    first-order upwind convection for a wind ``w = (1,1)`` / ``(1,1,1)``, and
    the whole operator scaled by ``h**2``.  Diagonal ``2d + d*Pe*h``, upwind
    (west/south/down) neighbours ``-1 - Pe*h``, downwind neighbours ``-1``.
dense_nonnormal
    ``A0 = U diag(s) W^T`` with Haar-random orthogonal ``U, W`` (QR of a
    standard normal matrix with the signs of ``diag(R)`` made positive),
    ``s`` log-spaced from 1 to ``s_min``; then ``A = A0 + upper_scale *
    triu(A0, 1)``.
simoncini_diag, walker, embree_bidiag, helmert
    The small test matrices of the numerical-results section (ill-conditioned
    diagonal, Walker's non-normal matrix, Embree's defective bidiagonal, the
    textbook Helmert matrix).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class Csr:
    """A square CSR matrix: int32 indices, float64 values, sorted columns."""

    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    vals: np.ndarray

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])

    def to_dense(self) -> np.ndarray:
        if self.n > 8192:
            raise ValueError("to_dense is for small matrices only")
        a = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.row_ptr))
        a[rows, self.col_idx] = self.vals
        return a


def csr_from_dense(a: np.ndarray, drop_zeros: bool = True) -> Csr:
    """CSR copy of a dense square matrix (exact zeros dropped if asked)."""
    a = np.asarray(a, dtype=np.float64)
    n = a.shape[0]
    if a.shape != (n, n):
        raise ValueError("square matrix expected")
    mask = a != 0.0 if drop_zeros else np.ones_like(a, dtype=bool)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    rows, cols = np.nonzero(mask)
    return Csr(n, row_ptr.astype(np.int32), cols.astype(np.int32), a[rows, cols].copy())


def _stencil_csr(n: int, offsets, valid, coeffs) -> Csr:
    """Assemble CSR from per-row stencil entries.

    ``offsets`` ascend, so flattening the (row, entry) table row by row keeps
    each row's columns sorted.
    """
    rows = np.arange(n, dtype=np.int64)
    cols = rows[:, None] + np.asarray(offsets, dtype=np.int64)[None, :]
    mask = np.stack(valid, axis=1)
    vals = np.broadcast_to(np.asarray(coeffs, dtype=np.float64)[None, :], mask.shape)
    counts = mask.sum(axis=1)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("nnz exceeds int32 indexing")
    return Csr(n, row_ptr.astype(np.int32), cols[mask].astype(np.int32),
               np.ascontiguousarray(vals[mask]))


def convdiff2d(N: int, pe: float) -> Csr:
    """5-point upwind convection-diffusion on an N x N interior grid, wind (1,1)."""
    n = N * N
    h = 1.0 / (N + 1)
    idx = np.arange(n, dtype=np.int64)
    i, j = idx % N, idx // N
    up = -1.0 - pe * h
    offsets = (-N, -1, 0, 1, N)
    valid = (j > 0, i > 0, np.ones(n, bool), i < N - 1, j < N - 1)
    coeffs = (up, up, 4.0 + 2.0 * pe * h, -1.0, -1.0)
    return _stencil_csr(n, offsets, valid, coeffs)


def convdiff3d(N: int, pe: float) -> Csr:
    """7-point upwind convection-diffusion on an N^3 interior grid, wind (1,1,1)."""
    n = N * N * N
    h = 1.0 / (N + 1)
    idx = np.arange(n, dtype=np.int64)
    i, j, k = idx % N, (idx // N) % N, idx // (N * N)
    up = -1.0 - pe * h
    NN = N * N
    offsets = (-NN, -N, -1, 0, 1, N, NN)
    valid = (k > 0, j > 0, i > 0, np.ones(n, bool), i < N - 1, j < N - 1, k < N - 1)
    coeffs = (up, up, up, 6.0 + 3.0 * pe * h, -1.0, -1.0, -1.0)
    return _stencil_csr(n, offsets, valid, coeffs)


def haar_orthogonal(n: int, seed: int) -> np.ndarray:
    """Q factor of a seeded standard normal matrix, signs fixed so diag(R) > 0."""
    g = np.random.default_rng(seed).standard_normal((n, n))
    q, r = np.linalg.qr(g)
    q *= np.sign(np.diag(r))[None, :]
    return q


def dense_nonnormal(n: int, s_min: float = 1e-10, upper_scale: float = 1e2,
                    seed_u: int = 1, seed_w: int = 2) -> np.ndarray:
    """Highly non-normal dense matrix U diag(s) W^T plus a scaled strict upper part."""
    u = haar_orthogonal(n, seed_u)
    w = haar_orthogonal(n, seed_w)
    s = np.logspace(0.0, np.log10(s_min), n)
    a0 = (u * s[None, :]) @ w.T
    a = a0 + upper_scale * np.triu(a0, 1)
    return np.ascontiguousarray(a)


def simoncini_diag(n: int = 100) -> np.ndarray:
    """diag(1e-4, 2, 3, ..., n): the ill-conditioned diagonal test matrix."""
    d = np.arange(1, n + 1, dtype=np.float64)
    d[0] = 1e-4
    return np.diag(d)


def walker(n: int = 10, alpha: float = 2000.0) -> np.ndarray:
    """diag(1..n) with alpha in the top-right corner (Walker's non-normal matrix)."""
    a = np.diag(np.arange(1, n + 1, dtype=np.float64))
    a[0, n - 1] = alpha
    return a


def embree_bidiag(n: int = 100, delta: float = 0.1) -> np.ndarray:
    """Unit upper bidiagonal matrix with delta on the superdiagonal (defective)."""
    return np.eye(n) + delta * np.eye(n, k=1)


def helmert(n: int) -> np.ndarray:
    """Textbook orthogonal Helmert matrix: first row constant, then contrast rows."""
    a = np.zeros((n, n))
    a[0, :] = 1.0 / np.sqrt(n)
    for k in range(2, n + 1):
        c = 1.0 / np.sqrt(k * (k - 1))
        a[k - 1, : k - 1] = c
        a[k - 1, k - 1] = -(k - 1) * c
    return a


def clustered_spectrum(n: int = 120, centers=(1.0, 2.0, 3.0, 5.0, 8.0, 13.0),
                       spread: float = 1e-7, seed: int = 0) -> np.ndarray:
    """Symmetric matrix Q diag(d) Q^T whose eigenvalues form tight clusters.

    With ``len(centers)`` clusters of width ~``spread`` the Krylov space almost
    becomes invariant after ``len(centers)`` steps, so the Arnoldi process
    passes close to a breakdown (a tiny subdiagonal) and then continues.
    """
    rng = np.random.default_rng(seed)
    c = np.asarray(centers, dtype=np.float64)
    d = np.repeat(c, n // c.size)
    d = np.concatenate([d, np.full(n - d.size, c[-1])])
    d = d + spread * rng.standard_normal(n)
    q = haar_orthogonal(n, seed + 100)
    return (q * d[None, :]) @ q.T


def rhs_normal(n: int, seed: int = 0) -> np.ndarray:
    """b ~ N(0, 1), drawn with numpy's PCG64 generator."""
    return np.random.default_rng(seed).standard_normal(n)


def random_wellcond(n: int, seed: int) -> np.ndarray:
    """Random non-symmetric matrix with a dominant diagonal (well conditioned)."""
    rng = np.random.default_rng(seed)
    return np.eye(n) * 4.0 + rng.standard_normal((n, n)) / np.sqrt(n)


# ---------------------------------------------------------------------------
# Named workloads (sizes and solver settings of the benchmark suite)
# ---------------------------------------------------------------------------

@dataclass(frozen=True)
class Workload:
    name: str
    restart: int
    tol: float
    gs_iters: int


CONVDIFF2D_32 = Workload("convdiff2d_N32_Pe10", restart=50, tol=1e-12, gs_iters=2)
CONVDIFF3D_128 = Workload("convdiff3d_N128_Pe50", restart=60, tol=1e-10, gs_iters=2)
DENSE_NONNORMAL_4096 = Workload("dense_nonnormal_n4096", restart=200, tol=0.0, gs_iters=2)
CONVDIFF3D_96 = Workload("convdiff3d_N96_Pe50", restart=40, tol=1e-10, gs_iters=2)


def make_convdiff2d_32():
    """2D 5-point upwind, 32x32 grid (n=1024), Pe 10, b ~ N(0,1) seed 0."""
    a = convdiff2d(32, 10.0)
    return a, rhs_normal(a.n, 0)


def make_convdiff3d(N: int = 128, pe: float = 50.0):
    """3D 7-point upwind, N^3 grid, wind (1,1,1)*Pe, b ~ N(0,1) seed 0."""
    a = convdiff3d(N, pe)
    return a, rhs_normal(a.n, 0)


def make_dense_nonnormal(n: int = 4096):
    """Dense non-normal matrix (s from 1 to 1e-10, upper part x1e2), b seed 0."""
    a = dense_nonnormal(n)
    return a, rhs_normal(n, 0)


@dataclass(frozen=True)
class Request:
    """One request of a serving trace: a 2D convection-diffusion system and
    the time (seconds after the start) at which it arrives."""
    rid: int
    side: int
    pe: float
    arrival: float
    a: Csr
    b: np.ndarray


def serving_trace(count: int = 512, seed: int = 7, side_lo: int = 32, side_hi: int = 512,
                  pe_lo: float = 1.0, pe_hi: float = 100.0, rate: float = 200.0):
    """A seeded trace of independent solves of uneven size: grid sides uniform
    on the integers [side_lo, side_hi] (n = side^2), Pe uniform on [pe_lo,
    pe_hi], Poisson arrivals at `rate` per second (exponential gaps), and
    b ~ N(0, 1) seeded by the request id."""
    rng = np.random.default_rng(seed)
    sides = rng.integers(side_lo, side_hi + 1, size=count)
    pes = rng.uniform(pe_lo, pe_hi, size=count)
    arrivals = np.cumsum(rng.exponential(1.0 / rate, size=count)) if rate > 0 else np.zeros(count)
    out = []
    for i in range(count):
        a = convdiff2d(int(sides[i]), float(pes[i]))
        out.append(Request(i, int(sides[i]), float(pes[i]), float(arrivals[i]), a,
                           rhs_normal(a.n, 1000 + i)))
    return out


SERVING = Workload("serving_convdiff2d_side32-512_Pe1-100_poisson200", restart=50, tol=1e-12,
                   gs_iters=2)
