"""GPU parity of each hot-path step kernel against the oracle's step functions,
called through the C ABI on seeded inputs with ragged, multi-block sizes."""
import numpy as np
import pytest

import oracle as O
import oracle.arnoldi as OA
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ctx_csr(a):
    from paper_2205_07805_amd import igs
    return igs.igs_create(a.n, a.nnz, a.row_ptr, a.col_idx, a.vals, 0, None)


def _random_csr(n, avg, seed, empty_rows=()):
    rng = np.random.default_rng(seed)
    counts = rng.poisson(avg, n)
    counts[list(empty_rows)] = 0
    counts = np.minimum(counts, n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    cols = np.concatenate([np.sort(rng.choice(n, c, replace=False)) for c in counts]).astype(np.int32)
    vals = rng.standard_normal(cols.size)
    return W.Csr(n, row_ptr.astype(np.int32), cols, vals)


CSR_CASES = {
    "convdiff3d_17": lambda: W.convdiff3d(17, 50.0),
    "convdiff3d_16": lambda: W.convdiff3d(16, 50.0),
    "convdiff2d_31": lambda: W.convdiff2d(31, 10.0),
    "convdiff2d_32": lambda: W.convdiff2d(32, 10.0),
    "random_short_rows_empty": lambda: _random_csr(3001, 3.0, 1, empty_rows=(0, 17, 3000)),
    "random_two_lanes": lambda: _random_csr(2049, 1.6, 5, empty_rows=(5,)),
    "diagonal_one_lane": lambda: W.csr_from_dense(np.diag(np.arange(1.0, 40.0))),
    "random_long_rows": lambda: _random_csr(1500, 40.0, 2),
    "single_row": lambda: W.csr_from_dense(np.array([[2.5]])),
}


@pytest.mark.parametrize("case", sorted(CSR_CASES))
def test_spmv_csr_matches_oracle(torch, case):
    from paper_2205_07805_amd import igs
    a = CSR_CASES[case]()
    print(f"spmv csr case={case} n={a.n} nnz={a.nnz}", flush=True)
    ctx = _ctx_csr(a)
    try:
        u = W.rhs_normal(a.n, 7)
        ud = torch.tensor(u, device="cuda")
        zd = torch.empty_like(ud)
        igs.igs_kernel_spmv(ctx, ud, zd)
        ref = O.as_operator(a).matvec(u)
        scale = np.abs(a.vals).max() * np.abs(u).max() * max(1, np.diff(a.row_ptr).max())
        np.testing.assert_allclose(zd.cpu().numpy(), ref, rtol=0, atol=1e-14 * scale)
    finally:
        igs.igs_destroy(ctx)


@pytest.mark.parametrize("variant", ["valu", "mfma", "lds"])
@pytest.mark.parametrize("n", [1, 63, 1000, 1001, 4096])
def test_gemv_dense_matches_oracle(torch, n, variant):
    """The dense kernels (one wave per row; the matrix cores; the vector in
    shared memory) against the
    oracle's product: one row, a partial 16-row tile and 32-column step,
    several tiles with a ragged tail, and the dense workload's size."""
    from paper_2205_07805_amd import igs
    a = W.random_wellcond(n, 3) if n > 1 else np.array([[3.0]])
    print(f"gemv dense n={n} variant={variant}", flush=True)
    ctx = igs.igs_create_dense(n, a, n, 0, None)
    try:
        igs.igs_dense_variant(ctx, {"valu": igs.IGS_DENSE_VALU, "mfma": igs.IGS_DENSE_MFMA,
                                    "lds": igs.IGS_DENSE_LDS}[variant])
        u = W.rhs_normal(n, 8)
        ud = torch.tensor(u, device="cuda")
        zd = torch.empty_like(ud)
        igs.igs_kernel_spmv(ctx, ud, zd)
        ref = O.as_operator(a).matvec(u)
        np.testing.assert_allclose(zd.cpu().numpy(), ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    finally:
        igs.igs_destroy(ctx)


def test_dense_variant_rejects_csr_and_unknown(torch):
    from paper_2205_07805_amd import igs
    ctx = _ctx_csr(W.convdiff2d(8, 1.0))
    try:
        with pytest.raises(igs.IgsError):
            igs.igs_dense_variant(ctx, igs.IGS_DENSE_MFMA)
    finally:
        igs.igs_destroy(ctx)
    ctx = igs.igs_create_dense(4, np.eye(4), 4, 0, None)
    try:
        with pytest.raises(igs.IgsError):
            igs.igs_dense_variant(ctx, 7)
    finally:
        igs.igs_destroy(ctx)


_CTX = {}


def ctx_of_size(n):
    """A context whose n matches the step-kernel buffers (the operator is unused)."""
    if n not in _CTX:
        _CTX[n] = _ctx_csr(W.csr_from_dense(np.eye(1)) if n == 1 else
                           W.Csr(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32),
                                 np.ones(n)))
    return _CTX[n]


@pytest.fixture(scope="module", autouse=True)
def _release_contexts():
    yield
    from paper_2205_07805_amd import igs
    for ctx in _CTX.values():
        igs.igs_destroy(ctx)
    _CTX.clear()


def _basis(torch, n, ncols, seed, ldv=None):
    """Random near-orthonormal columns (as a Krylov basis would be) plus an
    arbitrary last column, stored column-major with leading dimension ldv."""
    ldv = ldv or n
    rng = np.random.default_rng(seed)
    Vt = rng.standard_normal((ncols, n)) / np.sqrt(n)
    host = np.zeros((ncols, ldv))
    host[:, :n] = Vt
    return Vt, torch.tensor(host, device="cuda")


@pytest.mark.parametrize("pad", [13, 64], ids=["ld_odd", "ld_even"])
@pytest.mark.parametrize("j", [0, 1, 5, 8, 15, 16, 17, 31, 60, 127, 200])
@pytest.mark.parametrize("n", [100_003, 4_099])
def test_reduce_matches_oracle(torch, n, j, pad):
    """Odd leading dimension: 8-byte path; even: 16-byte row-pair path."""
    from paper_2205_07805_amd import igs
    print(f"reduce n={n} j={j} ldv=n+{pad}", flush=True)
    ctx_small = ctx_of_size(n)
    ldv = n + pad
    Vt, Vd = _basis(torch, n, j + 1, seed=j + n, ldv=ldv)
    z = W.rhs_normal(n, j)
    zd = torch.tensor(z, device="cuda")
    P = np.zeros(j + 1)
    Q = np.zeros(j + 1)
    igs.igs_kernel_reduce(ctx_small, Vd, ldv, j, zd, P, Q)
    p, alpha, q, beta = OA.one_reduction(Vt[:j], Vt[j], z)
    Pref = np.concatenate([p, [alpha]])
    Qref = np.concatenate([q, [beta]])
    tol_p = 1e-14 * np.sqrt(n) * np.linalg.norm(Vt, axis=1) * np.linalg.norm(Vt[j])
    tol_q = 1e-14 * np.sqrt(n) * np.linalg.norm(Vt, axis=1) * np.linalg.norm(z)
    assert np.all(np.abs(P - Pref) <= tol_p)
    assert np.all(np.abs(Q - Qref) <= tol_q)
    # without z (the tail iteration)
    P2 = np.zeros(j + 1)
    igs.igs_kernel_reduce(ctx_small, Vd, ldv, j, None, P2, None)
    assert np.array_equal(P2, P)


# 300,001 and 600,001 rows take two and four row vectors per thread (the
# tiles then number at least one per CU), with a partial last tile; with
# pad 3 the leading dimension is even and the vector path runs
@pytest.mark.parametrize("n,j", [(100_003, 3), (100_003, 30), (1_048_576, 50)])
def test_reduce_repeated_calls_agree_bit_for_bit(torch, n, j):
    """The blocks of a launch hand their partial sums over with write-through
    stores, a wait before the arrival counter and coherent loads in the last
    block.  Many launches on the same input must all give the same bits (a
    partial sum read before it landed would change them) and match the
    oracle; at 1,048,576 rows the grid has 256 blocks, 32 per counter."""
    from paper_2205_07805_amd import igs
    print(f"repeated reduce n={n} j={j}", flush=True)
    ctx_small = ctx_of_size(n)
    Vt, Vd = _basis(torch, n, j + 1, seed=7 * j + n)
    z = W.rhs_normal(n, 11 + j)
    zd = torch.tensor(z, device="cuda")
    P0 = np.zeros(j + 1)
    Q0 = np.zeros(j + 1)
    igs.igs_kernel_reduce(ctx_small, Vd, n, j, zd, P0, Q0)
    p, alpha, q, beta = OA.one_reduction(Vt[:j], Vt[j], z)
    tol_p = 1e-14 * np.sqrt(n) * np.linalg.norm(Vt, axis=1) * np.linalg.norm(Vt[j])
    tol_q = 1e-14 * np.sqrt(n) * np.linalg.norm(Vt, axis=1) * np.linalg.norm(z)
    assert np.all(np.abs(P0 - np.concatenate([p, [alpha]])) <= tol_p)
    assert np.all(np.abs(Q0 - np.concatenate([q, [beta]])) <= tol_q)
    P = np.zeros(j + 1)
    Q = np.zeros(j + 1)
    for rep in range(40):
        igs.igs_kernel_reduce(ctx_small, Vd, n, j, zd, P, Q)
        assert np.array_equal(P, P0) and np.array_equal(Q, Q0), rep


# n = 1,050,001 with an even leading dimension takes eight row vectors of
# doubles per thread (257 tiles of 4,096 rows, the last one ragged)
@pytest.mark.parametrize("pad", [3, 64], ids=["ld_odd", "ld_even"])
@pytest.mark.parametrize("j", [0, 1, 7, 33, 60])
@pytest.mark.parametrize("n", [100_003, 1_025, 4_096, 300_001, 600_001, 1_050_001])
def test_update_matches_oracle(torch, n, j, pad):
    from paper_2205_07805_amd import igs
    print(f"update n={n} j={j} ldv=n+{pad}", flush=True)
    ctx_small = ctx_of_size(n)
    ldv = n + pad
    Vt, Vd = _basis(torch, n, j + 2, seed=3 * j + n, ldv=ldv)
    rng = np.random.default_rng(j)
    t = rng.standard_normal(j) * 1e-3
    r1 = rng.standard_normal(j + 1)
    gamma = 0.37
    z = W.rhs_normal(n, 100 + j)
    zd = torch.tensor(z, device="cuda")
    igs.igs_kernel_update(ctx_small, Vd, ldv, j, zd, t if j else None, r1, 1.0 / gamma)
    out = Vd.cpu().numpy()
    vj = OA.normalise_after_second_sweep(Vt[:j], Vt[j], t, gamma)
    Vnew = np.vstack([Vt[:j], vj[None, :]])
    un = OA.first_sweep_next(Vnew, z, gamma, r1)
    np.testing.assert_allclose(out[j, :n], vj, rtol=0, atol=1e-13 * np.abs(vj).max())
    np.testing.assert_allclose(out[j + 1, :n], un, rtol=0, atol=1e-13 * np.abs(un).max())
    # untouched: the other columns and the padding
    np.testing.assert_array_equal(out[:j, :n], Vt[:j])
    assert np.all(out[:, n:] == 0.0)


# odd n: one row per thread; even n: two
@pytest.mark.parametrize("case", ["convdiff2d_31", "convdiff3d_17", "convdiff2d_32", "convdiff3d_16"])
def test_ell_form_is_bit_identical_to_csr(torch, case):
    """Short-row operators also keep a column-major ELL form; its product
    must equal the CSR kernel's bit for bit.  A copy of the matrix with four
    explicit zeros appended to one row (9 entries, so no ELL form) runs the
    CSR kernel; every other row must agree exactly, with and without the
    subtracted right-hand side (the residual b - A x of a cycle start)."""
    from paper_2205_07805_amd import Solver, igs
    a = CSR_CASES[case]()
    n = a.n
    rp = a.row_ptr.astype(np.int64)
    r = n // 2
    s0, s1 = rp[r], rp[r + 1]
    used = set(a.col_idx[s0:s1].tolist())
    extra = np.array([c for c in range(n) if c not in used][:4], dtype=np.int32)
    ci2 = np.concatenate([a.col_idx[:s1], extra, a.col_idx[s1:]]).astype(np.int32)
    va2 = np.concatenate([a.vals[:s1], np.zeros(4), a.vals[s1:]])
    rp2 = rp.copy()
    rp2[r + 1:] += 4
    b2 = W.Csr(n, rp2.astype(np.int32), ci2, va2)
    print(f"ELL against CSR {case} n={n}", flush=True)
    ctx_e = _ctx_csr(a)
    ctx_c = _ctx_csr(b2)
    try:
        u = torch.tensor(W.rhs_normal(n, 3), device="cuda")
        ze = torch.empty_like(u)
        zc = torch.empty_like(u)
        igs.igs_kernel_spmv(ctx_e, u, ze)
        igs.igs_kernel_spmv(ctx_c, u, zc)
        mask = np.ones(n, bool)
        mask[r] = False
        assert np.array_equal(ze.cpu().numpy()[mask], zc.cpu().numpy()[mask])
    finally:
        igs.igs_destroy(ctx_e)
        igs.igs_destroy(ctx_c)
    # whole solves (residuals with a nonzero x0 included): the row with the
    # explicit zeros sums the same products, so the solves agree exactly
    b = W.rhs_normal(n, 4)
    x0 = W.rhs_normal(n, 5)
    se, sc = Solver(a), Solver(b2)
    try:
        xe, rce, ie = se.solve(b, x0=x0, restart=20, tol=1e-12)
        xc, rcc, ic = sc.solve(b, x0=x0, restart=20, tol=1e-12)
        assert ie["iters"] == ic["iters"] and np.array_equal(xe.cpu().numpy(), xc.cpu().numpy())
    finally:
        se.close()
        sc.close()
