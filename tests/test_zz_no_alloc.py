"""The fused reduction without allocation, igs_kernel_reduce_noalloc, against
the context entry point igs_kernel_reduce, through the C ABI.

Both run the same kernel with the same launch shape, so their sums must
agree bit for bit; the new entry point keeps its partial sums and arrival
counters in the library's static device array, which every call on the GPU
reuses.  Two calls in a row, the second on a smaller input (fewer rows and
columns, so fewer blocks and a shorter partial-sum row), each checked against
the context entry point and the oracle's one reduction; then a call without
z, a call on a non-default stream, and the size checks."""
import numpy as np
import pytest

import oracle.arnoldi as OA
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _ctx_of_size(n):
    """A context whose n matches the step-kernel buffers (its operator is unused)."""
    from paper_2205_07805_amd import igs
    a = W.Csr(n, np.arange(n + 1, dtype=np.int32), np.arange(n, dtype=np.int32), np.ones(n))
    return igs.igs_create(a.n, a.nnz, a.row_ptr, a.col_idx, a.vals, 0, None)


def _basis(torch, n, ncols, seed, ldv):
    rng = np.random.default_rng(seed)
    Vt = rng.standard_normal((ncols, n)) / np.sqrt(n)
    host = np.zeros((ncols, ldv))
    host[:, :n] = Vt
    return Vt, torch.tensor(host, device="cuda")


def _noalloc(torch, Vd, ldv, n, j, zd, stream=None):
    from paper_2205_07805_amd import igs
    PQ = torch.full((2 * (j + 1),), np.nan, dtype=torch.float64, device="cuda")
    igs.igs_kernel_reduce_noalloc(Vd, ldv, n, j, zd, PQ,
                                  None if stream is None else stream.cuda_stream)
    torch.cuda.synchronize()
    out = PQ.cpu().numpy()
    return out[: j + 1], out[j + 1:]


def _with_ctx(n, Vd, ldv, j, zd):
    from paper_2205_07805_amd import igs
    ctx = _ctx_of_size(n)
    try:
        P = np.zeros(j + 1)
        Q = np.zeros(j + 1)
        igs.igs_kernel_reduce(ctx, Vd, ldv, j, zd, P, Q if zd is not None else None)
    finally:
        igs.igs_destroy(ctx)
    return P, Q


def _oracle_close(Vt, z, j, P, Q):
    n = Vt.shape[1]
    p, alpha, q, beta = OA.one_reduction(Vt[:j], Vt[j], z)
    tol_p = 1e-14 * np.sqrt(n) * np.linalg.norm(Vt, axis=1) * np.linalg.norm(Vt[j])
    tol_q = 1e-14 * np.sqrt(n) * np.linalg.norm(Vt, axis=1) * np.linalg.norm(z)
    assert np.all(np.abs(P - np.concatenate([p, [alpha]])) <= tol_p)
    assert np.all(np.abs(Q - np.concatenate([q, [beta]])) <= tol_q)


def test_noalloc_reduce_two_calls_match_context_entry_point(torch):
    # first call: 1,048,576 rows and 61 columns (the full grid of blocks,
    # 8-column groups); second: 100,003 rows, 9 columns, odd ldv
    for n, j, pad, seed in ((1_048_576, 60, 64, 1), (100_003, 8, 13, 2)):
        ldv = n + pad
        print(f"noalloc reduce n={n} j={j} ldv=n+{pad}", flush=True)
        Vt, Vd = _basis(torch, n, j + 1, seed, ldv)
        z = W.rhs_normal(n, seed + 10)
        zd = torch.tensor(z, device="cuda")
        P, Q = _noalloc(torch, Vd, ldv, n, j, zd)
        Pc, Qc = _with_ctx(n, Vd, ldv, j, zd)
        assert np.array_equal(P, Pc) and np.array_equal(Q, Qc), (n, j)
        _oracle_close(Vt, z, j, P, Q)


def test_noalloc_reduce_without_z_and_on_a_stream(torch):
    from paper_2205_07805_amd import igs
    n, j = 50_001, 30
    print(f"noalloc reduce without z, side stream n={n} j={j}", flush=True)
    Vt, Vd = _basis(torch, n, j + 1, 5, n)
    z = W.rhs_normal(n, 6)
    zd = torch.tensor(z, device="cuda")
    P0, Q0 = _noalloc(torch, Vd, n, n, j, zd)
    P1, Q1 = _noalloc(torch, Vd, n, n, j, None)
    assert np.array_equal(P1, P0) and np.all(Q1 == 0.0)
    s = torch.cuda.Stream()
    P2, Q2 = _noalloc(torch, Vd, n, n, j, zd, stream=s)
    assert np.array_equal(P2, P0) and np.array_equal(Q2, Q0)
    # the largest column count the static array holds
    jm = igs.IGS_NOALLOC_MAX_COLS - 1
    n2 = 4_099
    Vt2, Vd2 = _basis(torch, n2, jm + 1, 8, n2)
    z2 = W.rhs_normal(n2, 9)
    zd2 = torch.tensor(z2, device="cuda")
    P3, Q3 = _noalloc(torch, Vd2, n2, n2, jm, zd2)
    Pc, Qc = _with_ctx(n2, Vd2, n2, jm, zd2)
    assert np.array_equal(P3, Pc) and np.array_equal(Q3, Qc)
    _oracle_close(Vt2, z2, jm, P3, Q3)


def test_noalloc_reduce_rejects_sizes_beyond_the_array(torch):
    from paper_2205_07805_amd import igs
    Vd = torch.zeros(16, dtype=torch.float64, device="cuda")
    PQ = torch.zeros(2 * (igs.IGS_NOALLOC_MAX_COLS + 1), dtype=torch.float64, device="cuda")
    for n, ldv, j in ((8, 8, igs.IGS_NOALLOC_MAX_COLS), (8, 8, -1), (0, 8, 0), (8, 4, 0)):
        with pytest.raises(igs.IgsError) as e:
            igs.igs_kernel_reduce_noalloc(Vd, ldv, n, j, None, PQ)
        assert e.value.code == igs.IGS_EINVAL
