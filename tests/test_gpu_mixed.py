"""Mixed precision through the C ABI: FP32 restart cycles (operator apply,
fused reduction with FP64 sums, basis update with FP64 coefficients) inside
FP64 restarts (residual b - A x, small solve, Givens least squares,
x = x0 + V y), against the FP64 oracle.

Bars: the solve reaches the same FP64 tolerance as the FP64 path (relative
residual <= tol, backward error <= 1e-14 at tol 1e-13); x agrees with the
oracle's FP64 solution to the accuracy the tolerance implies; the first
cycle's Hessenberg columns agree with the oracle's to FP32 rounding (about
1e-6 relative, bar 1e-5).  Each test prints its errors against the oracle.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W
from oracle import diagnostics as D

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def solve(a, b, restart, tol, gs, **opts):
    from paper_2205_07805_amd import Solver
    s = Solver(a)
    try:
        x, rc, info = s.solve(b, restart=restart, tol=tol, gs_iters=gs, **opts)
        H = s.first_cycle_H() if info["first_cycle_J"] > 0 else None
        return x.cpu().numpy(), rc, info, H
    finally:
        s.close()


def h_rel_err(H, Hr, ncols):
    k = min(ncols, H.shape[1], Hr.shape[1])
    return max(np.linalg.norm(H[: c + 2, c] - Hr[: c + 2, c]) / np.linalg.norm(Hr[: c + 2, c])
               for c in range(k))


@pytest.mark.parametrize("gs", [2, 1])
def test_mixed_convdiff2d_32_matches_fp64_oracle(torch, gs):
    a, b = W.make_convdiff2d_32()
    tol = 1e-13
    print(f"mixed convdiff2d_32 gs={gs}", flush=True)
    x, rc, info, H = solve(a, b, 50, tol, gs, inner_fp32=1)
    ref = O.gmres(a, b, restart=50, tol=tol, variant="igs1r" if gs == 2 else "igs2r", gs_iters=gs)
    op = O.as_operator(a)
    relres = np.linalg.norm(b - op.matvec(x)) / np.linalg.norm(b)
    beta = D.backward_error(op, b, x, D.norm2(op))
    xerr = np.abs(x - ref.x).max() / np.abs(ref.x).max()
    herr = h_rel_err(H, ref.first_cycle.H, 10)
    print(f"  iters {info['iters']} (FP64 oracle {ref.iters}), relres {relres:.2e}, beta {beta:.2e}, "
          f"max|x - x_oracle|/max|x| {xerr:.2e}, H cols 0..9 rel err {herr:.2e}", flush=True)
    assert rc == 0 and info["converged"] == 1
    assert relres <= tol and beta <= 1e-14
    assert xerr <= 1e2 * tol
    assert herr <= 1e-5
    # FP32 cycles may need a few more iterations, never many more
    assert info["iters"] <= 1.5 * ref.iters + 50


def test_mixed_convdiff3d_37_ragged(torch):
    """n = 37^3 = 50653 (not a multiple of the 4-row FP32 vectors)."""
    a = W.convdiff3d(37, 50.0)
    b = W.rhs_normal(a.n, 0)
    tol = 1e-12
    print("mixed convdiff3d_37", flush=True)
    x, rc, info, H = solve(a, b, 30, tol, 2, inner_fp32=1)
    ref = O.gmres(a, b, restart=30, tol=tol, variant="igs1r")
    op = O.as_operator(a)
    relres = np.linalg.norm(b - op.matvec(x)) / np.linalg.norm(b)
    herr = h_rel_err(H, ref.first_cycle.H, 10)
    xerr = np.abs(x - ref.x).max() / np.abs(ref.x).max()
    print(f"  iters {info['iters']} (FP64 oracle {ref.iters}), relres {relres:.2e}, "
          f"max|x - x_oracle|/max|x| {xerr:.2e}, H cols 0..9 rel err {herr:.2e}", flush=True)
    assert rc == 0 and relres <= tol
    assert herr <= 1e-5
    assert xerr <= 1e3 * tol


def test_convdiff3d_103_four_row_vectors_ragged(torch):
    """n = 103^3 = 1,092,727 rows: the update pass takes four row vectors per
    thread in FP64 (2,048-row tiles) and in FP32 (4,096-row tiles), each with
    a partial last tile, and the operator apply one row per thread (odd n).
    Both solves reach the tolerance, their first-cycle Hessenberg columns
    match the FP64 oracle's (FP64 to 1e-11, FP32 cycles to 1e-5), and the
    two solutions agree to what the tolerance implies."""
    a = W.convdiff3d(103, 50.0)
    b = W.rhs_normal(a.n, 0)
    tol = 1e-12
    op = O.as_operator(a)
    ref = O.gmres(a, b, restart=40, tol=tol, variant="igs1r", max_cycles=1).first_cycle
    print(f"convdiff3d_103 n={a.n}", flush=True)
    xs = {}
    for fp32 in (0, 1):
        x, rc, info, H = solve(a, b, 40, tol, 2, inner_fp32=fp32, maxit=6000)
        relres = np.linalg.norm(b - op.matvec(x)) / np.linalg.norm(b)
        herr = h_rel_err(H, ref.H, 10)
        print(f"  fp32={fp32}: rc {rc} iters {info['iters']} relres {relres:.2e} "
              f"H cols 0..9 rel err {herr:.2e}", flush=True)
        assert rc == 0 and info["converged"] == 1 and relres <= tol
        assert herr <= (1e-5 if fp32 else 1e-11)
        xs[fp32] = x
    d = np.abs(xs[1] - xs[0]).max() / np.abs(xs[0]).max()
    print(f"  max|x32 - x64|/max|x64| {d:.2e}", flush=True)
    assert d <= 1e3 * tol


def test_mixed_convdiff3d_96_backward_error(torch):
    """The 96^3 system (n = 884,736): GMRES(40) with FP32 cycles reaches
    backward error <= 1e-14 like the FP64 solve."""
    a, b = W.make_convdiff3d(96, 50.0)
    tol = 5e-14   # relative residual 1e-13 leaves beta at about 1.5e-14 here
    op = O.as_operator(a)
    anorm = D.norm2_estimate(op, a.n, iters=60)   # a lower bound: conservative
    print("mixed convdiff3d_96", flush=True)
    out = {}
    for fp32 in (0, 1):
        x, rc, info, _ = solve(a, b, 40, tol, 2, inner_fp32=fp32, maxit=4000)
        beta = D.backward_error(op, b, x, anorm)
        out[fp32] = (x, info["iters"], beta)
        print(f"  fp32={fp32}: rc {rc} iters {info['iters']} beta {beta:.2e}", flush=True)
        assert rc == 0 and beta <= 1e-14
    x64, x32 = out[0][0], out[1][0]
    print(f"  max|x32 - x64|/max|x64| {np.abs(x32 - x64).max() / np.abs(x64).max():.2e}", flush=True)
    assert out[1][1] <= 1.5 * out[0][1] + 80
    # each result against the FP64 oracle's solve of the same system: every
    # solution has relative residual <= tol, so ||A (x - x_oracle)|| <= 2 tol ||b||
    ref = O.gmres(a, b, restart=40, tol=tol, variant="igs1r", maxit=4000)
    assert ref.converged
    bn = np.linalg.norm(b)
    for fp32 in (0, 1):
        x = out[fp32][0]
        dres = np.linalg.norm(op.matvec(x - ref.x)) / bn
        dmax = np.abs(x - ref.x).max() / np.abs(ref.x).max()
        print(f"  fp32={fp32} against the FP64 oracle (iters {ref.iters}): "
              f"max|x - x_oracle|/max|x_oracle| {dmax:.2e}, ||A dx||/||b|| {dres:.2e}", flush=True)
        assert dres <= 2 * tol
        assert dmax <= 1e-9


def test_mixed_rejects_dense_and_first_basis(torch):
    from paper_2205_07805_amd import igs
    a = W.random_wellcond(32, 1)
    b = W.rhs_normal(32, 2)
    with pytest.raises(igs.IgsError) as e:
        solve(a, b, 10, 1e-10, 2, inner_fp32=1)
    assert e.value.code == igs.IGS_ENOTIMPL
    c = W.convdiff2d(8, 1.0)
    with pytest.raises(igs.IgsError) as e:
        solve(c, W.rhs_normal(c.n, 1), 10, 1e-10, 2, inner_fp32=1, keep_first_basis=1)
    assert e.value.code == igs.IGS_ENOTIMPL
