"""Parity at the bench workload's full size: the 3D convection-diffusion
system with 128^3 = 2,097,152 rows (14,581,760 nonzeros), GMRES(60), two
sweeps, tol 1e-10, through the C ABI in the launch configuration the bench
times (the step kernels on a basis with the solver's leading dimension).

The oracle's step functions are vectorised, so every output is compared,
not a sample: the operator apply, the fused reduction at j = 30 and 60 (with
and without z), and the update at j = 59.  The whole solve is checked on the
first cycle's Hessenberg columns 0..9 against the oracle's first cycle, and
on its true relative residual and backward error; with one and with two
sweeps it is run to convergence beside the oracle's solve (about half a
minute of host time each): the iteration count within +-2, the first-cycle
columns, and x.
"""
import numpy as np
import pytest

import oracle as O
import oracle.arnoldi as OA
import workloads as W
from oracle import diagnostics as D

pytestmark = pytest.mark.gpu

N = 128


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def system():
    return W.make_convdiff3d(N, 50.0)


def ldv_of(n):
    # the solver's layout: whole 64-row groups, no power-of-two column stride
    ld = (n + 63) // 64 * 64
    return ld + 64 if ld % 4096 == 0 else ld


def test_fullsize_step_kernels(torch, system):
    from paper_2205_07805_amd import igs
    a, _ = system
    n = a.n
    ldv = ldv_of(n)
    ctx = igs.igs_create(a.n, a.nnz, a.row_ptr, a.col_idx, a.vals, 0, None)
    try:
        op = O.as_operator(a)
        rng = np.random.default_rng(128)
        print(f"full-size step kernels n={n} ldv={ldv}", flush=True)
        # operator apply, every row
        u = rng.standard_normal(n)
        ud = torch.tensor(u, device="cuda")
        zd = torch.empty_like(ud)
        igs.igs_kernel_spmv(ctx, ud, zd)
        z = op.matvec(u)
        absz = O.as_operator(W.Csr(a.n, a.row_ptr, a.col_idx, np.abs(a.vals))).matvec(np.abs(u))
        assert np.all(np.abs(zd.cpu().numpy() - z) <= 4e-16 * 8 * absz + 1e-300)
        # fused reduction at j = 30 and j = 60, every entry
        m = 60
        Vt = rng.standard_normal((m + 2, n)) / np.sqrt(n)
        host = np.zeros((m + 2, ldv))
        host[:, :n] = Vt
        Vd = torch.tensor(host, device="cuda")
        zr = W.rhs_normal(n, 5)
        zrd = torch.tensor(zr, device="cuda")
        for j in (30, 60):
            P = np.zeros(j + 1)
            Q = np.zeros(j + 1)
            igs.igs_kernel_reduce(ctx, Vd, ldv, j, zrd, P, Q)
            p, alpha, q, beta = OA.one_reduction(Vt[:j], Vt[j], zr)
            Pref = np.concatenate([p, [alpha]])
            Qref = np.concatenate([q, [beta]])
            tol_p = 1e-14 * np.sqrt(n) * np.linalg.norm(Vt[: j + 1], axis=1) * np.linalg.norm(Vt[j])
            tol_q = 1e-14 * np.sqrt(n) * np.linalg.norm(Vt[: j + 1], axis=1) * np.linalg.norm(zr)
            assert np.all(np.abs(P - Pref) <= tol_p), j
            assert np.all(np.abs(Q - Qref) <= tol_q), j
            P2 = np.zeros(j + 1)
            igs.igs_kernel_reduce(ctx, Vd, ldv, j, None, P2, None)
            assert np.array_equal(P2, P), j
        # update at j = 59, every row of v_j and u_{j+1}
        j = 59
        t = rng.standard_normal(j) * 1e-3
        r1 = rng.standard_normal(j + 1)
        gamma = 0.61
        igs.igs_kernel_update(ctx, Vd, ldv, j, zrd, t, r1, 1.0 / gamma)
        out_j = Vd[j, :n].cpu().numpy()
        out_n = Vd[j + 1, :n].cpu().numpy()
        vj = OA.normalise_after_second_sweep(Vt[:j], Vt[j], t, gamma)
        un = OA.first_sweep_next(np.vstack([Vt[:j], vj[None, :]]), zr, gamma, r1)
        np.testing.assert_allclose(out_j, vj, rtol=0, atol=1e-13 * np.abs(vj).max())
        np.testing.assert_allclose(out_n, un, rtol=0, atol=1e-13 * np.abs(un).max())
        np.testing.assert_array_equal(Vd[:j, :n].cpu().numpy(), Vt[:j])
    finally:
        igs.igs_destroy(ctx)


def test_fullsize_solve(torch, system):
    from paper_2205_07805_amd import Solver
    a, b = system
    print(f"full-size solve n={a.n} GMRES(60) tol 1e-10", flush=True)
    s = Solver(a)
    try:
        x, rc, info = s.solve(b, restart=60, tol=1e-10, gs_iters=2)
        H = s.first_cycle_H()
    finally:
        s.close()
    xh = x.cpu().numpy()
    op = O.as_operator(a)
    relres = np.linalg.norm(b - op.matvec(xh)) / np.linalg.norm(b)
    anorm = D.norm2_estimate(op, a.n, iters=30)
    beta = D.backward_error(op, b, xh, anorm)
    print(f"  iters {info['iters']} relres {relres:.2e} beta {beta:.2e}", flush=True)
    assert rc == 0 and info["converged"] == 1 and relres <= 1e-10 and beta <= 1e-10
    ref = O.gmres(a, b, restart=60, tol=1e-10, variant="igs1r", max_cycles=1).first_cycle
    assert info["first_cycle_J"] == ref.J == 60
    for c in range(10):
        hc, hr = H[: c + 2, c], ref.H[: c + 2, c]
        assert np.linalg.norm(hc - hr) <= 1e-11 * np.linalg.norm(hr), c


@pytest.mark.parametrize("gs", [2, 1])
def test_fullsize_solve_to_convergence_matches_oracle(torch, system, gs):
    """Algorithm 4.2 (two sweeps) and Algorithm 4.1 stopped after its first
    sweep (one sweep), GMRES(60) to tol 1e-10 at 128^3, against the oracle's
    solve of the same variant.  x: both solutions have relative residual
    <= tol, so ||A (x - x_oracle)|| <= 2 tol ||b|| whatever the rounding; the
    two solves follow the same iterates up to rounding, so x also agrees to
    1e-6 relative (far inside kappa(A) * 2 tol)."""
    from paper_2205_07805_amd import Solver
    a, b = system
    tol = 1e-10
    print(f"full-size solve to convergence gs={gs} n={a.n}", flush=True)
    s = Solver(a)
    try:
        x, rc, info = s.solve(b, restart=60, tol=tol, gs_iters=gs)
        H = s.first_cycle_H()
    finally:
        s.close()
    xh = x.cpu().numpy()
    v, g = ("igs1r", 2) if gs == 2 else ("igs2r", 1)
    ref = O.gmres(a, b, restart=60, tol=tol, variant=v, gs_iters=g)
    op = O.as_operator(a)
    bn = np.linalg.norm(b)
    dres = np.linalg.norm(op.matvec(xh - ref.x)) / bn
    dx = np.linalg.norm(xh - ref.x) / np.linalg.norm(ref.x)
    print(f"  gpu iters {info['iters']} oracle iters {ref.iters}; "
          f"||A dx||/||b|| {dres:.2e}; ||dx||/||x|| {dx:.2e}", flush=True)
    assert rc == 0 and info["converged"] == 1 and ref.converged
    assert abs(info["iters"] - ref.iters) <= 2, (info["iters"], ref.iters)
    assert np.linalg.norm(b - op.matvec(xh)) <= tol * bn
    assert dres <= 2 * tol
    assert dx <= 1e-6
    assert info["first_cycle_J"] == ref.first_cycle.J == 60
    for c in range(10):
        hc, hr = H[: c + 2, c], ref.first_cycle.H[: c + 2, c]
        nrm = np.linalg.norm(hr)
        assert np.linalg.norm(hc - hr) <= 1e-11 * nrm, c
        assert np.all(np.abs(hc - hr) <= 1e-11 * np.maximum(np.abs(hr), 1e-3 * nrm)), c
