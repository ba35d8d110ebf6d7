"""Batched kernels through the C ABI: igs_solve_batch (many systems advanced
by each launch) and igs_serve_batched (continuous batching at restart-cycle
granularity on one stream).

Bars:
* with the lone-solve grids (batch_reduce_rows = batch_update_tiles = 1)
  every member's x is bit-identical to a lone igs_solve_opts of the same
  system, with the same iteration count and return code;
* with the default coarse grids (fewer, larger blocks per instance) each
  member's x is bit-identical alone (a batch of one) and in the mix, since
  an instance's grid depends on its own size only; against igs_solve_opts
  it differs by summation order only: the same tolerance is met, the
  iteration count agrees within 2 (FP32 cycles: within 10 + 5%) and x within
  1e3 tol (relative);
* the relative residual of each converged member meets the tolerance
  against the oracle's operator.
"""
import numpy as np
import pytest

import oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def lone(a, b, restart, tol, gs, **opts):
    from paper_2205_07805_amd import Solver, igs
    s = Solver(a)
    try:
        x, rc, info = s.solve(b, restart=restart, tol=tol, gs_iters=gs, **opts)
        return x.cpu().numpy(), rc, info
    except igs.IgsError as e:
        return None, e.code, None
    finally:
        s.close()


def batch(systems, restart, tol, gs, **opts):
    from paper_2205_07805_amd import Solver, solve_batch
    solvers = [Solver(a) for a, _ in systems]
    try:
        xs, rc, infos, rcs = solve_batch(solvers, [b for _, b in systems], restart=restart, tol=tol,
                                         gs_iters=gs, **opts)
        return [x.cpu().numpy() for x in xs], rc, infos, rcs
    finally:
        for s in solvers:
            s.close()


SIDES = [(20, 5.0), (33, 40.0), (47, 1.0), (64, 80.0), (90, 20.0), (128, 50.0)]
LONE_GRIDS = dict(batch_reduce_rows=1, batch_update_tiles=1)


@pytest.mark.parametrize("gs,fp32", [(2, 0), (1, 0), (2, 1)])
def test_solve_batch_matches_lone(torch, gs, fp32):
    systems = [(W.convdiff2d(s, pe), W.rhs_normal(s * s, 10 + s)) for s, pe in SIDES]
    restart, tol = 30, 1e-12
    print(f"batch of {len(systems)} gs={gs} fp32={fp32}", flush=True)
    xs, rc, infos, rcs = batch(systems, restart, tol, gs, inner_fp32=fp32, **LONE_GRIDS)
    assert rc == 0 and rcs == [0] * len(systems)
    for (a, b), x, info in zip(systems, xs, infos):
        x1, rc1, info1 = lone(a, b, restart, tol, gs, inner_fp32=fp32)
        assert rc1 == 0 and info["iters"] == info1["iters"] and info["cycles"] == info1["cycles"]
        assert np.array_equal(x, x1), f"n={a.n}: batch differs from lone"
        rel = np.linalg.norm(b - O.as_operator(a).matvec(x)) / np.linalg.norm(b)
        assert rel <= tol
        print(f"  n={a.n:6d} iters {info['iters']:5d} relres {rel:.2e}", flush=True)


def test_solve_batch_mixed_outcomes(torch):
    """Members that converge at once (b = 0), run out of iterations, have
    n < restart, or bring non-finite input, beside an ordinary member."""
    good = W.convdiff2d(40, 10.0)
    tiny = W.convdiff2d(4, 3.0)           # n = 16 < restart
    bad_b = W.rhs_normal(good.n, 3)
    bad_b[7] = np.nan
    systems = [(good, W.rhs_normal(good.n, 1)), (good, np.zeros(good.n)),
               (tiny, W.rhs_normal(tiny.n, 2)), (good, bad_b)]
    restart, tol = 30, 1e-12
    print("batch with mixed outcomes", flush=True)
    xs, rc, infos, rcs = batch(systems, restart, tol, 2, maxit=0, **LONE_GRIDS)
    # a small budget for the second call: the ordinary member stops early
    xs2, rc2, infos2, rcs2 = batch(systems[:1] + systems[2:3], restart, tol, 2, maxit=45,
                                   **LONE_GRIDS)
    assert rcs[3] == -1 and np.all(xs[3] == 0.0)
    for k in range(3):
        x1, rc1, info1 = lone(*systems[k], restart, tol, 2)
        assert rcs[k] == rc1 and infos[k]["iters"] == info1["iters"]
        assert np.array_equal(xs[k], x1)
    x1, rc1, info1 = lone(*systems[0], restart, tol, 2, maxit=45)
    assert rcs2[0] == rc1 == 1 and infos2[0]["iters"] == info1["iters"]
    assert np.array_equal(xs2[0], x1)
    assert rc == -1 and rc2 == 1


def test_solve_batch_rejects_dense_and_two_reduce(torch):
    from paper_2205_07805_amd import Solver, igs, solve_batch
    d = Solver(W.random_wellcond(64, 1))
    c = Solver(W.convdiff2d(10, 1.0))
    try:
        with pytest.raises(igs.IgsError) as e:
            solve_batch([c, d], [np.ones(100), np.ones(64)], restart=10, tol=1e-10)
        assert e.value.code == igs.IGS_ENOTIMPL
        with pytest.raises(igs.IgsError) as e:
            solve_batch([c], [np.ones(100)], restart=10, tol=1e-10, two_reduce=1)
        assert e.value.code == igs.IGS_ENOTIMPL
    finally:
        d.close()
        c.close()


@pytest.mark.parametrize("fp32", [0, 1])
def test_serve_batched_matches_lone(torch, fp32):
    from paper_2205_07805_amd import serve
    trace = W.serving_trace(count=24, seed=5, side_lo=16, side_hi=72, rate=3000.0)
    restart, tol = 30, 1e-12
    print(f"serve_batched 24 requests fp32={fp32}", flush=True)
    res, wall, rc = serve([(q.a, q.b, q.arrival) for q in trace], batch=8, mem_cap=1 << 30,
                          restart=restart, tol=tol, gs_iters=2, inner_fp32=fp32, **LONE_GRIDS)
    assert rc == 0
    for q, r in zip(trace, res):
        x1, rc1, info1 = lone(q.a, q.b, restart, tol, 2, inner_fp32=fp32)
        assert r["rc"] == rc1 == 0 and r["iters"] == info1["iters"], (q.rid, r["iters"], info1)
        assert np.array_equal(r["x"], x1), f"request {q.rid} differs from its lone solve"
    spans = sorted((r["t_admit"], r["t_done"]) for r in res)
    concurrent = max(sum(1 for a, d in spans if a <= t < d) for t, _ in spans)
    print(f"  wall {wall * 1e3:.1f} ms, most requests in flight at once {concurrent}", flush=True)
    assert concurrent > 1


def test_serve_batched_memory_cap_and_bad_request(torch):
    from paper_2205_07805_amd import serve
    a = W.convdiff2d(36, 20.0)
    need = (12 * a.nnz + 4 * (a.n + 1) + 8 * a.n * 35 + 32 * 32 ** 2)
    bad = W.Csr(a.n, a.row_ptr.copy(), a.col_idx.copy(), a.vals.copy())
    bad.col_idx[3] = -1
    systems = [(a, W.rhs_normal(a.n, 60 + i), 0.0) for i in range(5)] + [(bad, W.rhs_normal(a.n, 9), 0.0)]
    print("serve_batched under a cap of 1.5 requests", flush=True)
    res, _, rc = serve(systems, batch=8, mem_cap=int(1.5 * need), restart=30, tol=1e-10,
                       **LONE_GRIDS)
    assert rc == 0 and [r["rc"] for r in res] == [0] * 5 + [-1]
    spans = sorted((r["t_admit"], r["t_done"]) for r in res[:5])
    assert all(spans[k][0] >= spans[k - 1][1] for k in range(1, 5))
    x1, _, _ = lone(a, systems[2][1], 30, 1e-10, 2)
    assert np.array_equal(res[2]["x"], x1)


@pytest.mark.parametrize("fp32", [0, 1])
def test_solve_batch_coarse_grids_alone_equals_mix(torch, fp32):
    """Default batch grids: alone (a batch of one) and in the mix agree bit
    for bit; against igs_solve_opts they agree to the tolerance."""
    systems = [(W.convdiff2d(s, pe), W.rhs_normal(s * s, 30 + s)) for s, pe in SIDES]
    systems.append((W.convdiff2d(300, 30.0), W.rhs_normal(90000, 7)))   # many blocks per instance
    restart, tol = 30, 1e-12
    print(f"coarse-grid batch of {len(systems)} fp32={fp32}", flush=True)
    xs, rc, infos, rcs = batch(systems, restart, tol, 2, inner_fp32=fp32)
    assert rc == 0 and rcs == [0] * len(systems)
    for (a, b), x, info in zip(systems, xs, infos):
        xa, rca, infa, _ = batch([(a, b)], restart, tol, 2, inner_fp32=fp32)
        assert rca == 0 and infa[0]["iters"] == info["iters"]
        assert np.array_equal(xa[0], x), f"n={a.n}: alone and in the mix differ"
        x1, rc1, info1 = lone(a, b, restart, tol, 2, inner_fp32=fp32)
        rel = np.linalg.norm(b - O.as_operator(a).matvec(x)) / np.linalg.norm(b)
        dx = np.abs(x - x1).max() / np.abs(x1).max()
        print(f"  n={a.n:6d} iters {info['iters']:5d} (lone {info1['iters']}) relres {rel:.2e} "
              f"max|x - x_lone|/max|x_lone| {dx:.1e}", flush=True)
        # FP32 cycles round differently under another summation order, which
        # can move a cycle's end by a few iterations
        slack = 2 if not fp32 else 10 + info1["iters"] // 20
        assert rel <= tol and abs(info["iters"] - info1["iters"]) <= slack
        assert dx <= 1e3 * tol
