"""The restart cycle recorded in a HIP graph and replayed (opts.cycle_graph)
against the same solve launched eagerly, through the C ABI.

Bar: bit-identical x and the same iteration count.  Every solve replays the
graph once per cycle with host synchronisations and eager work (the check
cycle, the copies of the control block) between the replays; the graph is
reused across solves with the same buffers and recorded again when b, x or
the settings change.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("gs,fp32", [(2, 0), (1, 0), (2, 1)])
def test_graph_cycles_match_eager(torch, gs, fp32):
    from paper_2205_07805_amd import Solver
    a = W.convdiff2d(48, 30.0)
    b = W.rhs_normal(a.n, 4)
    s = Solver(a)
    try:
        bd = s.to_device(b)
        print(f"graph vs eager gs={gs} fp32={fp32}", flush=True)
        x0, rc0, i0 = s.solve(bd, restart=25, tol=1e-12, gs_iters=gs, inner_fp32=fp32)
        x0 = x0.cpu().numpy()
        assert rc0 == 0 and i0["cycles"] > 3
        # the same buffers for both graph solves: the second reuses the graph
        from paper_2205_07805_amd import igs
        x = torch.zeros_like(bd)
        o = igs.IgsOpts(inner_fp32=fp32, cycle_graph=1)
        for rep in range(2):
            x.zero_()
            with torch.cuda.stream(s.stream):
                rc1, i1 = igs.igs_solve_opts(s.ctx, bd, x, 25, 1e-12, gs, o)
            assert rc1 == 0 and i1["iters"] == i0["iters"] and i1["cycles"] == i0["cycles"]
            assert np.array_equal(x.cpu().numpy(), x0), f"replay pass {rep} differs"
        # other settings: recorded again
        x2, rc2, i2 = s.solve(bd, restart=20, tol=1e-12, gs_iters=gs, inner_fp32=fp32,
                              cycle_graph=1)
        x3, rc3, i3 = s.solve(bd, restart=20, tol=1e-12, gs_iters=gs, inner_fp32=fp32)
        assert i2["iters"] == i3["iters"] and np.array_equal(x2.cpu().numpy(), x3.cpu().numpy())
    finally:
        s.close()


def test_graph_cycles_maxit_and_nonzero_x0(torch):
    from paper_2205_07805_amd import Solver
    a = W.convdiff2d(40, 5.0)
    b = W.rhs_normal(a.n, 8)
    x0 = W.rhs_normal(a.n, 9)
    s = Solver(a)
    try:
        print("graph with maxit and x0", flush=True)
        for kw in (dict(maxit=70), dict()):
            xe, rce, ie = s.solve(b, x0=x0, restart=30, tol=1e-12, **kw)
            xg, rcg, ig = s.solve(b, x0=x0, restart=30, tol=1e-12, cycle_graph=1, **kw)
            assert rce == rcg and ie["iters"] == ig["iters"]
            assert np.array_equal(xe.cpu().numpy(), xg.cpu().numpy())
    finally:
        s.close()
