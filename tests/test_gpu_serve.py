"""The serving loop through the C ABI (igs_serve): a trace of uneven 2D
convection-diffusion solves arriving over time, admitted as slots and the
memory cap allow, solved on per-slot streams that overlap on the device.

Bars: every request's x is bit-identical to a lone solve of the same system
(the kernels reduce in a fixed order, so what runs beside a request cannot
change it); each converged x meets the relative residual tolerance against
the oracle's operator; requests overlap in time when slots allow it and never
when the memory cap admits one at a time; a malformed request fails alone.
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


def request_bytes(n, nnz, m, fp32=False):
    """Device memory a request holds while it runs (the formula in igs.h)."""
    mm = min(m, n)
    return (12 * nnz + 4 * (n + 1) + 8 * n * (mm + 5) + 32 * (mm + 2) ** 2
            + ((4 * nnz + 4 * n * (mm + 2)) if fp32 else 0))


def lone(a, b, restart, tol, gs, **opts):
    from paper_2205_07805_amd import Solver
    s = Solver(a)
    try:
        x, rc, info = s.solve(b, restart=restart, tol=tol, gs_iters=gs, **opts)
        return x.cpu().numpy(), rc, info
    finally:
        s.close()


def overlaps(res):
    spans = sorted((r["t_admit"], r["t_done"]) for r in res)
    return sum(1 for k in range(1, len(spans)) if spans[k][0] < max(e for _, e in spans[:k]))


@pytest.mark.parametrize("gs,fp32", [(2, 0), (1, 0), (2, 1)])
def test_serve_matches_lone_solves(torch, gs, fp32):
    from paper_2205_07805_amd import serve
    trace = W.serving_trace(count=24, seed=3, side_lo=16, side_hi=64, rate=4000.0)
    restart, tol = 30, 1e-12
    print(f"serve 24 requests gs={gs} fp32={fp32}", flush=True)
    res, wall, rc = serve([(q.a, q.b, q.arrival) for q in trace], slots=4, mem_cap=1 << 30,
                          restart=restart, tol=tol, gs_iters=gs, inner_fp32=fp32)
    assert rc == 0
    worst = 0.0
    for q, r in zip(trace, res):
        x1, rc1, info1 = lone(q.a, q.b, restart, tol, gs, inner_fp32=fp32)
        assert r["rc"] == rc1 and r["iters"] == info1["iters"], (q.rid, r, info1)
        assert np.array_equal(r["x"], x1), f"request {q.rid} differs from its lone solve"
        op = O.as_operator(q.a)
        rel = np.linalg.norm(q.b - op.matvec(r["x"])) / np.linalg.norm(q.b)
        worst = max(worst, rel)
        assert rc1 != 0 or rel <= tol
        assert r["t_admit"] >= r["arrival"] - 1e-3 and r["t_done"] >= r["t_admit"]
    print(f"  wall {wall * 1e3:.1f} ms, overlapping admissions {overlaps(res)}, "
          f"worst relres {worst:.2e}", flush=True)
    assert overlaps(res) > 0


def test_serve_memory_cap_admits_one_at_a_time(torch):
    from paper_2205_07805_amd import serve
    side, restart = 40, 30
    a = W.convdiff2d(side, 20.0)
    need = request_bytes(a.n, int(a.row_ptr[-1]), restart)
    systems = [(a, W.rhs_normal(a.n, 50 + i), 0.0) for i in range(6)]
    print(f"serve with a cap of 1.5 requests ({need} bytes each)", flush=True)
    res, _, rc = serve(systems, slots=4, mem_cap=int(1.5 * need), restart=restart, tol=1e-10)
    assert rc == 0 and all(r["rc"] == 0 for r in res)
    assert overlaps(res) == 0
    res2, _, _ = serve(systems, slots=4, mem_cap=int(4.5 * need), restart=restart, tol=1e-10)
    for r, r2 in zip(res, res2):
        assert np.array_equal(r["x"], r2["x"])
    print(f"  overlaps with cap 1.5: 0, with cap 4.5: {overlaps(res2)}", flush=True)


def test_serve_malformed_request_fails_alone(torch):
    from paper_2205_07805_amd import serve
    good = W.convdiff2d(20, 5.0)
    bad = W.Csr(good.n, good.row_ptr.copy(), good.col_idx.copy(), good.vals.copy())
    bad.col_idx[5] = good.n + 3          # out of range: rejected on the host
    systems = [(good, W.rhs_normal(good.n, 1), 0.0), (bad, W.rhs_normal(good.n, 2), 0.0),
               (good, W.rhs_normal(good.n, 3), 0.0)]
    res, _, rc = serve(systems, slots=2, restart=20, tol=1e-10)
    assert rc == 0
    assert res[1]["rc"] == -1 and res[0]["rc"] == 0 and res[2]["rc"] == 0
