"""Marshalling for ``igs_serve``: build the request array from CSR systems,
keep the host arrays alive for the call, and return the per-request results.
The queue, admission and the solves all run in the library."""
from __future__ import annotations

import ctypes

import numpy as np

from . import igs as _igs


def serve(systems, slots=8, mem_cap=64 << 30, restart=50, tol=1e-12, gs_iters=2, batch=0,
          **opts):
    """systems: iterable of (csr, b, arrival_seconds), csr with row_ptr,
    col_idx, vals.  batch = 0: `slots` solver slots on streams of their own
    (igs_serve); batch > 0: up to `batch` requests advanced by each launch on
    one stream (igs_serve_batched).  Returns (results, wall_seconds, rc)
    where results[i] is a dict with x (numpy), iters, rc, status, t_admit,
    t_done, arrival."""
    systems = list(systems)
    keep = []
    reqs = (_igs.IgsRequest * len(systems))()
    for i, (a, b, arrival) in enumerate(systems):
        rp = np.ascontiguousarray(a.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(a.col_idx, dtype=np.int32)
        va = np.ascontiguousarray(a.vals, dtype=np.float64)
        bb = np.ascontiguousarray(b, dtype=np.float64)
        x = np.zeros(len(bb), dtype=np.float64)
        keep.append((rp, ci, va, bb, x))
        r = reqs[i]
        r.n, r.nnz = len(bb), int(rp[-1])
        r.row_ptr, r.col_idx = rp.ctypes.data, ci.ctypes.data
        r.vals, r.b, r.x = va.ctypes.data, bb.ctypes.data, x.ctypes.data
        r.arrival = float(arrival)
    o = _igs.IgsOpts()
    for k, v in opts.items():
        setattr(o, k, v)
    if batch > 0:
        rc, wall = _igs.igs_serve_batched(reqs, batch, mem_cap, restart, tol, gs_iters, o)
    else:
        rc, wall = _igs.igs_serve(reqs, slots, mem_cap, restart, tol, gs_iters, o)
    out = []
    for i, r in enumerate(reqs):
        out.append({"x": keep[i][4], "iters": int(r.iters), "rc": int(r.rc), "status": int(r.status),
                    "t_admit": r.t_admit, "t_done": r.t_done, "arrival": r.arrival})
    return out, wall, rc
