"""Convenience wrapper around one ``igs_ctx``: torch tensors hold the device
buffers, the library does all the work.  Argument marshalling only."""
from __future__ import annotations

import numpy as np

from . import igs as _igs


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("the IGS-GMRES library needs a ROCm GPU (torch.cuda is unavailable)")
    return torch


class Solver:
    """Solver context for a CSR (``row_ptr``/``col_idx``/``vals`` attributes) or
    dense (2-D numpy array) operator, on the current torch device and stream."""

    def __init__(self, a, stream=None):
        torch = _torch()
        _igs.load_library()
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        handle = self.stream.cuda_stream
        if hasattr(a, "row_ptr"):
            self.n = int(a.n)
            rp = np.ascontiguousarray(a.row_ptr, dtype=np.int32)
            ci = np.ascontiguousarray(a.col_idx, dtype=np.int32)
            va = np.ascontiguousarray(a.vals, dtype=np.float64)
            self.ctx = _igs.igs_create(self.n, int(rp[-1]), rp, ci, va, 0, handle)
        else:
            d = np.ascontiguousarray(a, dtype=np.float64)
            self.n = d.shape[0]
            self.ctx = _igs.igs_create_dense(self.n, d, d.shape[1], 0, handle)

    def to_device(self, v):
        torch = _torch()
        if isinstance(v, torch.Tensor):
            return v.to(device=self.device, dtype=torch.float64).contiguous()
        return torch.as_tensor(np.ascontiguousarray(v, dtype=np.float64), device=self.device)

    def solve(self, b, x0=None, restart=50, tol=1e-12, gs_iters=2, **opts):
        """Return (x, rc, info).  b, x0: numpy arrays or torch tensors."""
        torch = _torch()
        bd = self.to_device(b)
        x = self.to_device(x0).clone() if x0 is not None else torch.zeros_like(bd)
        o = _igs.IgsOpts()
        for k, v in opts.items():
            setattr(o, k, v)
        with torch.cuda.stream(self.stream):
            rc, info = _igs.igs_solve_opts(self.ctx, bd, x, restart, tol, gs_iters, o)
        return x, rc, info

    def first_cycle_H(self):
        """H (J+1 x J, before rotation) of the first cycle of the last solve."""
        ld = _igs.IGS_MAX_RESTART + 1
        buf = np.zeros(ld * _igs.IGS_MAX_RESTART, dtype=np.float64)
        ncols = _igs.igs_debug_copy_H(self.ctx, buf, ld)
        return buf[: ld * ncols].reshape(ncols, ld).T[: ncols + 1, :].copy()

    def first_cycle_V(self, ncols_max):
        torch = _torch()
        V = torch.empty((ncols_max, self.n), dtype=torch.float64, device=self.device)
        ncols = _igs.igs_debug_copy_V(self.ctx, V, self.n)
        return V[:ncols]

    def profile(self):
        out = {}
        for k, name in enumerate(_igs.KERNEL_NAMES):
            out[name] = _igs.igs_profile_get(self.ctx, k)
        return out

    def profile_reset(self):
        _igs.igs_profile_reset(self.ctx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            _igs.igs_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(solvers, bs, x0s=None, restart=50, tol=1e-12, gs_iters=2, **opts):
    """Solve one system per Solver together (igs_solve_batch).  Returns
    (xs, rc, infos, rcs); xs are device tensors."""
    torch = _torch()
    bds = [s.to_device(b) for s, b in zip(solvers, bs)]
    xs = [s.to_device(x).clone() if x0s is not None and x is not None else torch.zeros_like(bd)
          for s, bd, x in zip(solvers, bds, x0s if x0s is not None else [None] * len(bds))]
    o = _igs.IgsOpts()
    for k, v in opts.items():
        setattr(o, k, v)
    torch.cuda.synchronize()
    rc, infos, rcs = _igs.igs_solve_batch([s.ctx for s in solvers], bds, xs, restart, tol,
                                          gs_iters, o)
    return xs, rc, infos, rcs
