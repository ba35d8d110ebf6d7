"""ctypes binding of the C ABI in include/igs.h (argument marshalling only).

Every function here forwards to the function of the same name in
``libigs.so``; all arithmetic of the solve runs in the library's HIP kernels.
Pointer arguments accept a torch tensor (its ``data_ptr()``), a numpy array
(host memory) or a plain integer address.  Loading fails loudly when the
library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_double, c_int, c_int32, c_int64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libigs.so")

IGS_OK, IGS_ENOCONV, IGS_EINVAL, IGS_ENOMEM, IGS_EDEVICE, IGS_ENOTIMPL, IGS_ENUMERIC = 0, 1, -1, -2, -3, -4, -5
IGS_MAX_RESTART = 512
IGS_MAX_BATCH = 32
IGS_NOALLOC_MAX_COLS = 256
IGS_NOALLOC_BYTES = (2048 + 64) * 2 * IGS_NOALLOC_MAX_COLS * 8 + 512
(IGS_K_SPMV, IGS_K_REDUCE, IGS_K_UPDATE, IGS_K_XUPDATE, IGS_K_RESIDUAL, IGS_K_OPREDUCE,
 IGS_K_COUNT) = range(7)
KERNEL_NAMES = ("spmv", "reduce", "update", "xupdate", "residual", "opreduce")
CYCLE_STATUS = ("running", "converged_at_start", "arnoldi_converged", "full", "breakdown",
                "lagnorm", "maxit", "nonfinite")

EXPORTED = (
    "igs_create", "igs_create_dense", "igs_solve", "igs_solve_opts", "igs_destroy",
    "igs_last_error", "igs_debug_copy_H", "igs_debug_copy_V", "igs_kernel_spmv",
    "igs_kernel_reduce", "igs_kernel_update", "igs_profile_get", "igs_profile_reset",
    "igs_serve", "igs_solve_batch", "igs_serve_batched", "igs_tune", "igs_tune_reset",
    "igs_kernel_reduce_noalloc", "igs_anorm_estimate", "igs_dense_variant",
)


class IgsOpts(ctypes.Structure):
    _fields_ = [("maxit", c_int64), ("lagnorm_tau", c_double), ("final_basis_vector", c_int),
                ("profile", c_int), ("max_cycles", c_int), ("keep_first_basis", c_int),
                ("profile_kernels", c_int), ("inner_fp32", c_int), ("two_reduce", c_int),
                ("separate_apply", c_int),
                ("inner_rtol", c_double), ("batch_reduce_rows", c_int),
                ("batch_update_tiles", c_int), ("cycle_graph", c_int), ("mgs", c_int),
                ("products_in_update", c_int)]


class IgsInfo(ctypes.Structure):
    _fields_ = [("iters", c_int64), ("cycles", c_int64), ("relres_true", c_double),
                ("arnoldi_relres", c_double), ("bnorm", c_double), ("converged", c_int),
                ("breakdowns", c_int), ("lagnorm_fallbacks", c_int), ("last_cycle_status", c_int),
                ("first_cycle_J", c_int), ("stagnant_cycles", c_int), ("seconds", c_double)]

    def as_dict(self) -> dict:
        d = {name: getattr(self, name) for name, _ in self._fields_ if name != "reserved"}
        d["last_cycle_status"] = CYCLE_STATUS[self.last_cycle_status] \
            if 0 <= self.last_cycle_status < len(CYCLE_STATUS) else self.last_cycle_status
        return d


class IgsRequest(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnz", c_int64), ("row_ptr", c_void_p), ("col_idx", c_void_p),
                ("vals", c_void_p), ("b", c_void_p), ("x", c_void_p), ("arrival", c_double),
                ("t_admit", c_double), ("t_done", c_double), ("iters", c_int64), ("rc", c_int),
                ("status", c_int)]


class IgsTuneReport(ctypes.Structure):
    _fields_ = [("cycle_ms_before", c_double), ("cycle_ms_after", c_double),
                ("spmv_rpg", c_int), ("reduce_halved", c_int), ("update_halved", c_int),
                ("reserved", c_int)]


class IgsError(RuntimeError):
    def __init__(self, func: str, code: int, message: str):
        super().__init__(f"{func} failed with code {code}: {message}")
        self.code = code


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libigs.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with `python -m paper_2205_07805_amd.build` "
                           "(there is no CPU fallback)")
    lib = ctypes.CDLL(path)
    P = c_void_p
    sig = {
        "igs_create": (c_int, [POINTER(P), c_int64, c_int64, P, P, P, c_int, P]),
        "igs_create_dense": (c_int, [POINTER(P), c_int64, P, c_int64, c_int, P]),
        "igs_solve": (c_int, [P, P, P, c_int, c_double, c_int, POINTER(IgsInfo)]),
        "igs_solve_opts": (c_int, [P, P, P, c_int, c_double, c_int, POINTER(IgsOpts), POINTER(IgsInfo)]),
        "igs_destroy": (c_int, [P]),
        "igs_last_error": (ctypes.c_char_p, [P]),
        "igs_debug_copy_H": (c_int, [P, P, c_int, POINTER(c_int)]),
        "igs_debug_copy_V": (c_int, [P, P, c_int64, POINTER(c_int)]),
        "igs_kernel_spmv": (c_int, [P, P, P]),
        "igs_kernel_reduce": (c_int, [P, P, c_int64, c_int, P, P, P]),
        "igs_kernel_update": (c_int, [P, P, c_int64, c_int, P, P, P, c_double]),
        "igs_kernel_reduce_noalloc": (c_int, [P, c_int64, c_int64, c_int, P, P, P]),
        "igs_anorm_estimate": (c_int, [P, POINTER(c_double)]),
        "igs_dense_variant": (c_int, [P, c_int]),
        "igs_profile_get": (c_int, [P, c_int, POINTER(c_int64), POINTER(c_double), POINTER(c_double)]),
        "igs_profile_reset": (c_int, [P]),
        "igs_serve": (c_int, [POINTER(IgsRequest), c_int, c_int, c_int64, c_int, c_double, c_int,
                              POINTER(IgsOpts), POINTER(c_double)]),
        "igs_solve_batch": (c_int, [POINTER(P), POINTER(P), POINTER(P), c_int, c_int, c_double,
                                    c_int, POINTER(IgsOpts), POINTER(IgsInfo), POINTER(c_int)]),
        "igs_serve_batched": (c_int, [POINTER(IgsRequest), c_int, c_int, c_int64, c_int, c_double,
                                      c_int, POINTER(IgsOpts), POINTER(c_double)]),
        "igs_tune": (c_int, [P, c_int, c_int, POINTER(IgsTuneReport)]),
        "igs_tune_reset": (c_int, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(x) -> c_void_p:
    """Address of a torch tensor, numpy array, ctypes object or integer."""
    if x is None:
        return c_void_p(None)
    if hasattr(x, "data_ptr"):
        return c_void_p(x.data_ptr())
    if hasattr(x, "ctypes"):
        return c_void_p(x.ctypes.data)
    if isinstance(x, c_void_p):
        return x
    return c_void_p(int(x))


def _check(func: str, rc: int, ctx=None, allow=(IGS_OK,)):
    if rc in allow:
        return rc
    msg = load_library().igs_last_error(ctx)
    raise IgsError(func, rc, msg.decode() if msg else "")


def igs_create(n, nnz, row_ptr, col_idx, vals, ptrs_on_device, hip_stream=None) -> c_void_p:
    lib = load_library()
    ctx = c_void_p()
    rc = lib.igs_create(ctypes.byref(ctx), int(n), int(nnz), _ptr(row_ptr), _ptr(col_idx),
                        _ptr(vals), int(ptrs_on_device), _ptr(hip_stream))
    _check("igs_create", rc)
    return ctx


def igs_create_dense(n, A, lda, ptr_on_device, hip_stream=None) -> c_void_p:
    lib = load_library()
    ctx = c_void_p()
    rc = lib.igs_create_dense(ctypes.byref(ctx), int(n), _ptr(A), int(lda), int(ptr_on_device),
                              _ptr(hip_stream))
    _check("igs_create_dense", rc)
    return ctx


def igs_solve(ctx, b, x, restart, tol, gs_iters):
    """Returns (return code, info dict); raises on negative codes."""
    info = IgsInfo()
    rc = load_library().igs_solve(ctx, _ptr(b), _ptr(x), int(restart), float(tol), int(gs_iters),
                                  ctypes.byref(info))
    _check("igs_solve", rc, ctx, allow=(IGS_OK, IGS_ENOCONV))
    return rc, info.as_dict()


def igs_solve_opts(ctx, b, x, restart, tol, gs_iters, opts: IgsOpts | None = None):
    info = IgsInfo()
    rc = load_library().igs_solve_opts(ctx, _ptr(b), _ptr(x), int(restart), float(tol),
                                       int(gs_iters), ctypes.byref(opts) if opts else None,
                                       ctypes.byref(info))
    _check("igs_solve_opts", rc, ctx, allow=(IGS_OK, IGS_ENOCONV))
    return rc, info.as_dict()


def igs_destroy(ctx) -> int:
    return load_library().igs_destroy(ctx)


def igs_last_error(ctx=None) -> str:
    msg = load_library().igs_last_error(ctx)
    return msg.decode() if msg else ""


def igs_debug_copy_H(ctx, H_host, ldh) -> int:
    ncols = c_int()
    _check("igs_debug_copy_H", load_library().igs_debug_copy_H(ctx, _ptr(H_host), int(ldh),
                                                               ctypes.byref(ncols)), ctx)
    return ncols.value


def igs_debug_copy_V(ctx, V_dev, ldv) -> int:
    ncols = c_int()
    _check("igs_debug_copy_V", load_library().igs_debug_copy_V(ctx, _ptr(V_dev), int(ldv),
                                                               ctypes.byref(ncols)), ctx)
    return ncols.value


def igs_kernel_spmv(ctx, u, z) -> None:
    _check("igs_kernel_spmv", load_library().igs_kernel_spmv(ctx, _ptr(u), _ptr(z)), ctx)


def igs_kernel_reduce(ctx, V, ldv, j, z, P_host, Q_host) -> None:
    _check("igs_kernel_reduce", load_library().igs_kernel_reduce(
        ctx, _ptr(V), int(ldv), int(j), _ptr(z), _ptr(P_host), _ptr(Q_host)), ctx)


def igs_kernel_update(ctx, V, ldv, j, z, t_host, r1_host, inv_gamma) -> None:
    _check("igs_kernel_update", load_library().igs_kernel_update(
        ctx, _ptr(V), int(ldv), int(j), _ptr(z), _ptr(t_host), _ptr(r1_host),
        float(inv_gamma)), ctx)


def igs_kernel_reduce_noalloc(V, ldv, n, j, z, PQ, hip_stream=None) -> None:
    """Queues the reduction on hip_stream (a torch stream's cuda_stream, or
    None for the null stream) and returns without waiting."""
    _check("igs_kernel_reduce_noalloc", load_library().igs_kernel_reduce_noalloc(
        _ptr(V), int(ldv), int(n), int(j), _ptr(z), _ptr(PQ), _ptr(hip_stream)), None)


IGS_DENSE_VALU, IGS_DENSE_MFMA, IGS_DENSE_LDS = 0, 1, 2


def igs_dense_variant(ctx, variant) -> None:
    _check("igs_dense_variant", load_library().igs_dense_variant(ctx, int(variant)), ctx)


def igs_anorm_estimate(ctx) -> float:
    out = c_double(0.0)
    _check("igs_anorm_estimate", load_library().igs_anorm_estimate(ctx, ctypes.byref(out)), ctx)
    return out.value


def igs_profile_get(ctx, which):
    n, ms, by = c_int64(), c_double(), c_double()
    _check("igs_profile_get", load_library().igs_profile_get(
        ctx, int(which), ctypes.byref(n), ctypes.byref(ms), ctypes.byref(by)), ctx)
    return n.value, ms.value, by.value


def igs_profile_reset(ctx) -> None:
    _check("igs_profile_reset", load_library().igs_profile_reset(ctx), ctx)


def igs_serve(reqs, slots, mem_cap, restart, tol, gs_iters, opts: IgsOpts | None = None):
    """reqs: a ctypes array of IgsRequest whose host arrays the caller keeps
    alive.  Returns (return code, wall seconds); raises on argument errors."""
    wall = c_double(0.0)
    rc = load_library().igs_serve(reqs, len(reqs), int(slots), int(mem_cap), int(restart),
                                  float(tol), int(gs_iters), ctypes.byref(opts) if opts else None,
                                  ctypes.byref(wall))
    _check("igs_serve", rc, None)
    return rc, wall.value


def igs_solve_batch(ctxs, bs, xs, restart, tol, gs_iters, opts: IgsOpts | None = None):
    """ctxs: contexts; bs, xs: device vectors (tensors or addresses), one per
    context.  Returns (return code, [info dict], [member return code]);
    raises when the call itself is invalid (then no member ran)."""
    k = len(ctxs)
    arr = lambda vals: (c_void_p * k)(*[_ptr(v).value for v in vals])
    infos = (IgsInfo * k)()
    unset = 99
    rcs = (c_int * k)(*([unset] * k))
    ctx_arr = (c_void_p * k)(*[c.value if isinstance(c, c_void_p) else int(c) for c in ctxs])
    rc = load_library().igs_solve_batch(ctx_arr, arr(bs), arr(xs), k, int(restart), float(tol),
                                        int(gs_iters), ctypes.byref(opts) if opts else None,
                                        infos, rcs)
    if all(r == unset for r in rcs):   # the call itself failed: no member ran
        _check("igs_solve_batch", rc, ctxs[0] if k else None, allow=(IGS_OK, IGS_ENOCONV))
    return rc, [i.as_dict() for i in infos], list(rcs)


def igs_serve_batched(reqs, batch, mem_cap, restart, tol, gs_iters, opts: IgsOpts | None = None):
    """As igs_serve, with up to `batch` requests advanced by each launch."""
    wall = c_double(0.0)
    rc = load_library().igs_serve_batched(reqs, len(reqs), int(batch), int(mem_cap), int(restart),
                                          float(tol), int(gs_iters),
                                          ctypes.byref(opts) if opts else None, ctypes.byref(wall))
    _check("igs_serve_batched", rc, None)
    return rc, wall.value


def igs_tune(ctx, restart, gs_iters=2) -> dict:
    """Choose launch shapes for ctx on the device; returns the report."""
    rep = IgsTuneReport()
    rc = load_library().igs_tune(ctx, int(restart), int(gs_iters), ctypes.byref(rep))
    _check("igs_tune", rc, ctx)
    return {name: getattr(rep, name) for name, _ in rep._fields_ if name != "reserved"}


def igs_tune_reset(ctx) -> None:
    _check("igs_tune_reset", load_library().igs_tune_reset(ctx), ctx)

