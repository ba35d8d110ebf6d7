"""CPU checks of the C-ABI boundary: the library loads, exports every symbol
declared in include/igs.h, and the ctypes structures match the C layout.
No compute calls (there is no GPU here)."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "igs.h")
LIB = os.path.join(ROOT, "paper_2205_07805_amd", "libigs.so")


def declared_functions():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(igs_\w+)\s*\(", text, re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        from paper_2205_07805_amd import build
        build.build()
    return ctypes.CDLL(LIB)


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("igs_create", "igs_create_dense", "igs_solve", "igs_destroy",
                     "igs_last_error", "igs_debug_copy_H", "igs_debug_copy_V"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_binding_covers_every_declared_symbol():
    from paper_2205_07805_amd import igs
    assert sorted(igs.EXPORTED) == declared_functions()
    for name in declared_functions():
        assert callable(getattr(igs, name)), name


def test_struct_layout_matches_c(tmp_path):
    """Compile a C probe against the header and compare sizes/offsets with ctypes."""
    from paper_2205_07805_amd.igs import IgsInfo, IgsOpts
    src = tmp_path / "probe.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "igs.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\n", sizeof(igs_opts), offsetof(igs_opts, lagnorm_tau),
         offsetof(igs_opts, keep_first_basis), sizeof(igs_info), offsetof(igs_info, seconds));
  printf("%d %d\n", IGS_MAX_RESTART, IGS_K_COUNT);
  printf("%zu %zu\n", offsetof(igs_opts, inner_fp32), offsetof(igs_opts, inner_rtol));
  printf("%zu\n", offsetof(igs_opts, batch_update_tiles));
  printf("%zu %zu\n", sizeof(igs_tune_report), offsetof(igs_tune_report, update_halved));
  printf("%zu %zu %zu %zu %zu\n", sizeof(igs_request), offsetof(igs_request, arrival),
         offsetof(igs_request, iters), offsetof(igs_request, rc), offsetof(igs_request, status));
  return 0;
}
''')
    exe = tmp_path / "probe"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    vals = [int(v) for v in out]
    assert vals[0] == ctypes.sizeof(IgsOpts)
    assert vals[1] == IgsOpts.lagnorm_tau.offset
    assert vals[2] == IgsOpts.keep_first_basis.offset
    assert vals[3] == ctypes.sizeof(IgsInfo)
    assert vals[4] == IgsInfo.seconds.offset
    from paper_2205_07805_amd import igs
    assert vals[5] == igs.IGS_MAX_RESTART and vals[6] == igs.IGS_K_COUNT
    assert vals[7] == IgsOpts.inner_fp32.offset and vals[8] == IgsOpts.inner_rtol.offset
    assert vals[9] == IgsOpts.batch_update_tiles.offset
    from paper_2205_07805_amd.igs import IgsRequest, IgsTuneReport
    assert vals[10] == ctypes.sizeof(IgsTuneReport)
    assert vals[11] == IgsTuneReport.update_halved.offset
    assert vals[12] == ctypes.sizeof(IgsRequest) and vals[13] == IgsRequest.arrival.offset
    assert vals[14] == IgsRequest.iters.offset and vals[15] == IgsRequest.rc.offset
    assert vals[16] == IgsRequest.status.offset


def test_missing_library_fails_loudly(tmp_path):
    from paper_2205_07805_amd import igs
    with pytest.raises(RuntimeError, match="missing"):
        saved = igs._lib
        igs._lib = None
        try:
            igs.load_library(str(tmp_path / "nope.so"))
        finally:
            igs._lib = saved


def test_create_rejects_bad_input_without_gpu_work(lib):
    """Argument validation happens before any device call."""
    from paper_2205_07805_amd import igs
    igs.load_library()
    ctx = ctypes.c_void_p()
    rc = igs.load_library().igs_create(ctypes.byref(ctx), 0, 0, None, None, None, 0, None)
    assert rc == igs.IGS_EINVAL and not ctx.value
    assert "invalid" in igs.igs_last_error(None)


def test_serve_rejects_bad_arguments_without_gpu_work(lib):
    """igs_serve checks its arguments and every request's size against the
    memory cap before it touches the device."""
    import numpy as np
    from paper_2205_07805_amd import igs
    L = igs.load_library()
    reqs = (igs.IgsRequest * 1)()
    b = np.ones(4)
    x = np.zeros(4)
    r = reqs[0]
    r.n, r.nnz, r.b, r.x = 4, 4, b.ctypes.data, x.ctypes.data
    assert L.igs_serve(reqs, 1, 0, 1 << 30, 10, 1e-10, 2, None, None) == igs.IGS_EINVAL
    assert L.igs_serve(reqs, 1, 1, 0, 10, 1e-10, 2, None, None) == igs.IGS_EINVAL
    assert L.igs_serve(reqs, 1, 1, 1 << 30, 0, 1e-10, 2, None, None) == igs.IGS_EINVAL
    # 4 rows need a few KiB: a 1 KiB cap admits nothing, so nothing runs
    assert L.igs_serve(reqs, 1, 1, 1024, 10, 1e-10, 2, None, None) == igs.IGS_EINVAL
    assert "more than the cap" in igs.igs_last_error(None)
    assert r.rc == igs.IGS_EINVAL and r.t_admit == -1.0
    with pytest.raises(igs.IgsError):
        igs.igs_serve(reqs, 0, 1 << 30, 10, 1e-10, 2)


def test_batch_entry_points_reject_bad_arguments_without_gpu_work(lib):
    import numpy as np
    from paper_2205_07805_amd import igs
    L = igs.load_library()
    assert L.igs_solve_batch(None, None, None, 0, 10, 1e-10, 2, None, None, None) == igs.IGS_EINVAL
    reqs = (igs.IgsRequest * 1)()
    b = np.ones(4)
    x = np.zeros(4)
    reqs[0].n, reqs[0].nnz, reqs[0].b, reqs[0].x = 4, 4, b.ctypes.data, x.ctypes.data
    for batch in (0, igs.IGS_MAX_BATCH + 1):
        assert L.igs_serve_batched(reqs, 1, batch, 1 << 30, 10, 1e-10, 2, None, None) == igs.IGS_EINVAL
    o = igs.IgsOpts(two_reduce=1)
    assert L.igs_serve_batched(reqs, 1, 4, 1 << 30, 10, 1e-10, 2, ctypes.byref(o), None) == \
        igs.IGS_ENOTIMPL
    assert L.igs_serve_batched(reqs, 1, 4, 1024, 10, 1e-10, 2, None, None) == igs.IGS_EINVAL


def test_noalloc_reduce_checks_sizes_before_any_device_call(lib):
    """Out-of-range sizes and NULL buffers are refused before the library
    touches a device (the fake addresses are never dereferenced)."""
    from paper_2205_07805_amd import igs
    fake = 4096
    cases = ((8, 8, igs.IGS_NOALLOC_MAX_COLS), (8, 8, -1), (0, 8, 0), (8, 4, 0))
    for n, ldv, j in cases:
        with pytest.raises(igs.IgsError) as e:
            igs.igs_kernel_reduce_noalloc(fake, ldv, n, j, None, fake)
        assert e.value.code == igs.IGS_EINVAL, (n, ldv, j)
        assert "no-allocation" in e.value.args[0] or "n >= 1" in e.value.args[0]
    for V, PQ in ((None, fake), (fake, None)):
        with pytest.raises(igs.IgsError) as e:
            igs.igs_kernel_reduce_noalloc(V, 8, 8, 0, None, PQ)
        assert e.value.code == igs.IGS_EINVAL


def test_noalloc_limits_match_the_header():
    from paper_2205_07805_amd import igs
    text = open(HEADER).read()
    cols = int(re.search(r"#define IGS_NOALLOC_MAX_COLS (\d+)", text).group(1))
    assert cols == igs.IGS_NOALLOC_MAX_COLS
    expr = re.search(r"#define IGS_NOALLOC_BYTES (.+)", text).group(1).replace(
        "IGS_NOALLOC_MAX_COLS", str(cols))
    assert eval(expr) == igs.IGS_NOALLOC_BYTES  # a plain integer expression of the header
