"""The C ABI on the host (no GPU needed): the library loads, exports every
function include/mr3.h declares, the ctypes structures match the C layout,
and argument errors come back as the documented codes without any device
work."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest
import torch

import paper_1304_1864_amd as mr3

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "mr3.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^[A-Za-z_][\w\s\*]*?\b(mr3_\w+)\s*\(", text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_entry_points():
    names = declared_functions()
    for must in ("mr3_solve_f32", "mr3_solve_f64", "mr3_solve_batched", "mr3_server_create",
                 "mr3_server_submit", "mr3_server_wait", "mr3_check_f64"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = mr3.load_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(mr3.EXPORTS) == declared_functions()
    assert mr3.version().startswith("mr3-mi355x")


def _c_layout():
    """sizeof/offsetof of the ABI structures as the C compiler sees them."""
    src = r"""
#include <stddef.h>
#include <stdio.h>
#include "mr3.h"
#define F(T, f) printf(#T "." #f " %zu\n", offsetof(T, f));
int main(void) {
    printf("mr3_params %zu\nmr3_stats %zu\nmr3_range_desc %zu\nmr3_request %zu\nmr3_result %zu\n",
           sizeof(mr3_params), sizeof(mr3_stats), sizeof(mr3_range_desc), sizeof(mr3_request),
           sizeof(mr3_result));
    printf("mr3_tune_entry %zu\n", sizeof(mr3_tune_entry));
    F(mr3_stats, bisect_count) F(mr3_stats, bisect_rows) F(mr3_stats, bisect_lanes)
    F(mr3_tune_entry, count_lo) F(mr3_tune_entry, rows_hi) F(mr3_tune_entry, lanes)
    F(mr3_params, seed) F(mr3_params, profile) F(mr3_params, points_per_lane) F(mr3_params, gaptol_abs) F(mr3_params, initial)
    F(mr3_stats, stage_ms) F(mr3_stats, twist_row_steps) F(mr3_stats, dqds_transforms)
    F(mr3_stats, n_sliced_roots) F(mr3_stats, n_singleton_first_levels)
    F(mr3_request, range) F(mr3_request, ldz) F(mr3_result, batch_size)
    return 0;
}
"""
    with tempfile.TemporaryDirectory() as td:
        c = os.path.join(td, "layout.c")
        exe = os.path.join(td, "layout")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        out = subprocess.check_output([exe]).decode().split("\n")
    return dict(line.split() for line in out if line.strip())


def test_struct_layout_matches_c():
    lay = _c_layout()
    for name in ("mr3_params", "mr3_stats", "mr3_range_desc", "mr3_request", "mr3_result",
                 "mr3_tune_entry"):
        assert ctypes.sizeof(getattr(mr3, name)) == int(lay[name]), name
    for key, val in lay.items():
        if "." in key:
            t, f = key.split(".")
            assert getattr(getattr(mr3, t), f).offset == int(val), key


def test_defaults():
    p32, p64 = mr3.default_params(32), mr3.default_params(64)
    assert p32.gaptol == 1e-5 and p64.gaptol == 1e-10
    assert p32.bisect_rel == pytest.approx(1e-7) and p64.bisect_rel == pytest.approx(1e-12)
    assert p32.xi == 2.0 ** -24 and p64.xi == 2.0 ** -53
    assert p32.k_elg == 10 and p32.k_rs == 1 and p32.rqi_max_iter == 10
    lib = mr3.load_library()
    assert lib.mr3_default_params(ctypes.byref(mr3.mr3_params()), 16) == -2
    assert lib.mr3_default_params(None, 64) == -1


def test_argument_errors_without_device_work():
    lib = mr3.load_library()
    m = ctypes.c_int64(0)
    # null handle
    assert lib.mr3_solve_f64(None, 4, None, None, 0, 0.0, 0.0, 1, 4, ctypes.byref(m), None, None,
                             4, None, 0, None) == -1
    assert lib.mr3_solve_batched(None, 1, 64, None, None, None, None, None, None, None, None,
                                 None, None, None, None, 0, None) == -1
    assert lib.mr3_solve_noalloc(None, 64, 4, None, None, 0, 0.0, 0.0, 1, 4, ctypes.byref(m), None,
                                 None, 4, None) == -1
    assert lib.mr3_check_f64(None, 1, 1, None, None, None, None, 1, None, None, None) == -1
    assert lib.mr3_destroy(None) == -1
    assert lib.mr3_set_tuning(None, None, -1) == -1
    assert lib.mr3_get_tuning(None, None, 0) == -1
    assert lib.mr3_bisect_lanes(None, mr3.MR3_TUNE_ROOT, 64, 100, 100) == -1
    assert lib.mr3_server_destroy(None) == -1
    assert lib.mr3_server_create(ctypes.byref(ctypes.c_void_p()), None, 1 << 20, 4) == -2
    if not torch.cuda.is_available():
        h = ctypes.c_void_p()
        assert lib.mr3_create(ctypes.byref(h), 0) == mr3.MR3_ERR_NO_DEVICE


def test_request_bytes_monotone():
    b = [mr3.mr3_request_bytes(n, k, 64) for n, k in ((0, 0), (64, 64), (1000, 100), (1000, 1000))]
    assert b[0] > 0 and b[1] < b[2] < b[3]
    assert mr3.mr3_request_bytes(20000, 20000, 64) >= 8 * 20000 * 20000


def test_workspace_query():
    """mr3_workspace_bytes (no handle needed for the defaults): zero for
    invalid arguments and n = 0; at least the eigenvector tiles of a whole
    level (n (k + 32) binary64 values per side-stream parity); growing with
    n and with the wanted pairs; more for double-double than binary64
    working precision; the batched query of one problem equals the single
    one."""
    q = mr3.mr3_workspace_bytes
    A, V, I = mr3.RANGE_ALL, mr3.RANGE_VALUE, mr3.RANGE_INDEX
    assert q(None, 0, A, 0, 64) == 0 and q(None, -1, A, 0, 64) == 0
    assert q(None, 10, 7, 0, 64) == 0 and q(None, 10, A, 0, 16) == 0
    for n in (1, 100, 4096, 20000):
        full = q(None, n, A, 0, 64)
        assert full >= 2 * 8 * n * (n + 32)
        assert q(None, n, A, 0, 32) < full
        assert q(None, n, I, max(1, n // 10), 64) <= full
        assert n == 1 or q(None, n, I, n // 10, 64) < full
        assert q(None, n, V, 0, 64) == full  # unknown count: all pairs
        assert mr3.mr3_workspace_bytes_batched(None, 64, [n]) == full
        low = mr3.mr3_workspace_min_bytes(None, n, A, 0, 64)
        assert 0 < low <= full and (n < 1000 or low < full / 8)
    assert q(None, 2000, A, 0, 64) < q(None, 4000, A, 0, 64)
    assert q(None, 4000, I, 100, 64) < q(None, 4000, I, 1000, 64)
    two = mr3.mr3_workspace_bytes_batched(None, 32, [300, 500], [(A, 0.0, 0.0, 1, 300),
                                                              (I, 0.0, 0.0, 1, 50)])
    assert two > q(None, 500, I, 50, 32)
    assert mr3.mr3_workspace_bytes_batched(None, 32, []) == 0


def test_noalloc_limits_declared():
    text = open(HEADER).read()
    assert "MR3_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)" in text
    assert "MR3_NOALLOC_MAX_N 16384" in text
    lib = mr3.load_library()
    m = ctypes.c_int64(0)
    # precision and size are checked before the handle is used
    assert lib.mr3_solve_noalloc(ctypes.c_void_p(1), 16, 4, None, None, 0, 0.0, 0.0, 1, 4,
                                 ctypes.byref(m), None, None, 4, None) == -2
    assert lib.mr3_solve_noalloc(ctypes.c_void_p(1), 64, 16385, None, None, 0, 0.0, 0.0, 1, 4,
                                 ctypes.byref(m), None, None, 16385, None) == -3
