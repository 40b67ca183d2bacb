"""MI355X-native mixed-precision MRRR for the symmetric tridiagonal eigenproblem.

Thin ctypes binding over ``libmr3.so`` (C ABI in ``include/mr3.h``).  The
functions named like the C entry points take torch tensors where the C call
takes device pointers and only marshal arguments; every step of the solve runs
in the library's HIP kernels.  There is no CPU fallback: importing works
without a GPU, but any call fails loudly if the library or the device is
missing.

Convenience wrappers:
    solve(d, e, range="all", vl=..., vu=..., il=..., iu=..., vectors=True)
        d, e: 1-D CUDA tensors (float32 -> FP32 I/O with binary64 inside,
        float64 -> FP64 I/O with double-double inside).  Returns (W, Z).
    solve_batched(ds, es, ...)   many problems in one pass
    check(d, e, W, Z)            (orthogonality, residual) of FP64 results
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmr3.so")

RANGE_ALL, RANGE_VALUE, RANGE_INDEX = 0, 1, 2
STAGES = ["prep", "bisect", "classify", "rqi", "zout", "child", "cbisect", "verify"]
MR3_OK, MR3_ERR_NUMERIC, MR3_ERR_HIP, MR3_ERR_NO_DEVICE, MR3_ERR_GAPTOL = 0, 1, 2, 3, 4
MR3_INITIAL_BISECTION, MR3_INITIAL_DQDS = 0, 1
MR3_DQDS_MAX_N = 4096
MR3_NOALLOC_SCRATCH_BYTES = 128 << 20
MR3_NOALLOC_MAX_N = 16384


class MR3Error(RuntimeError):
    def __init__(self, fn: str, code: int):
        super().__init__(f"{fn} returned {code}")
        self.code = code


class mr3_params(ctypes.Structure):
    _fields_ = [
        ("gaptol", ctypes.c_double),
        ("bisect_rel", ctypes.c_double),
        ("xi", ctypes.c_double),
        ("k_elg", ctypes.c_double),
        ("k_rs", ctypes.c_double),
        ("max_depth", ctypes.c_int),
        ("rqi_max_iter", ctypes.c_int),
        ("lanes_per_eig", ctypes.c_int),
        ("seed", ctypes.c_ulonglong),
        ("force_rqi_fallback", ctypes.c_int),
        ("force_best_candidate", ctypes.c_int),
        ("profile", ctypes.c_int),
        ("points_per_lane", ctypes.c_int),
        ("gaptol_abs", ctypes.c_double),
        ("initial", ctypes.c_int),
        ("refine_ends", ctypes.c_int),
        ("force_resort", ctypes.c_int),
        ("derive_lld", ctypes.c_int),
    ]


class mr3_stats(ctypes.Structure):
    _fields_ = [
        ("n_eigenpairs", ctypes.c_int64),
        ("n_blocks", ctypes.c_int64),
        ("d_max", ctypes.c_int),
        ("n_clusters", ctypes.c_int64),
        ("largest_cluster", ctypes.c_int64),
        ("n_rqi_iters", ctypes.c_int64),
        ("n_fallbacks", ctypes.c_int64),
        ("n_best_candidate", ctypes.c_int64),
        ("stage_ms", ctypes.c_double * 8),
        ("stage_launches", ctypes.c_int64 * 8),
        ("bisect_row_steps", ctypes.c_double),
        ("rqi_row_steps", ctypes.c_double),
        ("twist_row_steps", ctypes.c_double),
        ("n_dqds_roots", ctypes.c_int64),
        ("dqds_transforms", ctypes.c_int64),
        ("n_sliced_roots", ctypes.c_int64),
        ("n_singleton_first_levels", ctypes.c_int),
        ("n_y_refined", ctypes.c_int64),
        ("n_resorted", ctypes.c_int64),
        ("bisect_count", ctypes.c_int64 * 2),
        ("bisect_rows", ctypes.c_int64 * 2),
        ("bisect_lanes", ctypes.c_int * 2),
    ]


MR3_TUNE_ROOT, MR3_TUNE_CHILD = 0, 1
LANE_CANDIDATES = (1, 2, 3, 4, 6, 8, 12, 16, 24, 32, 64)


class mr3_tune_entry(ctypes.Structure):
    _fields_ = [
        ("stage", ctypes.c_int),
        ("precision", ctypes.c_int),
        ("count_lo", ctypes.c_int64),
        ("count_hi", ctypes.c_int64),
        ("rows_lo", ctypes.c_int64),
        ("rows_hi", ctypes.c_int64),
        ("lanes", ctypes.c_int),
        ("reserved", ctypes.c_int),
    ]


class mr3_range_desc(ctypes.Structure):
    _fields_ = [
        ("range", ctypes.c_int),
        ("vl", ctypes.c_double),
        ("vu", ctypes.c_double),
        ("il", ctypes.c_int64),
        ("iu", ctypes.c_int64),
    ]


class mr3_request(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int),
        ("n", ctypes.c_int64),
        ("d", ctypes.c_void_p),
        ("e", ctypes.c_void_p),
        ("range", mr3_range_desc),
        ("W", ctypes.c_void_p),
        ("Z", ctypes.c_void_p),
        ("ldz", ctypes.c_int64),
        ("stream", ctypes.c_void_p),
    ]


class mr3_result(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("m", ctypes.c_int64),
        ("submit_ms", ctypes.c_double),
        ("start_ms", ctypes.c_double),
        ("done_ms", ctypes.c_double),
        ("batch_id", ctypes.c_int64),
        ("batch_size", ctypes.c_int),
        ("slot", ctypes.c_int),
    ]


# int fn(void* ctx, int64_t count, const mr3_request* reqs, int64_t* m)
EXECUTOR_FN = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_int64,
                               ctypes.POINTER(mr3_request), ctypes.POINTER(ctypes.c_int64))

EXPORTS = [
    "mr3_create", "mr3_destroy", "mr3_default_params", "mr3_set_params", "mr3_get_stats",
    "mr3_solve_f32", "mr3_solve_f64", "mr3_solve_batched", "mr3_check_f64", "mr3_version",
    "mr3_workspace_bytes", "mr3_workspace_min_bytes", "mr3_workspace_bytes_batched",
    "mr3_solve_noalloc", "mr3_set_tuning", "mr3_get_tuning", "mr3_bisect_lanes",
    "mr3_dense_f32", "mr3_dense_f64", "mr3_dense_c64", "mr3_dense_c128",
    "mr3_request_bytes", "mr3_server_create", "mr3_server_create_ex",
    "mr3_server_create_with_executor",
    "mr3_server_submit", "mr3_server_poll", "mr3_server_wait", "mr3_server_destroy",
]

_lib = None


def load_library(path: str | None = None):
    """Load libmr3.so (raises if it is not built)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is not built: run __graft_entry__.build() first")
    lib = ctypes.CDLL(p)
    vp, i64, i32, dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    pi64 = ctypes.POINTER(ctypes.c_int64)
    lib.mr3_create.argtypes = [ctypes.POINTER(vp), i32]
    lib.mr3_destroy.argtypes = [vp]
    lib.mr3_default_params.argtypes = [ctypes.POINTER(mr3_params), i32]
    lib.mr3_set_params.argtypes = [vp, ctypes.POINTER(mr3_params)]
    lib.mr3_get_stats.argtypes = [vp, ctypes.POINTER(mr3_stats)]
    sz = ctypes.c_size_t
    for name in ("mr3_solve_f32", "mr3_solve_f64"):
        getattr(lib, name).argtypes = [vp, i64, vp, vp, i32, dbl, dbl, i64, i64, pi64, vp, vp, i64,
                                       vp, sz, vp]
    lib.mr3_solve_batched.argtypes = [vp, i64, i32, pi64, pi64, vp, vp,
                                      ctypes.POINTER(mr3_range_desc), pi64, vp, pi64, vp, pi64,
                                      pi64, vp, sz, vp]
    lib.mr3_workspace_bytes.argtypes = [vp, i64, i32, i64, i32]
    lib.mr3_workspace_min_bytes.argtypes = [vp, i64, i32, i64, i32]
    lib.mr3_workspace_bytes_batched.argtypes = [vp, i64, i32, pi64, ctypes.POINTER(mr3_range_desc)]
    lib.mr3_solve_noalloc.argtypes = [vp, i32, i64, vp, vp, i32, dbl, dbl, i64, i64, pi64, vp, vp,
                                      i64, vp]
    for name in ("mr3_dense_f32", "mr3_dense_f64", "mr3_dense_c64", "mr3_dense_c128"):
        getattr(lib, name).argtypes = [vp, i64, vp, i64, i32, dbl, dbl, i64, i64, pi64, vp, vp,
                                       i64, vp]
    lib.mr3_set_tuning.argtypes = [vp, ctypes.POINTER(mr3_tune_entry), i32]
    lib.mr3_get_tuning.argtypes = [vp, ctypes.POINTER(mr3_tune_entry), i32]
    lib.mr3_bisect_lanes.argtypes = [vp, i32, i32, i64, i64]
    lib.mr3_check_f64.argtypes = [vp, i64, i64, vp, vp, vp, vp, i64,
                                  ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), vp]
    lib.mr3_request_bytes.argtypes = [i64, i64, i32]
    lib.mr3_server_create.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_size_t, i32]
    lib.mr3_server_create_ex.argtypes = [ctypes.POINTER(vp), vp, ctypes.c_size_t, i32, i32]
    lib.mr3_server_create_with_executor.argtypes = [ctypes.POINTER(vp), EXECUTOR_FN, vp,
                                                    ctypes.c_size_t, i32, i32]
    lib.mr3_server_submit.argtypes = [vp, ctypes.POINTER(mr3_request), ctypes.POINTER(ctypes.c_uint64)]
    lib.mr3_server_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int)]
    lib.mr3_server_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(mr3_result)]
    lib.mr3_server_destroy.argtypes = [vp]
    lib.mr3_version.restype = ctypes.c_char_p
    for name in EXPORTS:
        if name != "mr3_version":
            getattr(lib, name).restype = ctypes.c_int
    for name in ("mr3_request_bytes", "mr3_workspace_bytes", "mr3_workspace_min_bytes",
                 "mr3_workspace_bytes_batched"):
        getattr(lib, name).restype = ctypes.c_size_t
    if path is None:
        _lib = lib
    return lib


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _check(fn, rc):
    if rc != MR3_OK:
        raise MR3Error(fn, rc)


class Handle:
    """Owns an mr3_handle (device, parameters, workspace pool)."""

    def __init__(self, device: int | None = None):
        lib = load_library()
        if device is None:
            device = torch.cuda.current_device() if torch.cuda.is_available() else 0
        self._h = ctypes.c_void_p()
        _check("mr3_create", lib.mr3_create(ctypes.byref(self._h), int(device)))
        self.device = device

    def close(self):
        if self._h:
            load_library().mr3_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def ptr(self):
        return self._h

    def set_params(self, **kw):
        p = default_params(kw.pop("precision", 64))
        for k, v in kw.items():
            setattr(p, k, v)
        _check("mr3_set_params", load_library().mr3_set_params(self._h, ctypes.byref(p)))

    def reset_params(self):
        _check("mr3_set_params", load_library().mr3_set_params(self._h, None))

    def set_tuning(self, entries=None):
        """Replace the handle's multisection tuning table: a list of
        (stage, precision, count_lo, count_hi, rows_lo, rows_hi, lanes)
        tuples ([] = no table), or None for the built-in table."""
        lib = load_library()
        if entries is None:
            _check("mr3_set_tuning", lib.mr3_set_tuning(self._h, None, -1))
            return
        arr = (mr3_tune_entry * max(len(entries), 1))()
        for i, t in enumerate(entries):
            arr[i] = mr3_tune_entry(*t, 0)
        _check("mr3_set_tuning", lib.mr3_set_tuning(self._h, arr, len(entries)))

    def tuning(self) -> list:
        """The handle's tuning table as a list of 7-tuples."""
        lib = load_library()
        nt = lib.mr3_get_tuning(self._h, None, 0)
        arr = (mr3_tune_entry * max(nt, 1))()
        lib.mr3_get_tuning(self._h, arr, nt)
        return [(t.stage, t.precision, t.count_lo, t.count_hi, t.rows_lo, t.rows_hi, t.lanes)
                for t in arr[:nt]]

    def bisect_lanes(self, stage: int, precision: int, count: int, rows: int) -> int:
        """Lanes per eigenvalue from the override or the table (0: size rule)."""
        r = load_library().mr3_bisect_lanes(self._h, stage, precision, count, rows)
        if r < 0:
            raise MR3Error("mr3_bisect_lanes", r)
        return r

    def stats(self) -> dict:
        s = mr3_stats()
        _check("mr3_get_stats", load_library().mr3_get_stats(self._h, ctypes.byref(s)))
        out = {}
        for f, _ in mr3_stats._fields_:
            v = getattr(s, f)
            out[f] = list(v) if hasattr(v, "__len__") else v
        return out


def default_params(precision: int = 64) -> mr3_params:
    p = mr3_params()
    _check("mr3_default_params", load_library().mr3_default_params(ctypes.byref(p), precision))
    return p


_default_handle = None


def default_handle() -> Handle:
    global _default_handle
    if _default_handle is None:
        _default_handle = Handle()
    return _default_handle


# --------------------------------------------------------------------------
# same-name wrappers of the C entry points
# --------------------------------------------------------------------------
def _work(work):
    """(pointer, bytes) of a work region: None, or a device tensor (uint8)."""
    if work is None:
        return None, 0
    return ctypes.c_void_p(work.data_ptr()), work.numel() * work.element_size()


def mr3_solve_f32(h, n, d, e, range_, vl, vu, il, iu, W, Z, ldz, stream=None, work=None) -> int:
    m = ctypes.c_int64(0)
    wp, wb = _work(work)
    rc = load_library().mr3_solve_f32(h.ptr, n, _ptr(d), _ptr(e), range_, vl, vu, il, iu,
                                      ctypes.byref(m), _ptr(W), _ptr(Z), ldz, wp, wb,
                                      _stream_ptr(stream))
    _check("mr3_solve_f32", rc)
    return m.value


def mr3_solve_f64(h, n, d, e, range_, vl, vu, il, iu, W, Z, ldz, stream=None, work=None) -> int:
    m = ctypes.c_int64(0)
    wp, wb = _work(work)
    rc = load_library().mr3_solve_f64(h.ptr, n, _ptr(d), _ptr(e), range_, vl, vu, il, iu,
                                      ctypes.byref(m), _ptr(W), _ptr(Z), ldz, wp, wb,
                                      _stream_ptr(stream))
    _check("mr3_solve_f64", rc)
    return m.value


def mr3_solve_noalloc(h, precision, n, d, e, range_, vl, vu, il, iu, W, Z, ldz, stream=None) -> int:
    m = ctypes.c_int64(0)
    rc = load_library().mr3_solve_noalloc(h.ptr, precision, n, _ptr(d), _ptr(e), range_, vl, vu,
                                          il, iu, ctypes.byref(m), _ptr(W), _ptr(Z), ldz,
                                          _stream_ptr(stream))
    _check("mr3_solve_noalloc", rc)
    return m.value


def mr3_workspace_bytes(h, n: int, range_: int, k_max: int, precision: int) -> int:
    return int(load_library().mr3_workspace_bytes(h.ptr if h is not None else None, n, range_,
                                                  k_max, precision))


def mr3_workspace_min_bytes(h, n: int, range_: int, k_max: int, precision: int) -> int:
    return int(load_library().mr3_workspace_min_bytes(h.ptr if h is not None else None, n, range_,
                                                      k_max, precision))


def mr3_workspace_bytes_batched(h, precision: int, n, ranges=None) -> int:
    count = len(n)
    n_a = (ctypes.c_int64 * count)(*n)
    rg = None
    if ranges is not None:
        rg = (mr3_range_desc * count)()
        for p, r in enumerate(ranges):
            rg[p].range, rg[p].vl, rg[p].vu, rg[p].il, rg[p].iu = r
    return int(load_library().mr3_workspace_bytes_batched(h.ptr if h is not None else None, count,
                                                          precision, n_a, rg))


def mr3_check_f64(h, n, m, d, e, W, Z, ldz, stream=None):
    orth = (ctypes.c_double * 2)()
    res = (ctypes.c_double * 1)()
    rc = load_library().mr3_check_f64(h.ptr, n, m, _ptr(d), _ptr(e), _ptr(W), _ptr(Z), ldz,
                                      orth, res, _stream_ptr(stream))
    _check("mr3_check_f64", rc)
    return (orth[0], orth[1]), res[0]


def _i64(x, count):
    """A host int64 array of `count` entries (numpy arrays of that type pass
    without a copy) and the pointer the C call takes."""
    a = np.ascontiguousarray(x, dtype=np.int64)
    if a.shape != (count,):
        raise ValueError(f"expected {count} entries, got shape {a.shape}")
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def mr3_solve_batched(h, count, precision, n, de_off, d, e, ranges, W, w_off, Z, z_off, ldz,
                      stream=None, work=None):
    """Per-problem host arguments (n, de_off, w_off, z_off, ldz) may be lists
    or int64 numpy arrays; returns the eigenpair counts m as a list."""
    keep = []
    def arr(x):
        a, ptr = _i64(x, count)
        keep.append(a)
        return ptr
    n_a, de_a, wo_a = arr(n), arr(de_off), arr(w_off)
    zo_a = arr(z_off) if Z is not None else None
    ld_a = arr(ldz) if Z is not None else None
    m_np = np.zeros(count, dtype=np.int64)
    m_a = m_np.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
    rg = None
    if ranges is not None:
        rg = (mr3_range_desc * count)()
        for p, r in enumerate(ranges):
            rg[p].range, rg[p].vl, rg[p].vu, rg[p].il, rg[p].iu = r
    wp, wb = _work(work)
    rc = load_library().mr3_solve_batched(h.ptr, count, precision, n_a, de_a, _ptr(d), _ptr(e), rg,
                                          m_a, _ptr(W), wo_a, _ptr(Z), zo_a, ld_a, wp, wb,
                                          _stream_ptr(stream))
    _check("mr3_solve_batched", rc)
    return m_np.tolist()


# --------------------------------------------------------------------------
# convenience wrappers
# --------------------------------------------------------------------------
_RANGES = {"all": RANGE_ALL, "value": RANGE_VALUE, "index": RANGE_INDEX}


def solve(d: torch.Tensor, e: torch.Tensor, range: str = "all", vl: float = 0.0, vu: float = 0.0,
          il: int = 1, iu: int | None = None, vectors: bool = True, handle: Handle | None = None,
          stream=None, work: torch.Tensor | None = None, noalloc: bool = False):
    """Eigenpairs of the tridiagonal (d, e); returns (W[m], Z[n, m] or None).
    work: a device tensor used as the call's work region (None: the handle's
    pool); noalloc: run mr3_solve_noalloc (the library's static scratch)."""
    if not d.is_cuda:
        raise ValueError("d and e must be device tensors")
    h = handle or default_handle()
    n = d.numel()
    if iu is None:
        iu = n
    rk = _RANGES[range]
    cap = n if rk != RANGE_INDEX else max(iu - il + 1, 0)
    W = torch.empty(max(cap, 1), dtype=d.dtype, device=d.device)
    # column-major n x cap == row-major (cap, n)
    Zt = torch.empty((max(cap, 1), max(n, 1)), dtype=d.dtype, device=d.device) if vectors else None
    fn = mr3_solve_f32 if d.dtype == torch.float32 else mr3_solve_f64
    if d.dtype not in (torch.float32, torch.float64) or e.dtype != d.dtype:
        raise ValueError("d and e must both be float32 or both float64")
    dc, ec = d.contiguous(), (e.contiguous() if n > 1 else None)
    if noalloc:
        prec = 32 if d.dtype == torch.float32 else 64
        m = mr3_solve_noalloc(h, prec, n, dc, ec, rk, vl, vu, il, iu, W, Zt, max(n, 1), stream)
    else:
        m = fn(h, n, dc, ec, rk, vl, vu, il, iu, W, Zt, max(n, 1), stream, work)
    W = W[:m]
    Z = Zt[:m].T if vectors else None
    return W, Z


def dense(A: torch.Tensor, range: str = "all", vl: float = 0.0, vu: float = 0.0, il: int = 1,
          iu: int | None = None, vectors: bool = True, handle: Handle | None = None, stream=None):
    """Eigenpairs of the dense symmetric (float32, float64) or Hermitian
    (complex64, complex128) device matrix A (its lower triangle is read; A itself is not
    modified): reduction to tridiagonal form, this library's solver,
    back-transformation.  Returns (W[m], Z[n, m] or None)."""
    if not A.is_cuda or A.dim() != 2 or A.shape[0] != A.shape[1]:
        raise ValueError("A must be a square device matrix")
    fns = {torch.float32: mr3_dense_f32, torch.float64: mr3_dense_f64,
           torch.complex64: mr3_dense_c64, torch.complex128: mr3_dense_c128}
    if A.dtype not in fns:
        raise ValueError("A must be float32, float64, complex64 or complex128")
    h = handle or default_handle()
    n = A.shape[0]
    if iu is None:
        iu = n
    rk = _RANGES[range]
    cap = n if rk != RANGE_INDEX else max(iu - il + 1, 0)
    Ac = A.t().contiguous()  # row-major storage of A^T is column-major A
    wdt = torch.float32 if A.dtype in (torch.float32, torch.complex64) else torch.float64
    W = torch.empty(max(cap, 1), dtype=wdt, device=A.device)
    Zt = torch.empty((max(cap, 1), max(n, 1)), dtype=A.dtype, device=A.device) if vectors else None
    m = fns[A.dtype](h, n, Ac, max(n, 1), rk, vl, vu, il, iu, W, Zt, max(n, 1), stream)
    return W[:m], (Zt[:m].T if vectors else None)


def _dense_raw(name):
    def call(h, n, A, lda, range_, vl, vu, il, iu, W, Z, ldz, stream=None) -> int:
        m = ctypes.c_int64(0)
        hp = h.ptr if isinstance(h, Handle) else h
        _check(name, getattr(load_library(), name)(hp, n, _ptr(A), lda, range_, vl, vu, il, iu,
                                                   ctypes.byref(m), _ptr(W), _ptr(Z), ldz,
                                                   _stream_ptr(stream)))
        return m.value
    call.__name__ = name
    return call


mr3_dense_f32 = _dense_raw("mr3_dense_f32")
mr3_dense_f64 = _dense_raw("mr3_dense_f64")
mr3_dense_c64 = _dense_raw("mr3_dense_c64")
mr3_dense_c128 = _dense_raw("mr3_dense_c128")


def solve_batched(ds, es, ranges=None, vectors: bool = True, handle: Handle | None = None,
                  stream=None, work: torch.Tensor | None = None):
    """Solve many problems (lists of 1-D device tensors of one dtype) in one
    pass.  Returns lists of W and Z (Z[p] is n_p x m_p)."""
    h = handle or default_handle()
    dtype = ds[0].dtype
    dev = ds[0].device
    count = len(ds)
    n = [int(x.numel()) for x in ds]
    off, o = [], 0
    for k in n:
        off.append(o)
        o += k
    dcat = torch.cat([x.reshape(-1) for x in ds]) if o else torch.empty(1, dtype=dtype, device=dev)
    ecat = torch.zeros(max(o, 1), dtype=dtype, device=dev)
    for p, x in enumerate(es):
        if n[p] > 1:
            ecat[off[p]:off[p] + n[p] - 1] = x.reshape(-1)[: n[p] - 1]
    caps = []
    for p in range(count):
        if ranges is not None and ranges[p][0] == RANGE_INDEX:
            caps.append(max(ranges[p][4] - ranges[p][3] + 1, 0))
        else:
            caps.append(n[p])
    w_off, z_off, acc_w, acc_z = [], [], 0, 0
    for p in range(count):
        w_off.append(acc_w)
        z_off.append(acc_z)
        acc_w += caps[p]
        acc_z += caps[p] * n[p]
    W = torch.empty(max(acc_w, 1), dtype=dtype, device=dev)
    Z = torch.empty(max(acc_z, 1), dtype=dtype, device=dev) if vectors else None
    ldz = [max(k, 1) for k in n]
    ms = mr3_solve_batched(h, count, 32 if dtype == torch.float32 else 64, n, off, dcat, ecat,
                           ranges, W, w_off, Z, z_off, ldz, stream, work)
    Ws = [W[w_off[p]:w_off[p] + ms[p]] for p in range(count)]
    Zs = None
    if vectors:
        Zs = [Z[z_off[p]:z_off[p] + ms[p] * n[p]].view(ms[p], n[p]).T for p in range(count)]
    return Ws, Zs


def check(d: torch.Tensor, e: torch.Tensor, W: torch.Tensor, Z: torch.Tensor,
          handle: Handle | None = None, stream=None):
    """(max off-diagonal |Z^T Z|, max |diag - 1|), max ||T z - lambda z||_1/||T||_1
    for FP64 results, computed on the device (FP64 MFMA Gram matrix)."""
    h = handle or default_handle()
    n, m = d.numel(), W.numel()
    Zcm = Z.T.contiguous()  # (m, n) row-major == n x m column-major, ldz = n
    return mr3_check_f64(h, n, m, d.contiguous(), e.contiguous() if n > 1 else None,
                         W.contiguous(), Zcm, max(n, 1), stream)


def version() -> str:
    return load_library().mr3_version().decode()


# --------------------------------------------------------------------------
# serving
# --------------------------------------------------------------------------
def mr3_request_bytes(n: int, k: int, precision: int) -> int:
    return int(load_library().mr3_request_bytes(n, k, precision))


def mr3_server_create(h, hbm_budget_bytes: int, max_batch: int):
    s = ctypes.c_void_p()
    _check("mr3_server_create",
           load_library().mr3_server_create(ctypes.byref(s), h.ptr, hbm_budget_bytes, max_batch))
    return s


def mr3_server_create_ex(h, hbm_budget_bytes: int, max_batch: int, max_inflight: int):
    s = ctypes.c_void_p()
    _check("mr3_server_create_ex",
           load_library().mr3_server_create_ex(ctypes.byref(s), h.ptr, hbm_budget_bytes, max_batch,
                                               max_inflight))
    return s


def mr3_server_create_with_executor(fn, ctx, hbm_budget_bytes: int, max_batch: int,
                                    max_inflight: int = 1):
    s = ctypes.c_void_p()
    _check("mr3_server_create_with_executor",
           load_library().mr3_server_create_with_executor(ctypes.byref(s), fn, ctx,
                                                          hbm_budget_bytes, max_batch, max_inflight))
    return s


def mr3_server_submit(s, req: mr3_request) -> int:
    t = ctypes.c_uint64(0)
    _check("mr3_server_submit", load_library().mr3_server_submit(s, ctypes.byref(req), ctypes.byref(t)))
    return t.value


def mr3_server_poll(s, ticket: int) -> bool:
    done = ctypes.c_int(0)
    _check("mr3_server_poll", load_library().mr3_server_poll(s, ticket, ctypes.byref(done)))
    return bool(done.value)


def mr3_server_wait(s, ticket: int) -> dict:
    r = mr3_result()
    rc = load_library().mr3_server_wait(s, ticket, ctypes.byref(r))
    if rc < 0:
        raise MR3Error("mr3_server_wait", rc)
    return {f: getattr(r, f) for f, _ in mr3_result._fields_}


def mr3_server_destroy(s) -> None:
    _check("mr3_server_destroy", load_library().mr3_server_destroy(s))


def make_request(d, e, W, Z=None, range: str = "all", vl: float = 0.0, vu: float = 0.0,
                 il: int = 1, iu: int | None = None, stream=None) -> mr3_request:
    """Request for tensors d, e (inputs) and W, Z (outputs, Z an (m, n)
    row-major == n x m column-major buffer or None); the solve is ordered
    after the work queued on `stream` (default: torch's current stream)."""
    n = d.numel()
    r = mr3_request()
    r.precision = 32 if d.dtype == torch.float32 else 64
    r.n = n
    r.d = d.data_ptr()
    r.e = e.data_ptr() if (e is not None and n > 1) else None
    r.range.range = _RANGES[range]
    r.range.vl, r.range.vu = vl, vu
    r.range.il, r.range.iu = il, (n if iu is None else iu)
    r.W = W.data_ptr()
    r.Z = Z.data_ptr() if Z is not None else None
    r.ldz = max(n, 1)
    if d.is_cuda:
        r.stream = _stream_ptr(stream).value
    return r


class Server:
    """Continuous-batching server over a handle (which it takes over while it
    lives).  submit() returns a ticket; the tensors of a request are kept
    alive by the server until wait() has returned for it."""

    def __init__(self, handle: Handle | None = None, hbm_budget_bytes: int | None = None,
                 max_batch: int = 256, max_inflight: int = 2):
        self.handle = handle or Handle()
        if hbm_budget_bytes is None:
            free, _ = torch.cuda.mem_get_info(self.handle.device)
            hbm_budget_bytes = free // 2
        self.budget = int(hbm_budget_bytes)
        self._s = mr3_server_create_ex(self.handle, self.budget, max_batch, max_inflight)
        self._keep = {}

    def submit(self, d, e, range: str = "all", vl: float = 0.0, vu: float = 0.0, il: int = 1,
               iu: int | None = None, vectors: bool = True):
        n = d.numel()
        if iu is None:
            iu = n
        cap = n if range != "index" else max(iu - il + 1, 0)
        W = torch.empty(max(cap, 1), dtype=d.dtype, device=d.device)
        Z = torch.empty((max(cap, 1), max(n, 1)), dtype=d.dtype, device=d.device) if vectors else None
        req = make_request(d, e, W, Z, range, vl, vu, il, iu)
        t = mr3_server_submit(self._s, req)
        self._keep[t] = (d, e, W, Z)
        return t

    def poll(self, ticket: int) -> bool:
        return mr3_server_poll(self._s, ticket)

    def wait(self, ticket: int):
        """-> (result dict, W[m], Z[n, m] or None)"""
        res = mr3_server_wait(self._s, ticket)
        d, e, W, Z = self._keep.pop(ticket)
        if res["status"] != MR3_OK:
            raise MR3Error("mr3_server_wait", res["status"])
        m = res["m"]
        return res, W[:m], (Z[:m].T if Z is not None else None)

    def close(self):
        if self._s:
            mr3_server_destroy(self._s)
            self._s = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
