"""Python binding of libfespmv (FP64 FEM SpMV and CG on MI355X).

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libfespmv.so``.  PyTorch supplies device memory and streams;
the names mirror the C ABI in ``include/fespmv.h``.

There is no CPU fallback: if the library cannot be built or loaded, or no
GPU is present, the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import sys as _sys

from . import _build

FS_OK, FS_E_ARG, FS_E_BAD_CSR, FS_E_NOT_SQUARE, FS_E_OOM, FS_E_BUDGET, \
    FS_E_HIP, FS_E_NOT_CONVERGED, FS_E_BREAKDOWN, FS_E_UNSUPPORTED = range(10)
STATUS_NAMES = {0: "FS_OK", 1: "FS_E_ARG", 2: "FS_E_BAD_CSR",
                3: "FS_E_NOT_SQUARE", 4: "FS_E_OOM", 5: "FS_E_BUDGET",
                6: "FS_E_HIP", 7: "FS_E_NOT_CONVERGED", 8: "FS_E_BREAKDOWN",
                9: "FS_E_UNSUPPORTED"}
REORDER_AUTO, REORDER_NONE, REORDER_RCM, REORDER_USER = range(4)
BUILD_DEVICE, BUILD_HOST = 0, 1
BUILD_DEVICE_MAX_ROW = 4096
DT_F64, DT_F32, DT_BF16 = 1, 2, 4
ASM_AUTO, ASM_GATHER, ASM_ROWGROUP = 0, 1, 2
PC_NONE, PC_JACOBI = 0, 1
PREC_F64, PREC_IR_F32, PREC_IR_BF16 = 0, 1, 2
TO_LAYOUT, FROM_LAYOUT = 0, 1


class FsError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), msg))
        self.status = status


class CsrOpts(C.Structure):
    _fields_ = [("reorder", C.c_int32), ("perm", C.c_void_p),
                ("sort_window", C.c_int32), ("threshold", C.c_int32),
                ("lanes_min", C.c_int32), ("lanes_max", C.c_int32),
                ("dtypes", C.c_int32), ("vec", C.c_int32),
                ("index_bits", C.c_int32), ("autotune", C.c_int32),
                ("build", C.c_int32), ("reserved", C.c_int32 * 4)]


class CsrStats(C.Structure):
    _fields_ = [("n_rows", C.c_int32), ("n_cols", C.c_int32),
                ("nnz", C.c_int64), ("slots", C.c_int64),
                ("n_groups", C.c_int32), ("reorder", C.c_int32),
                ("padding", C.c_double), ("bytes_algorithmic", C.c_int64),
                ("bytes_layout", C.c_int64),
                ("groups_by_lanes", C.c_int32 * 7), ("dtypes", C.c_int32),
                ("vec", C.c_int32), ("mean_band_before", C.c_double),
                ("mean_band_after", C.c_double),
                ("t_build_ms", C.c_double), ("device_bytes", C.c_int64),
                ("tuned", C.c_int32), ("tune_candidates", C.c_int32),
                ("tune_best_us", C.c_double), ("index_bits", C.c_int32),
                ("build", C.c_int32)]

    def as_dict(self):
        d = {}
        for name, _ in self._fields_:
            v = getattr(self, name)
            d[name] = list(v) if name == "groups_by_lanes" else v
        return d


class CgOpts(C.Structure):
    _fields_ = [("rtol", C.c_double), ("maxit", C.c_int32),
                ("precond", C.c_int32), ("precision", C.c_int32),
                ("inner_rtol", C.c_double), ("check_every", C.c_int32),
                ("x0_zero", C.c_int32), ("use_graph", C.c_int32),
                ("max_outer", C.c_int32), ("ir_restart", C.c_int32),
                ("ir_scaled", C.c_int32), ("estimate_cond", C.c_int32),
                ("wg_threads", C.c_int32), ("reserved", C.c_int32 * 2)]


class CgInfo(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32),
                ("outer", C.c_int32), ("replacements", C.c_int32),
                ("relres", C.c_double), ("ms", C.c_double),
                ("bytes", C.c_double), ("cond_est", C.c_double)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class AsmStats(C.Structure):
    _fields_ = [("n_elem", C.c_int32), ("nde", C.c_int32),
                ("contrib_matrix", C.c_int64), ("contrib_vector", C.c_int64),
                ("stored_matrix", C.c_int64), ("stored_vector", C.c_int64),
                ("bytes_algorithmic_matrix", C.c_int64),
                ("bytes_algorithmic_vector", C.c_int64),
                ("device_bytes", C.c_int64), ("t_build_ms", C.c_double),
                ("plan", C.c_int32), ("reserved", C.c_int32 * 7)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_
                if n != "reserved"}


# every symbol include/fespmv.h declares
EXPORTS = ["fs_last_error", "csr_opts_default", "csr_create",
           "csr_layout_host",
           "csr_update_values", "csr_add_dtype", "csr_info", "csr_get_perm",
           "csr_get_layout",
           "csr_destroy", "spmv", "spmv_csr", "spmv_batch", "spmv_perm",
           "probe_read_bandwidth",
           "csr_permute",
           "spmm",
           "spmv_lowp", "cg_opts_default", "cg_solve", "cg_solve_async",
           "cg_solve_async_noalloc",
           "cg_solve_multi",
           "cg_solve_batch", "cg_solve_batch_wg",
           "server_opts_default", "server_create",
           "server_submit", "server_poll", "server_stats", "server_destroy",
           "asm_create", "asm_plan_host", "asm_plan_host_groups",
           "asm_matrix", "asm_vector", "asm_system", "asm_element_rows",
           "asm_matrix_ordered",
           "asm_info",
           "asm_destroy", "csr_get_values"]

_lib = None


def lib_path():
    """The library this process loads: libfespmv.so, or the file named by
    the FESPMV_LIB environment variable (e.g. the sanitizer build)."""
    return os.environ.get("FESPMV_LIB") or _build.LIB


def load(build_if_missing=True):
    """Load libfespmv.so (building it with hipcc when absent or stale)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if path == _build.LIB and build_if_missing and _build.needs_build():
        _build.build()
    if not os.path.exists(path):
        raise FsError(FS_E_HIP, "%s is not built" % os.path.basename(path))
    L = C.CDLL(path)
    vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
    P = C.POINTER
    L.fs_last_error.restype = C.c_char_p
    L.fs_last_error.argtypes = []
    sigs = {
        "csr_opts_default": [P(CsrOpts)],
        "csr_create": [i32, i32, i64, vp, vp, vp, P(CsrOpts), vp, P(vp)],
        "csr_layout_host": [i32, i32, i64, vp, vp, P(CsrOpts), P(i32),
                            P(i64), P(i32), vp, vp, vp, vp],
        "csr_update_values": [vp, vp, vp],
        "csr_add_dtype": [vp, i32, vp],
        "csr_info": [vp, P(CsrStats)],
        "csr_get_perm": [vp, vp],
        "csr_get_layout": [vp, vp, vp, vp, vp, vp],
        "csr_destroy": [vp],
        "spmv": [vp, vp, vp, vp],
        "spmv_batch": [i32, vp, vp, vp, vp],
        "spmv_csr": [i32, i32, i64, vp, vp, vp, vp, vp, vp],
        "probe_read_bandwidth": [vp, i64, vp, i32, vp],
        "spmv_perm": [vp, vp, vp, vp],
        "csr_permute": [vp, i32, vp, vp, vp],
        "spmm": [vp, i32, vp, i64, vp, i64, vp],
        "spmv_lowp": [vp, i32, vp, vp, vp],
        "cg_opts_default": [P(CgOpts)],
        "cg_solve": [vp, vp, vp, P(CgOpts), P(CgInfo), vp],
        "cg_solve_async": [vp, vp, vp, P(CgOpts), vp, vp],
        "cg_solve_async_noalloc": [vp, vp, vp, P(CgOpts), vp, vp],
        "cg_solve_multi": [vp, i32, vp, i64, vp, i64, P(CgOpts), P(CgInfo),
                           vp],
        "cg_solve_batch": [i32, vp, vp, vp, vp, P(CgOpts), P(CgInfo), vp],
        "cg_solve_batch_wg": [i32, vp, vp, vp, P(CgOpts), P(CgInfo), vp],
        "asm_create": [vp, i32, i32, vp, i32, vp, P(vp)],
        "asm_plan_host_groups": [i32, i64, vp, vp, P(CsrOpts), i32, i32, vp,
                                 P(i32), P(i32), P(i64), P(i64), P(i32), vp,
                                 vp, vp, vp],
        "asm_plan_host": [i32, i64, vp, vp, P(CsrOpts), i32, i32, vp, i32,
                          P(i64), P(i32), P(i64), vp, vp, vp],
        "asm_matrix": [vp, vp, vp],
        "asm_vector": [vp, vp, vp, vp],
        "asm_system": [vp, vp, vp, vp, vp],
        "asm_element_rows": [vp, vp, P(i64)],
        "asm_matrix_ordered": [vp, vp, vp],
        "asm_info": [vp, P(AsmStats)],
        "asm_destroy": [vp],
        "csr_get_values": [vp, vp, vp],
    }
    for name, args in sigs.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int32
    _lib = L
    return L


def last_error():
    return load().fs_last_error().decode()


def _check(status):
    if status != FS_OK:
        raise FsError(status, last_error())
    return status


def _stream(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def _ptr(t, dtype=None, n=None, name="tensor"):
    """Device pointer of a contiguous CUDA tensor (checked)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise FsError(FS_E_ARG, "%s must be a device tensor" % name)
    if not t.is_contiguous():
        raise FsError(FS_E_ARG, "%s must be contiguous" % name)
    if dtype is not None and t.dtype != dtype:
        raise FsError(FS_E_ARG, "%s must be %s" % (name, dtype))
    if n is not None and t.numel() != n:
        raise FsError(FS_E_ARG, "%s has %d entries, expected %d"
                      % (name, t.numel(), n))
    return t.data_ptr() if t.numel() else None


def _finalize(close, _is_finalizing=_sys.is_finalizing):
    """Release a handle from a finalizer.  While the interpreter shuts down
    the HIP runtime (and any tool attached to it) may already be gone, so
    nothing is released then: the process exit returns the memory.  Owners
    that want a clean teardown call close() themselves.  (Everything used
    here is bound when the module loads: module globals may already be
    cleared when a finalizer runs at shutdown.)"""
    if _is_finalizing():
        return
    try:
        close()
    except Exception:
        pass


class Matrix:
    """Owning wrapper of an fs_csr_t handle."""

    def __init__(self, handle, n_rows, n_cols, nnz):
        self.handle = handle
        self.n_rows, self.n_cols, self.nnz = n_rows, n_cols, nnz

    def __del__(self, _fin=_finalize):
        _fin(self.close)

    def close(self):
        if self.handle:
            load().csr_destroy(self.handle)
            self.handle = None

    @property
    def _h(self):
        if not self.handle:
            raise FsError(FS_E_ARG, "matrix handle already destroyed")
        return self.handle


def csr_opts(**kw):
    o = CsrOpts()
    load().csr_opts_default(C.byref(o))
    perm = kw.pop("perm", None)
    for k, v in kw.items():
        setattr(o, k, v)
    if perm is not None:
        import numpy as np
        arr = np.ascontiguousarray(perm, dtype=np.int32)
        o._perm_keep = arr
        o.perm = arr.ctypes.data
        o.reorder = REORDER_USER
    return o


def csr_create(rowptr, col, val, n_rows=None, n_cols=None, stream=None,
               **opts):
    """Build the layout from device CSR tensors (int32, int32, float64)."""
    import torch
    L = load()
    n_rows = rowptr.numel() - 1 if n_rows is None else n_rows
    n_cols = n_rows if n_cols is None else n_cols
    nnz = col.numel()
    o = csr_opts(**opts)
    h = C.c_void_p()
    _check(L.csr_create(n_rows, n_cols, nnz,
                        _ptr(rowptr, torch.int32, n_rows + 1, "rowptr"),
                        _ptr(col, torch.int32, None, "col"),
                        _ptr(val, torch.float64, nnz, "val"),
                        C.byref(o), _stream(stream), C.byref(h)))
    return Matrix(h.value, n_rows, n_cols, nnz)


def csr_layout_host(rowptr, col, n_rows=None, n_cols=None, **opts):
    """Host-only layout dry run on numpy arrays; returns a dict with
    groups (n_groups x 4), slot_col, map and perm."""
    import numpy as np
    L = load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    n_rows = len(rowptr) - 1 if n_rows is None else n_rows
    n_cols = n_rows if n_cols is None else n_cols
    o = csr_opts(**opts)
    ng = C.c_int32()
    ns = C.c_int64()
    nv = C.c_int32()
    _check(L.csr_layout_host(n_rows, n_cols, len(col), rowptr.ctypes.data,
                             col.ctypes.data, C.byref(o), C.byref(ng),
                             C.byref(ns), C.byref(nv), None, None, None,
                             None))
    groups = np.zeros((ng.value, 4), dtype=np.int32)
    slot_col = np.zeros(ns.value, dtype=np.int32)
    mp = np.zeros(len(col), dtype=np.int32)
    perm = np.zeros(n_rows, dtype=np.int32)
    _check(L.csr_layout_host(n_rows, n_cols, len(col), rowptr.ctypes.data,
                             col.ctypes.data, C.byref(o), C.byref(ng),
                             C.byref(ns), C.byref(nv), groups.ctypes.data,
                             slot_col.ctypes.data, mp.ctypes.data,
                             perm.ctypes.data))
    return dict(groups=groups, slot_col=slot_col, map=mp, perm=perm,
                slots=ns.value, vec=nv.value)


def csr_update_values(A, val, stream=None):
    import torch
    _check(load().csr_update_values(A._h, _ptr(val, torch.float64, A.nnz,
                                                 "val"), _stream(stream)))


def csr_get_values(A, out=None, stream=None):
    """A's FP64 values in the CSR order csr_create saw (device tensor)."""
    import torch
    if out is None:
        out = torch.empty(A.nnz, dtype=torch.float64, device="cuda")
    _check(load().csr_get_values(A._h, _ptr(out, torch.float64, A.nnz,
                                              "out"), _stream(stream)))
    return out


def csr_add_dtype(A, dtype, stream=None):
    _check(load().csr_add_dtype(A._h, int(dtype), _stream(stream)))


def csr_info(A):
    st = CsrStats()
    _check(load().csr_info(A._h, C.byref(st)))
    return st.as_dict()


def csr_get_perm(A):
    import numpy as np
    out = np.empty(A.n_rows, dtype=np.int32)
    _check(load().csr_get_perm(A._h, out.ctypes.data))
    return out


def csr_get_layout(A):
    """The handle's device layout copied to numpy: groups (n_groups x 4),
    slot_col, map, and col16 / gbase for a 16-bit layout (else None)."""
    import numpy as np
    st = csr_info(A)
    groups = np.empty((st["n_groups"], 4), dtype=np.int32)
    slot_col = np.empty(st["slots"], dtype=np.int32)
    mp = np.empty(st["nnz"], dtype=np.int32)
    narrow = st["index_bits"] == 16
    col16 = np.empty(st["slots"], dtype=np.uint16) if narrow else None
    gbase = np.empty(st["n_groups"], dtype=np.int32) if narrow else None
    _check(load().csr_get_layout(
        A._h, groups.ctypes.data, slot_col.ctypes.data, mp.ctypes.data,
        col16.ctypes.data if narrow else None,
        gbase.ctypes.data if narrow else None))
    return dict(groups=groups, slot_col=slot_col, map=mp, col16=col16,
                gbase=gbase)


def csr_destroy(A):
    A.close()


def spmv(A, x, y=None, stream=None):
    import torch
    if y is None:
        y = torch.empty(A.n_rows, dtype=torch.float64, device=x.device)
    _check(load().spmv(A._h, _ptr(x, torch.float64, A.n_cols, "x"),
                       _ptr(y, torch.float64, A.n_rows, "y"),
                       _stream(stream)))
    return y


def spmv_csr(rowptr, col, val, n_rows, n_cols, x, y=None, stream=None):
    """y = A x from CSR device tensors, no layout (the plain product)."""
    import torch
    nnz = col.numel()
    if y is None:
        y = torch.empty(n_rows, dtype=torch.float64, device=x.device)
    _check(load().spmv_csr(n_rows, n_cols, nnz,
                           _ptr(rowptr, torch.int32, n_rows + 1, "rowptr"),
                           _ptr(col, torch.int32, nnz, "col"),
                           _ptr(val, torch.float64, nnz, "val"),
                           _ptr(x, torch.float64, n_cols, "x"),
                           _ptr(y, torch.float64, n_rows, "y"),
                           _stream(stream)))
    return y


def probe_read_bandwidth(buf, sink, blocks, stream=None):
    """Stream the float64 device tensor buf once (measurement aid)."""
    import torch
    if sink.numel() < blocks:
        raise FsError(FS_E_ARG, "sink needs one entry per block")
    _check(load().probe_read_bandwidth(_ptr(buf, torch.float64), buf.numel(),
                                       _ptr(sink, torch.float64, None, "sink"),
                                       int(blocks), _stream(stream)))


def spmv_batch(mats, xs, ys=None, stream=None):
    """ys[i] = mats[i] @ xs[i] for every i, shared launches; returns ys."""
    import torch
    m = len(mats)
    if ys is None:
        ys = [torch.empty(M.n_rows, dtype=torch.float64, device=x.device)
              for M, x in zip(mats, xs)]
    hs = (C.c_void_p * max(1, m))(*[M._h for M in mats])
    xp = (C.c_void_p * max(1, m))(*[_ptr(x, torch.float64, M.n_cols, "x")
                                    for M, x in zip(mats, xs)])
    yp = (C.c_void_p * max(1, m))(*[_ptr(y, torch.float64, M.n_rows, "y")
                                    for M, y in zip(mats, ys)])
    _check(load().spmv_batch(m, hs, xp, yp, _stream(stream)))
    return ys


def spmv_perm(A, xp, yp=None, stream=None):
    import torch
    if yp is None:
        yp = torch.empty(A.n_rows, dtype=torch.float64, device=xp.device)
    _check(load().spmv_perm(A._h, _ptr(xp, torch.float64, A.n_cols, "x"),
                            _ptr(yp, torch.float64, A.n_rows, "y"),
                            _stream(stream)))
    return yp


def csr_permute(A, direction, inp, out=None, stream=None):
    import torch
    if out is None:
        out = torch.empty_like(inp)
    _check(load().csr_permute(A._h, int(direction),
                              _ptr(inp, torch.float64, A.n_rows, "in"),
                              _ptr(out, torch.float64, A.n_rows, "out"),
                              _stream(stream)))
    return out


def spmm(A, X, Y=None, stream=None):
    import torch
    k = X.shape[1]
    if Y is None:
        Y = torch.empty((A.n_rows, k), dtype=torch.float64, device=X.device)
    _check(load().spmm(A._h, k, _ptr(X, torch.float64, A.n_cols * k, "X"),
                       X.stride(0), _ptr(Y, torch.float64, A.n_rows * k, "Y"),
                       Y.stride(0), _stream(stream)))
    return Y


def spmv_lowp(A, dtype, xp, yp=None, stream=None):
    """y' = A'_lo x' in layout numbering with float vectors (FP32 or BF16
    values, float accumulation)."""
    import torch
    if yp is None:
        yp = torch.empty(A.n_rows, dtype=torch.float32, device=xp.device)
    _check(load().spmv_lowp(A._h, int(dtype),
                            _ptr(xp, torch.float32, A.n_cols, "x"),
                            _ptr(yp, torch.float32, A.n_rows, "y"),
                            _stream(stream)))
    return yp


def cg_opts(**kw):
    o = CgOpts()
    load().cg_opts_default(C.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def cg_solve(A, b, x=None, stream=None, check=True, **opts):
    """Solve A x = b; returns (x, info dict).  With check=False a
    not-converged or breakdown status is reported in info instead of
    raised."""
    import torch
    if x is None:
        x = torch.zeros(A.n_rows, dtype=torch.float64, device=b.device)
        opts.setdefault("x0_zero", 1)
    o = cg_opts(**opts)
    info = CgInfo()
    st = load().cg_solve(A._h, _ptr(b, torch.float64, A.n_rows, "b"),
                         _ptr(x, torch.float64, A.n_rows, "x"), C.byref(o),
                         C.byref(info), _stream(stream))
    d = info.as_dict()
    d["message"] = last_error() if st != FS_OK else ""
    if st != FS_OK and (check or st not in (FS_E_NOT_CONVERGED,
                                            FS_E_BREAKDOWN)):
        raise FsError(st, d["message"])
    return x, d


class AsyncSolve:
    """Result of cg_solve_async: x (filled when the stream gets there) and
    the info record in pinned host memory."""

    def __init__(self, x, buf, stream):
        self.x, self._buf, self._stream = x, buf, stream

    def info(self):
        """Wait for the stream, return the info dict."""
        import torch
        if self._stream is None:
            torch.cuda.current_stream().synchronize()
        elif isinstance(self._stream, int):
            torch.cuda.synchronize()
        else:
            self._stream.synchronize()
        d = CgInfo.from_address(self._buf.data_ptr()).as_dict()
        d["message"] = ""
        return d


def cg_solve_async(A, b, x=None, stream=None, **opts):
    """Enqueue the FP64 solve A x = b on the stream and return at once (an
    AsyncSolve; .x is the solution once the stream reaches it, .info()
    waits and returns the info dict)."""
    import torch
    if x is None:
        x = torch.zeros(A.n_rows, dtype=torch.float64, device=b.device)
        opts.setdefault("x0_zero", 1)
    o = cg_opts(**opts)
    buf = torch.zeros(C.sizeof(CgInfo), dtype=torch.uint8, pin_memory=True)
    _check(load().cg_solve_async(A._h, _ptr(b, torch.float64, A.n_rows, "b"),
                                 _ptr(x, torch.float64, A.n_rows, "x"),
                                 C.byref(o), C.c_void_p(buf.data_ptr()),
                                 _stream(stream)))
    return AsyncSolve(x, buf, stream)


def cg_solve_async_noalloc(A, b, x, info_buf, stream=None, **opts):
    """cg_solve_async without allocation: the caller passes x (device) and
    info_buf (a pinned uint8 host tensor of sizeof(fs_cg_info) bytes); the
    library uses its fixed device workspace.  Returns an AsyncSolve."""
    import torch
    o = cg_opts(**opts)
    if info_buf.numel() < C.sizeof(CgInfo) or info_buf.is_cuda:
        raise FsError(FS_E_ARG, "info_buf must be a host buffer of %d bytes"
                      % C.sizeof(CgInfo))
    _check(load().cg_solve_async_noalloc(
        A._h, _ptr(b, torch.float64, A.n_rows, "b"),
        _ptr(x, torch.float64, A.n_rows, "x"), C.byref(o),
        C.c_void_p(info_buf.data_ptr()), _stream(stream)))
    return AsyncSolve(x, info_buf, stream)


def info_buffer():
    """A pinned host buffer for one fs_cg_info record."""
    import torch
    return torch.zeros(C.sizeof(CgInfo), dtype=torch.uint8, pin_memory=True)


def cg_solve_multi(A, B, X=None, stream=None, check=True, **opts):
    """Solve A X[:, c] = B[:, c] for the k <= 16 columns of the n x k block
    B together; returns (X, list of k info dicts)."""
    import torch
    n, k = B.shape
    if X is None:
        X = torch.zeros((n, k), dtype=torch.float64, device=B.device)
        opts.setdefault("x0_zero", 1)
    o = cg_opts(**opts)
    infos = (CgInfo * k)()
    st = load().cg_solve_multi(A._h, k, _ptr(B, torch.float64, n * k, "B"),
                               B.stride(0),
                               _ptr(X, torch.float64, n * k, "X"),
                               X.stride(0), C.byref(o), infos,
                               _stream(stream))
    out = [i.as_dict() for i in infos]
    msg = last_error() if st != FS_OK else ""
    for d in out:
        d["message"] = msg
    if st != FS_OK and (check or st not in (FS_E_NOT_CONVERGED,
                                            FS_E_BREAKDOWN)):
        raise FsError(st, msg)
    return X, out


def cg_solve_batch(mats, Bs, Xs=None, stream=None, check=True, **opts):
    """Solve m independent systems mats[i] X_i = Bs[i] (each n_i x k_i, or a
    vector) with shared launches; returns (Xs, per-RHS info dicts)."""
    import torch
    m = len(mats)
    Bs = [b if b.dim() == 2 else b.reshape(-1, 1) for b in Bs]
    if Xs is None:
        Xs = [torch.zeros_like(b) for b in Bs]
        opts.setdefault("x0_zero", 1)
    else:
        Xs = [x if x.dim() == 2 else x.reshape(-1, 1) for x in Xs]
    ks = (C.c_int32 * m)(*[b.shape[1] for b in Bs])
    hs = (C.c_void_p * m)(*[M._h for M in mats])
    bp = (C.c_void_p * m)(*[_ptr(b, torch.float64, M.n_rows * b.shape[1],
                                 "B") for M, b in zip(mats, Bs)])
    xp = (C.c_void_p * m)(*[_ptr(x, torch.float64, M.n_rows * x.shape[1],
                                 "X") for M, x in zip(mats, Xs)])
    o = cg_opts(**opts)
    infos = (CgInfo * max(1, sum(ks)))()
    st = load().cg_solve_batch(m, hs, ks, bp, xp, C.byref(o), infos,
                               _stream(stream))
    out = [infos[i].as_dict() for i in range(sum(ks))]
    msg = last_error() if st != FS_OK else ""
    if st != FS_OK and (check or st not in (FS_E_NOT_CONVERGED,
                                            FS_E_BREAKDOWN)):
        raise FsError(st, msg)
    return Xs, out


def cg_solve_batch_wg(mats, bs, xs=None, stream=None, check=True, **opts):
    """Solve m small systems mats[i] x_i = bs[i] (vectors), each by one
    workgroup of a single launch; returns (xs, per-system info dicts)."""
    import torch
    m = len(mats)
    if xs is None:
        # one allocation, split into the systems' vectors; with a zero
        # initial guess the solve writes every entry
        opts.setdefault("x0_zero", 1)
        rows = [M.n_rows for M in mats]
        dev = bs[0].device if m else "cuda"
        mk = torch.empty if opts["x0_zero"] else torch.zeros
        xs = list(torch.split(mk(sum(rows), dtype=torch.float64, device=dev),
                              rows)) if m else []
    hs = (C.c_void_p * max(1, m))(*[M._h for M in mats])
    bp = (C.c_void_p * max(1, m))(*[_ptr(b, torch.float64, M.n_rows, "b")
                                    for M, b in zip(mats, bs)])
    xp = (C.c_void_p * max(1, m))(*[_ptr(x, torch.float64, M.n_rows, "x")
                                    for M, x in zip(mats, xs)])
    o = cg_opts(**opts)
    infos = (CgInfo * max(1, m))()
    st = load().cg_solve_batch_wg(m, hs, bp, xp, C.byref(o), infos,
                                  _stream(stream))
    out = [infos[i].as_dict() for i in range(m)]
    msg = last_error() if st != FS_OK else ""
    if st != FS_OK and (check or st not in (FS_E_NOT_CONVERGED,
                                            FS_E_BREAKDOWN)):
        raise FsError(st, msg)
    return xs, out


# ------------------------------------------------------------------ serving
class ServerOpts(C.Structure):
    _fields_ = [("hbm_budget_bytes", C.c_int64), ("max_slots", C.c_int32),
                ("check_every", C.c_int32), ("precond", C.c_int32),
                ("maxit", C.c_int32), ("rtol", C.c_double),
                ("use_graph", C.c_int32), ("reserved", C.c_int32 * 7)]


class ServerDone(C.Structure):
    _fields_ = [("req_id", C.c_uint64), ("k", C.c_int32), ("pad", C.c_int32),
                ("info", CgInfo), ("t_submit_ms", C.c_double),
                ("t_admit_ms", C.c_double), ("t_done_ms", C.c_double)]


class ServerStats(C.Structure):
    _fields_ = [("queued", C.c_int32), ("active", C.c_int32),
                ("peak_active", C.c_int32), ("pad", C.c_int32),
                ("submitted", C.c_uint64), ("completed", C.c_uint64),
                ("bytes_in_use", C.c_int64), ("peak_bytes", C.c_int64)]


def _declare_server(L):
    vp, i32 = C.c_void_p, C.c_int32
    P = C.POINTER
    for name, args in {
            "server_opts_default": [P(ServerOpts)],
            "server_create": [P(ServerOpts), P(vp)],
            "server_submit": [vp, vp, i32, vp, vp, P(C.c_uint64)],
            "server_poll": [vp, P(ServerDone), i32, P(i32)],
            "server_stats": [vp, P(ServerStats)],
            "server_destroy": [vp]}.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = C.c_int32


class Server:
    """Continuous-batching solve server (marshalling around server_*)."""

    def __init__(self, **opts):
        L = load()
        if not hasattr(L, "_server_declared"):
            _declare_server(L)
            L._server_declared = True
        o = ServerOpts()
        L.server_opts_default(C.byref(o))
        for k, v in opts.items():
            setattr(o, k, v)
        h = C.c_void_p()
        _check(L.server_create(C.byref(o), C.byref(h)))
        self.h = h.value
        self.keep = {}          # req_id -> (B, X) tensors kept alive

    def submit(self, A, B, X=None):
        import torch
        if B.dim() == 1:
            B = B.reshape(-1, 1)
        if X is None:
            X = torch.zeros_like(B)
        n, k = B.shape
        rid = C.c_uint64()
        _check(load().server_submit(self.h, A._h, k,
                                    _ptr(B, torch.float64, n * k, "B"),
                                    _ptr(X, torch.float64, n * k, "X"),
                                    C.byref(rid)))
        self.keep[rid.value] = (B, X, A)
        return rid.value, X

    def poll(self, cap=256):
        buf = (ServerDone * cap)()
        n = C.c_int32()
        _check(load().server_poll(self.h, buf, cap, C.byref(n)))
        out = []
        for i in range(n.value):
            d = buf[i]
            out.append({"req_id": d.req_id, "k": d.k,
                        "info": d.info.as_dict(),
                        "t_submit_ms": d.t_submit_ms,
                        "t_admit_ms": d.t_admit_ms,
                        "t_done_ms": d.t_done_ms})
            self.keep.pop(d.req_id, None)
        return out

    def stats(self):
        st = ServerStats()
        _check(load().server_stats(self.h, C.byref(st)))
        return {n: getattr(st, n) for n, _ in st._fields_ if n != "pad"}

    def drain(self, timeout_s=600.0):
        import time
        done = []
        t0 = time.time()
        while self.keep and time.time() - t0 < timeout_s:
            got = self.poll()
            done += got
            if not got:
                time.sleep(0.0005)
        return done

    def close(self):
        if self.h:
            st = load().server_destroy(self.h)
            self.h = None
            self.keep.clear()
            _check(st)

    def __del__(self, _fin=_finalize):
        _fin(self.close)


class Assembly:
    """Owning wrapper of an fs_asm_t plan; keeps its matrix alive."""

    def __init__(self, handle, A, n_elem, nde):
        self.handle, self.A = handle, A
        self.n_elem, self.nde = n_elem, nde

    def __del__(self, _fin=_finalize):
        _fin(self.close)

    def close(self):
        if self.handle:
            load().asm_destroy(self.handle)
            self.handle = None

    @property
    def _h(self):
        if not self.handle:
            raise FsError(FS_E_ARG, "assembly plan already destroyed")
        return self.handle


def asm_create(A, edof, plan=0, stream=None):
    """Assembly plan for A from the n_elem x nde int32 device tensor edof
    (-1 = DOF not in A); plan is ASM_AUTO, ASM_GATHER or ASM_ROWGROUP."""
    import torch
    if edof.dim() != 2:
        raise FsError(FS_E_ARG, "edof must be n_elem x nde")
    ne, nde = edof.shape
    h = C.c_void_p()
    _check(load().asm_create(A._h, ne, nde,
                             _ptr(edof, torch.int32, ne * nde, "edof"),
                             int(plan), _stream(stream), C.byref(h)))
    return Assembly(h.value, A, ne, nde)


def asm_plan_host(rowptr, col, edof, which=0, **opts):
    """Host-only dry run of asm_create (numpy arrays); returns dict(waves
    (nwaves x 2), tpos, aidx) of the matrix (which=0) or vector plan."""
    import numpy as np
    L = load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    edof = np.ascontiguousarray(edof, dtype=np.int32)
    ne, nde = edof.shape
    n = len(rowptr) - 1
    o = csr_opts(**opts)
    nt, nw, ns = C.c_int64(), C.c_int32(), C.c_int64()
    args = [n, len(col), rowptr.ctypes.data, col.ctypes.data, C.byref(o),
            ne, nde, edof.ctypes.data if edof.size else None, which,
            C.byref(nt), C.byref(nw), C.byref(ns)]
    _check(L.asm_plan_host(*args, None, None, None))
    waves = np.zeros((nw.value, 2), np.int32)
    tpos = np.zeros(nt.value, np.int32)
    aidx = np.zeros(ns.value, np.int32)
    _check(L.asm_plan_host(*args, waves.ctypes.data, tpos.ctypes.data,
                           aidx.ctypes.data))
    return dict(waves=waves, tpos=tpos, aidx=aidx)


def asm_plan_host_groups(rowptr, col, edof, **opts):
    """Host-only dry run of the row-group matrix plan; None when it does
    not apply, else dict(gdesc (ngroups x 4), bdesc (nbatch x 2), ea
    (nrec x rows), off (nrec x 64 uint16), rows)."""
    import numpy as np
    L = load()
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    col = np.ascontiguousarray(col, dtype=np.int32)
    edof = np.ascontiguousarray(edof, dtype=np.int32)
    ne, nde = edof.shape
    n = len(rowptr) - 1
    o = csr_opts(**opts)
    b, ng, nr = C.c_int32(), C.c_int32(), C.c_int32()
    nb, nrec = C.c_int64(), C.c_int64()
    args = [n, len(col), rowptr.ctypes.data, col.ctypes.data, C.byref(o),
            ne, nde, edof.ctypes.data if edof.size else None, C.byref(b),
            C.byref(ng), C.byref(nb), C.byref(nrec), C.byref(nr)]
    _check(L.asm_plan_host_groups(*args, None, None, None, None))
    if not b.value:
        return None
    gdesc = np.zeros((ng.value, 4), np.int32)
    bdesc = np.zeros((nb.value, 2), np.int32)
    ea = np.zeros((nrec.value, nr.value), np.int32)
    off = np.zeros((nrec.value, 64), np.uint16)
    _check(L.asm_plan_host_groups(*args, gdesc.ctypes.data, bdesc.ctypes.data,
                                  ea.ctypes.data, off.ctypes.data))
    return dict(gdesc=gdesc, bdesc=bdesc, ea=ea, off=off, rows=nr.value)


def asm_matrix(P, ke, stream=None):
    """Assemble the element matrices ke (n_elem x nde x nde float64, device)
    into the values of P's matrix."""
    import torch
    _check(load().asm_matrix(P._h, _ptr(ke, torch.float64,
                                        P.n_elem * P.nde * P.nde, "ke"),
                             _stream(stream)))


def asm_vector(P, re, r=None, stream=None):
    """r = assembled element vectors re (n_elem x nde float64, device), in
    the caller's row numbering; returns r."""
    import torch
    if r is None:
        r = torch.empty(P.A.n_rows, dtype=torch.float64, device="cuda")
    _check(load().asm_vector(P._h, _ptr(re, torch.float64, P.n_elem * P.nde,
                                        "re"),
                             _ptr(r, torch.float64, P.A.n_rows, "r"),
                             _stream(stream)))
    return r


def asm_system(P, ke, re, r=None, stream=None):
    """asm_matrix(P, ke) and asm_vector(P, re, r) in one pass; returns r."""
    import torch
    if r is None:
        r = torch.empty(P.A.n_rows, dtype=torch.float64, device="cuda")
    _check(load().asm_system(
        P._h, _ptr(ke, torch.float64, P.n_elem * P.nde * P.nde, "ke"),
        _ptr(re, torch.float64, P.n_elem * P.nde, "re"),
        _ptr(r, torch.float64, P.A.n_rows, "r"), _stream(stream)))
    return r


def asm_element_rows(P):
    """numpy int32 array pos (n_elem * nde): plan-ordered buffer row of each
    element row (-1: not assembled), and the buffer's row count."""
    import numpy as np
    rows = C.c_int64()
    _check(load().asm_element_rows(P._h, None, C.byref(rows)))
    pos = np.empty(P.n_elem * P.nde, np.int32)
    _check(load().asm_element_rows(P._h, pos.ctypes.data if pos.size else
                                   None, C.byref(rows)))
    return pos, rows.value


def asm_matrix_ordered(P, ke_ordered, stream=None):
    """Assemble from the plan-ordered element buffer (rows x nde float64,
    device)."""
    import torch
    _check(load().asm_matrix_ordered(
        P._h, _ptr(ke_ordered, torch.float64, None, "ke_ordered"),
        _stream(stream)))


def asm_info(P):
    st = AsmStats()
    _check(load().asm_info(P._h, C.byref(st)))
    return st.as_dict()


def asm_destroy(P):
    P.close()
