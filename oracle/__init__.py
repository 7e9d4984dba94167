"""CPU oracle for the FEM SpMV / CG path -- test infrastructure only.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The product library never does, and this
package never imports the product library: the two share no code.

The arithmetic lives in ``oracle.c`` (plain C, FP64, single thread, built
with ``gcc -O2 -ffp-contract=off``; one row-parallel OpenMP copy of the
product exists only to time the oracle on all host cores); this module only
marshals numpy arrays.
``build()`` compiles it; ``load()`` builds on first use when the shared
object is missing.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "oracle.c")
LIB = os.path.join(HERE, "liboracle.so")

OK, NOT_CONVERGED, BREAKDOWN, ARG = 0, 1, 2, 3

_lib = None


def build(force=True):
    if not force and os.path.exists(LIB):
        return LIB
    tmp = LIB + ".tmp%d" % os.getpid()
    subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fPIC",
                           "-fopenmp", "-shared", "-std=c11", SRC, "-o", tmp,
                           "-lm"])
    os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB) or \
                os.path.getmtime(LIB) < os.path.getmtime(SRC):
            build()
        _lib = C.CDLL(LIB)
        _declare(_lib)
    return _lib


_i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_f32p = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_u16p = np.ctypeslib.ndpointer(np.uint16, flags="C_CONTIGUOUS")


def _declare(L):
    i32, i64, f64 = C.c_int32, C.c_int64, C.c_double
    P = C.POINTER
    L.or_spmv.argtypes = [i32, _i32p, _i32p, _f64p, _f64p, _f64p]
    L.or_spmv_par.argtypes = [i32, _i32p, _i32p, _f64p, _f64p, _f64p]
    L.or_spmv_par.restype = C.c_int
    L.or_spmv_abs.argtypes = [i32, _i32p, _i32p, _f64p, _f64p, _f64p]
    L.or_spmm.argtypes = [i32, _i32p, _i32p, _f64p, i32, _f64p, i64, _f64p,
                          i64]
    L.or_spmv_f32.argtypes = [i32, _i32p, _i32p, _f32p, _f32p, _f32p]
    L.or_gather.argtypes = [i32, _i32p, _f64p, _f64p]
    L.or_scatter.argtypes = [i32, _i32p, _f64p, _f64p]
    L.or_inverse_perm.argtypes = [i32, _i32p, _i32p]
    L.or_permute.argtypes = [i32, _i32p, _i32p, _f64p, C.c_void_p,
                             C.c_void_p, i32, _i32p, _i32p, _f64p]
    L.or_round_f32.argtypes = [f64]
    L.or_round_f32.restype = C.c_float
    L.or_f32_to_bf16.argtypes = [C.c_float]
    L.or_f32_to_bf16.restype = C.c_uint16
    L.or_bf16_to_f32.argtypes = [C.c_uint16]
    L.or_bf16_to_f32.restype = C.c_float
    L.or_round_array_f32.argtypes = [i64, _f64p, _f32p]
    L.or_round_array_bf16.argtypes = [i64, _f64p, _u16p]
    L.or_assemble_matrix.argtypes = [i32, _i32p, _i32p, i32, i32, _i32p,
                                     _f64p, _f64p]
    L.or_assemble_matrix.restype = i64
    L.or_assemble_vector.argtypes = [i32, i32, i32, _i32p, _f64p, _f64p]
    L.or_pcg.argtypes = [i32, _i32p, _i32p, _f64p, _f64p, _f64p, i32, f64,
                         i32, P(i32), P(f64)]
    L.or_pcg.restype = C.c_int
    L.or_ir_cg.argtypes = [i32, _i32p, _i32p, _f64p, _f32p, _f64p, _f64p,
                           i32, f64, f64, i32, i32, P(i32), P(i32), P(f64),
                           C.c_void_p]
    L.or_ir_cg.restype = C.c_int
    L.or_ir_cg_keep.argtypes = [i32, _i32p, _i32p, _f64p, _f32p, _f64p, _f64p,
                           i32, f64, f64, i32, i32, P(i32), P(i32), P(f64),
                           C.c_void_p]
    L.or_ir_cg_keep.restype = C.c_int


def _csr(A):
    rp = np.ascontiguousarray(A.rowptr, dtype=np.int32)
    c = np.ascontiguousarray(A.col, dtype=np.int32)
    v = np.ascontiguousarray(A.val, dtype=np.float64)
    return rp, c, v


def _f64(x):
    return np.ascontiguousarray(x, dtype=np.float64)


# --------------------------------------------------------------------------
# numpy-facing wrappers (A is any object with n_rows, n_cols, rowptr, col,
# val: e.g. workloads.CSR)
# --------------------------------------------------------------------------
def spmv(A, x):
    L = load()
    rp, c, v = _csr(A)
    x = _f64(x)
    assert x.shape == (A.n_cols,)
    y = np.empty(A.n_rows)
    L.or_spmv(A.n_rows, rp, c, v, x, y)
    return y


def spmv_par(A, x):
    """spmv with rows split over OpenMP threads (bitwise the same result);
    returns (y, threads used)."""
    L = load()
    rp, c, v = _csr(A)
    x = _f64(x)
    assert x.shape == (A.n_cols,)
    y = np.empty(A.n_rows)
    used = L.or_spmv_par(A.n_rows, rp, c, v, x, y)
    return y, int(used)


def spmv_abs(A, x):
    """(|A| |x|)_i, the per-row scale of the rounding error."""
    L = load()
    rp, c, v = _csr(A)
    y = np.empty(A.n_rows)
    L.or_spmv_abs(A.n_rows, rp, c, v, _f64(x), y)
    return y


def spmm(A, X):
    L = load()
    rp, c, v = _csr(A)
    X = _f64(X)
    n, k = X.shape
    assert n == A.n_cols
    Y = np.empty((A.n_rows, k))
    L.or_spmm(A.n_rows, rp, c, v, k, X, k, Y, k)
    return Y


def spmv_f32(A, a_lo, x):
    """Single-precision product with stored single-precision values."""
    L = load()
    rp, c, _ = _csr(A)
    a = np.ascontiguousarray(a_lo, dtype=np.float32)
    xf = np.ascontiguousarray(x, dtype=np.float32)
    y = np.empty(A.n_rows, dtype=np.float32)
    L.or_spmv_f32(A.n_rows, rp, c, a, xf, y)
    return y


def gather(perm, x):
    L = load()
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    out = np.empty(len(perm))
    L.or_gather(len(perm), perm, _f64(x), out)
    return out


def scatter(perm, xp):
    L = load()
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    out = np.empty(len(perm))
    L.or_scatter(len(perm), perm, _f64(xp), out)
    return out


def inverse_perm(perm):
    L = load()
    perm = np.ascontiguousarray(perm, dtype=np.int32)
    out = np.empty(len(perm), dtype=np.int32)
    L.or_inverse_perm(len(perm), perm, out)
    return out


def permute(A, rperm=None, ciperm=None, sort_cols=False):
    """Return (rowptr, col, val) of the renumbered matrix."""
    L = load()
    rp, c, v = _csr(A)
    nrows = A.n_rows if rperm is None else len(rperm)
    orp = np.empty(nrows + 1, dtype=np.int32)
    oc = np.empty(len(c), dtype=np.int32)
    ov = np.empty(len(v))
    rp_arg = None if rperm is None else np.ascontiguousarray(rperm, np.int32)
    ci_arg = None if ciperm is None else np.ascontiguousarray(ciperm,
                                                              np.int32)
    L.or_permute(nrows, rp, c, v,
                 None if rp_arg is None else rp_arg.ctypes.data,
                 None if ci_arg is None else ci_arg.ctypes.data,
                 int(bool(sort_cols)), orp, oc, ov)
    return orp, oc, ov


def round_f32(v):
    L = load()
    v = _f64(np.atleast_1d(v))
    out = np.empty(v.shape, dtype=np.float32)
    L.or_round_array_f32(v.size, v.reshape(-1), out.reshape(-1))
    return out


def round_bf16(v):
    """FP64 -> FP32 (nearest) -> BF16 (nearest, ties to even); uint16 bits."""
    L = load()
    v = _f64(np.atleast_1d(v))
    out = np.empty(v.shape, dtype=np.uint16)
    L.or_round_array_bf16(v.size, v.reshape(-1), out.reshape(-1))
    return out


def f32_to_bf16_bits(f):
    L = load()
    return int(L.or_f32_to_bf16(float(np.float32(f))))


def bf16_bits_to_f32(bits):
    """Widen BF16 bit patterns to float32 (exact)."""
    b = np.asarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32)


def pcg(A, b, x0=None, precond=1, rtol=1e-8, maxit=20000):
    """Textbook preconditioned CG; returns (x, status, iters, relres)."""
    L = load()
    rp, c, v = _csr(A)
    b = _f64(b)
    x = np.zeros(A.n_rows) if x0 is None else _f64(x0).copy()
    it = C.c_int32(0)
    rr = C.c_double(0.0)
    st = L.or_pcg(A.n_rows, rp, c, v, b, x, int(precond), float(rtol),
                  int(maxit), C.byref(it), C.byref(rr))
    return x, st, it.value, rr.value


def ir_cg(A, a_lo, b, x0=None, precond=1, rtol=1e-8, inner_rtol=1e-3,
          max_outer=100, max_inner=20000, keep=False, scale=None):
    """FP64-outer / FP32-inner refinement; returns
    (x, status, outer, inner, relres).  keep=True: one inner CG kept across
    the steps (its residual replaced by the FP64 one at each step).
    scale = s (diag(A)^-1/2): a_lo holds round(S A S) and the inner solve
    runs on the Jacobi-scaled system (pass precond=0)."""
    L = load()
    rp, c, v = _csr(A)
    b = _f64(b)
    x = np.zeros(A.n_rows) if x0 is None else _f64(x0).copy()
    a = np.ascontiguousarray(a_lo, dtype=np.float32)
    o = C.c_int32(0)
    i = C.c_int32(0)
    rr = C.c_double(0.0)
    fn = L.or_ir_cg_keep if keep else L.or_ir_cg
    sc = None if scale is None else np.ascontiguousarray(scale,
                                                        dtype=np.float64)
    st = fn(A.n_rows, rp, c, v, a, b, x, int(precond), float(rtol),
            float(inner_rtol), int(max_outer), int(max_inner),
            C.byref(o), C.byref(i), C.byref(rr),
            None if sc is None else sc.ctypes.data)
    return x, st, o.value, i.value, rr.value


def jacobi_scaled_values(A):
    """(s, v): s_i = diag(A)_i^-1/2 and the values of S A S in CSR order,
    each formed as (a_ij s_i) s_j in FP64 (diagonal entries summed per row,
    as stored duplicates would be)."""
    rows = np.repeat(np.arange(A.n_rows), np.diff(A.rowptr))
    d = np.zeros(A.n_rows)
    on = A.col == rows
    np.add.at(d, rows[on], A.val[on])
    s = 1.0 / np.sqrt(d)
    return s, (A.val * s[rows]) * s[A.col]


def assemble_matrix(A, edof, ke):
    """Values of the pattern of A (CSR: rowptr, col) assembled from element
    matrices ke (n_elem x nde x nde) through edof (n_elem x nde, -1 = not
    assembled), elements in order.  Raises ValueError naming the first
    element whose coupling is missing from the pattern."""
    L = load()
    edof = np.ascontiguousarray(edof, dtype=np.int32)
    ne, nde = edof.shape
    ke = np.ascontiguousarray(ke, dtype=np.float64).reshape(ne, nde, nde)
    rp = np.ascontiguousarray(A.rowptr, dtype=np.int32)
    c = np.ascontiguousarray(A.col, dtype=np.int32)
    val = np.empty(len(c))
    bad = L.or_assemble_matrix(A.n_rows, rp, c, ne, nde, edof, ke, val)
    if bad:
        raise ValueError("element %d couples DOFs outside the pattern"
                         % (bad - 1))
    return val


def assemble_vector(n_rows, edof, re):
    """r[I] = sum of re[e, a] over edof[e, a] == I, elements in order."""
    L = load()
    edof = np.ascontiguousarray(edof, dtype=np.int32)
    ne, nde = edof.shape
    re = np.ascontiguousarray(re, dtype=np.float64).reshape(ne, nde)
    r = np.empty(n_rows)
    L.or_assemble_vector(n_rows, ne, nde, edof, re, r)
    return r
