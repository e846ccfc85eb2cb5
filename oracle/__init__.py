"""Oracle: plain FP64 CPU reference for the autotuned kernels.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package; the HIP library
and its Python binding never do.  The arithmetic lives in ``spk_oracle.c``
(built into ``liboracle.so`` with gcc, -O2 -ffp-contract=off, OpenMP over
rows/elements only); this module only marshals numpy arrays.

Every function cites the operation it computes in the paper's terms: the
unannotated reference program of Section 2 whose outputs tuned variants must
reproduce, applied to the WAXPY-type vector update of Figure 1 and to the
CSR sparse matrix-vector product of the prior GPU work quoted in Section 3.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "spk_oracle.c")

_lib = None

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_D = ctypes.c_double


def build(verbose: bool = False) -> str:
    """Compile spk_oracle.c into liboracle.so (always recompiles)."""
    cmd = ["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-Wextra", "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "orc_num_threads": (ctypes.c_int, []),
            "orc_set_num_threads": (None, [ctypes.c_int]),
            "orc_waxpy_f64": (None, [_I64, _D, _P, _P, _P]),
            "orc_waxpy_f32": (None, [_I64, _D, _P, _P, _P]),
            "orc_axpy_f64": (None, [_I64, _D, _P, _P]),
            "orc_axpy_f32": (None, [_I64, _D, _P, _P]),
            "orc_dot_f64": (_D, [_I64, _P, _P]),
            "orc_dot_f32": (_D, [_I64, _P, _P]),
            "orc_dot_absum_f64": (_D, [_I64, _P, _P]),
            "orc_dot_absum_f32": (_D, [_I64, _P, _P]),
            "orc_spmv_csr_f64": (None, [_I64, _P, _P, _P, _P, _P, _P]),
            "orc_spmv_csr_f32": (None, [_I64, _P, _P, _P, _P, _P, _P]),
            "orc_spmv_waxpy_f64": (None, [_I64, _P, _P, _P, _P, _D, _P, _P, _P]),
            "orc_batch_spmv_waxpy_f64": (None, [_I64, _P, _P, _P, _P, _P, _P, _P, _P, _D, _P, _P, _P]),
            "orc_max_ulp_f64": (_I64, [_I64, _P, _P, _P]),
            "orc_max_ulp_f32": (_I64, [_I64, _P, _P, _P]),
            "orc_check_rows": (_I64, [_I64, _P, _P, _P, _D, _P, _P]),
            "orc_cg_f64": (None, [_I64, _P, _P, _P, _P, _P, _I64, _P, _P, _P, _P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray | None):
    return None if a is None else a.ctypes.data


def _c(a, dtype):
    a = np.ascontiguousarray(a)
    if a.dtype != dtype:
        raise TypeError(f"expected {np.dtype(dtype)}, got {a.dtype}")
    return a


def _fdt(x):
    dt = np.asarray(x).dtype
    if dt not in (np.float64, np.float32):
        raise TypeError(f"unsupported dtype {dt}")
    return dt


def set_threads(t: int) -> None:
    lib().orc_set_num_threads(int(t))


def num_threads() -> int:
    return int(lib().orc_num_threads())


def waxpy(alpha: float, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """w = alpha*x + y with one rounding (the vector update of Figure 1)."""
    dt = _fdt(x)
    x, y = _c(x, dt), _c(y, dt)
    assert x.shape == y.shape
    w = np.empty_like(x)
    f = lib().orc_waxpy_f64 if dt == np.float64 else lib().orc_waxpy_f32
    f(x.size, float(alpha), _ptr(x), _ptr(y), _ptr(w))
    return w


def axpy(alpha: float, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Returns a copy of y after y <- alpha*x + y."""
    dt = _fdt(x)
    x = _c(x, dt)
    out = np.array(y, dtype=dt, copy=True)
    f = lib().orc_axpy_f64 if dt == np.float64 else lib().orc_axpy_f32
    f(x.size, float(alpha), _ptr(x), _ptr(out))
    return out


def dot(x: np.ndarray, y: np.ndarray) -> float:
    """sum_i x_i*y_i, compensated, in index order."""
    dt = _fdt(x)
    x, y = _c(x, dt), _c(y, dt)
    f = lib().orc_dot_f64 if dt == np.float64 else lib().orc_dot_f32
    return float(f(x.size, _ptr(x), _ptr(y)))


def dot_absum(x: np.ndarray, y: np.ndarray) -> float:
    """sum_i |x_i*y_i|: the scale of the dot tolerance (the magnitude sum of
    the same products the dot adds, as the per-row SpMV tolerance uses)."""
    dt = _fdt(x)
    x, y = _c(x, dt), _c(y, dt)
    f = lib().orc_dot_absum_f64 if dt == np.float64 else lib().orc_dot_absum_f32
    return float(f(x.size, _ptr(x), _ptr(y)))


def spmv(A, x: np.ndarray, with_absum: bool = True):
    """y = A*x over CSR ``A`` (any object with nrows/row_ptr/col_idx/val).

    Returns (y, absum) with y in float64 (FP32 data promoted exactly) and
    absum_i = sum_k |a_ik x_k| (None when not requested)."""
    dt = _fdt(A.val)
    rp, ci, val = _c(A.row_ptr, np.int32), _c(A.col_idx, np.int32), _c(A.val, dt)
    x = _c(x, dt)
    y = np.empty(A.nrows, np.float64)
    absum = np.empty(A.nrows, np.float64) if with_absum else None
    f = lib().orc_spmv_csr_f64 if dt == np.float64 else lib().orc_spmv_csr_f32
    f(A.nrows, _ptr(rp), _ptr(ci), _ptr(val), _ptr(x), _ptr(y), _ptr(absum))
    return y, absum


def spmv_waxpy(A, x: np.ndarray, alpha: float):
    """One Krylov-style step (FP64): y = A*x, w = alpha*y + x.  Returns (y, w, absum)."""
    rp, ci, val = _c(A.row_ptr, np.int32), _c(A.col_idx, np.int32), _c(A.val, np.float64)
    x = _c(x, np.float64)
    assert A.nrows == A.ncols == x.size
    y = np.empty(A.nrows, np.float64)
    w = np.empty(A.nrows, np.float64)
    absum = np.empty(A.nrows, np.float64)
    lib().orc_spmv_waxpy_f64(A.nrows, _ptr(rp), _ptr(ci), _ptr(val), _ptr(x), float(alpha),
                             _ptr(y), _ptr(w), _ptr(absum))
    return y, w, absum


def batch_spmv_waxpy(B, x: np.ndarray, alpha: float, count: int | None = None):
    """Per-instance spmv_waxpy over a concatenated batch (FP64).

    ``count`` limits the work to the first ``count`` instances."""
    count = B.count if count is None else int(count)
    m = _c(B.m, np.int64)
    rp_off, nz_off, vec_off = _c(B.rp_off, np.int64), _c(B.nz_off, np.int64), _c(B.vec_off, np.int64)
    rp, ci, val = _c(B.row_ptr, np.int32), _c(B.col_idx, np.int32), _c(B.val, np.float64)
    x = _c(x, np.float64)
    nv = int(vec_off[count - 1] + m[count - 1]) if count else 0
    y = np.empty(nv, np.float64)
    w = np.empty(nv, np.float64)
    absum = np.empty(nv, np.float64)
    lib().orc_batch_spmv_waxpy_f64(count, _ptr(m), _ptr(rp_off), _ptr(nz_off), _ptr(vec_off),
                                   _ptr(rp), _ptr(ci), _ptr(val), _ptr(x), float(alpha),
                                   _ptr(y), _ptr(w), _ptr(absum))
    return y, w, absum


def cg(A, b: np.ndarray, iters: int, x0: np.ndarray | None = None):
    """Conjugate gradients (FP64) on a square SPD CSR matrix: returns (x after
    `iters` iterations, rr_hist[0..iters]) -- the Krylov iteration built
    from the SpMV, dot and AXPY/WAXPY kernels of the library."""
    n = A.nrows
    assert A.ncols == n
    rp, ci, val = _c(A.row_ptr, np.int32), _c(A.col_idx, np.int32), _c(A.val, np.float64)
    b = _c(b, np.float64)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    hist = np.empty(iters + 1)
    r, p, q = np.empty(n), np.empty(n), np.empty(n)
    lib().orc_cg_f64(n, _ptr(rp), _ptr(ci), _ptr(val), _ptr(b), _ptr(x), int(iters), _ptr(hist), _ptr(r), _ptr(p),
                     _ptr(q))
    return x, hist


def max_ulp(a: np.ndarray, b: np.ndarray):
    """(largest ulp distance, index) between same-dtype arrays; NaN vs non-NaN is 2**63-1."""
    dt = _fdt(a)
    a, b = _c(a, dt), _c(b, dt)
    assert a.shape == b.shape
    where = ctypes.c_int64(-1)
    f = lib().orc_max_ulp_f64 if dt == np.float64 else lib().orc_max_ulp_f32
    d = f(a.size, _ptr(a), _ptr(b), ctypes.byref(where))
    return int(d), int(where.value)


def check_rows(y: np.ndarray, ref: np.ndarray, absum: np.ndarray, tau: float):
    """(failing rows, worst |y-ref|/absum, its index) of the per-row test."""
    y = np.ascontiguousarray(y, dtype=np.float64)
    ref, absum = _c(ref, np.float64), _c(absum, np.float64)
    worst = ctypes.c_double(0.0)
    where = ctypes.c_int64(-1)
    bad = lib().orc_check_rows(y.size, _ptr(y), _ptr(ref), _ptr(absum), float(tau),
                               ctypes.byref(worst), ctypes.byref(where))
    return int(bad), float(worst.value), int(where.value)


TAU_F64 = 1e-12
TAU_F32 = 1e-5


def tau_for(dtype) -> float:
    return TAU_F64 if np.dtype(dtype) == np.float64 else TAU_F32
