"""Thin Python binding of libspk (the C ABI declared in include/spk.h).

Only argument marshalling happens here: torch tensors are passed to the
library as raw device pointers together with torch's current HIP stream, and
every computation runs in the library's HIP kernels.  Function names are the
C entry points' names.  If libspk.so has not been built, importing this
module raises: there is no other implementation to fall back to.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspk.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it first (python -c 'import __graft_entry__ as g; g.build()')")

_lib = C.CDLL(LIB_PATH)

# ------------------------------------------------------------------ types --

SPK_OK = 0
SPK_F32, SPK_F64 = 0, 1
SPK_OP_SPMV, SPK_OP_WAXPY, SPK_OP_AXPY, SPK_OP_DOT, SPK_OP_SPMV_WAXPY = 0, 1, 2, 3, 4
SPK_FMT_AUTO, SPK_FMT_SCALAR, SPK_FMT_VECTOR, SPK_FMT_SELL, SPK_FMT_ADAPTIVE = 0, 1, 2, 3, 4
SPK_FMT_DIA, SPK_FMT_STENCIL, SPK_FMT_COLBLOCK, SPK_FMT_XWIN = 5, 6, 7, 8
# the formats that store the CSR entries, in some order (measured on the CSR
# algorithmic bytes)
CSR_FORMATS = ((1 << SPK_FMT_SCALAR) | (1 << SPK_FMT_VECTOR) | (1 << SPK_FMT_SELL) | (1 << SPK_FMT_ADAPTIVE) |
               (1 << SPK_FMT_COLBLOCK) | (1 << SPK_FMT_XWIN))
STATUS = {0: "SPK_OK", 1: "SPK_ERR_NULL", 2: "SPK_ERR_SHAPE", 3: "SPK_ERR_DTYPE", 4: "SPK_ERR_ALIAS",
          5: "SPK_ERR_CSR", 6: "SPK_ERR_OOM", 7: "SPK_ERR_BUDGET", 8: "SPK_ERR_HIP", 9: "SPK_ERR_VALIDATION",
          10: "SPK_ERR_NOT_FOUND", 11: "SPK_ERR_ARG", 12: "SPK_ERR_STATE", 13: "SPK_ERR_INTERRUPTED"}

_P = C.c_void_p
_I32 = C.c_int32
_I64 = C.c_int64
_D = C.c_double


class spk_csr(C.Structure):
    _fields_ = [("nrows", _I64), ("ncols", _I64), ("nnz", _I64), ("dtype", _I32),
                ("row_ptr", _P), ("col_idx", _P), ("val", _P)]


class spk_variant(C.Structure):
    _fields_ = [(f, _I32) for f in ("format", "block", "group", "unroll", "vec", "grid", "streams", "lds")]

    def as_dict(self):
        return {f: int(getattr(self, f)) for f, _ in self._fields_}

    def __repr__(self):
        return "spk_variant(" + ", ".join(f"{k}={v}" for k, v in self.as_dict().items()) + ")"


class spk_problem(C.Structure):
    _fields_ = [("op", _I32), ("dtype", _I32), ("n", _I64), ("alpha", _D), ("A", _P),
                ("x", _P), ("y", _P), ("w", _P), ("d_result", _P)]


class spk_tune_opts(C.Structure):
    _fields_ = [("reps", _I32), ("warmup", _I32), ("flush", _I32), ("max_variants", _I32), ("tau", _D),
                ("ref_host", _P), ("ref_scale", _P), ("record", _I32), ("verbose", _I32),
                ("formats", C.c_uint32), ("resume", _I32), ("stop_after", _I32)]


class spk_structure(C.Structure):
    _fields_ = [("formats", C.c_uint32), ("ndiag", _I32), ("offsets", _I32 * 16), ("dim", _I32), ("n1", _I32),
                ("n2", _I32), ("n3", _I32), ("coef", _D * 7)]


class spk_tune_report(C.Structure):
    _fields_ = [("best", spk_variant), ("best_us", _D), ("plain_us", _D), ("tried", _I32),
                ("rejected", _I32), ("pruned", _I32), ("class_key", C.c_char * 96), ("resumed", _I32)]


class spk_batch_desc(C.Structure):
    _fields_ = [("count", _I64), ("dtype", _I32), ("m", _P), ("nnz", _P), ("rp_off", _P), ("nz_off", _P),
                ("vec_off", _P), ("row_ptr", _P), ("col_idx", _P), ("val", _P), ("row_ptr_host", _P)]


class spk_batch_opts(C.Structure):
    _fields_ = [("persistent", _I32), ("use_graph", _I32), ("block", _I32), ("tile_nnz", _I32),
                ("waves_per_cu", _I32), ("x_window", _I32)]


class spk_serve_opts(C.Structure):
    _fields_ = [("streams", _I32), ("max_inflight", _I32), ("max_batch", _I32), ("mode", _I32),
                ("hbm_budget", _I64), ("alpha", _D), ("max_launches", _I32), ("reserved", _I32)]


class spk_serve_stats(C.Structure):
    _fields_ = [("submitted", _I64), ("completed", _I64), ("rejected", _I64), ("batches", _I64),
                ("uploads", _I64), ("evictions", _I64), ("resident_bytes", _I64), ("peak_bytes", _I64),
                ("p50_us", _D), ("p99_us", _D), ("mean_us", _D), ("max_us", _D), ("wall_s", _D),
                ("bytes_moved", _D), ("stage_in_s", _D), ("stage_out_s", _D), ("device_s", _D),
                ("direct", _I64)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


_S = C.c_int  # spk_status
_SIGS = {
    "spk_abi_version": (C.c_int, []),
    "spk_status_str": (C.c_char_p, [_S]),
    "spk_create": (_S, [C.c_int, C.c_char_p, C.POINTER(_P)]),
    "spk_destroy": (_S, [_P]),
    "spk_last_error": (C.c_char_p, []),
    "spk_check": (_S, [_P, _P]),
    "spk_set_plain": (_S, [_P, C.c_int]),
    "spk_device_info": (_S, [_P, C.POINTER(_I32), C.c_char_p, _I32]),
    "spk_waxpy": (_S, [_P, _I32, _I64, _D, _P, _P, _P, _P]),
    "spk_axpy": (_S, [_P, _I32, _I64, _D, _P, _P, _P]),
    "spk_dot": (_S, [_P, _I32, _I64, _P, _P, _P, _P]),
    "spk_dot_noalloc": (_S, [_P, _I32, _I64, _P, _P, _P, _P]),
    "spk_spmv_csr": (_S, [_P, C.POINTER(spk_csr), _P, _P, _P]),
    "spk_matrix_register": (_S, [_P, C.POINTER(spk_csr), _I32, _I32, C.POINTER(_P)]),
    "spk_matrix_release": (_S, [_P, _P]),
    "spk_matrix_bytes": (_S, [_P, _P, C.POINTER(_I64)]),
    "spk_matrix_formats": (_S, [_P, _P, C.POINTER(C.c_uint32)]),
    "spk_matrix_format_bytes": (_S, [_P, _P, _I32, _I32, C.POINTER(_I64)]),
    "spk_csr_structure": (_S, [C.POINTER(spk_csr), C.POINTER(spk_structure)]),
    "spk_spmv_mat": (_S, [_P, _P, _P, _P, _P]),
    "spk_spmv_waxpy": (_S, [_P, _P, _D, _P, _P, _P, _P]),
    "spk_cg": (_S, [_P, _P, _P, _P, _I32, _P, _P]),
    "spk_cg_tune": (_S, [_P, _P, _P, _I32, C.POINTER(spk_tune_opts), C.POINTER(spk_tune_report)]),
    "spk_run": (_S, [_P, C.POINTER(spk_problem), C.POINTER(spk_variant), _P]),
    "spk_variant_count": (_S, [_I32, _I32, C.POINTER(_I32)]),
    "spk_variant_get": (_S, [_I32, _I32, _I32, C.POINTER(spk_variant)]),
    "spk_plain_variant": (_S, [_I32, _I32, C.POINTER(spk_variant)]),
    "spk_tune": (_S, [_P, C.POINTER(spk_problem), C.POINTER(spk_tune_opts), C.POINTER(spk_tune_report)]),
    "spk_class_key": (_S, [_P, C.POINTER(spk_problem), C.c_char_p, _I32]),
    "spk_plan_get": (_S, [_P, C.c_char_p, C.POINTER(spk_variant)]),
    "spk_plan_put": (_S, [_P, C.c_char_p, C.POINTER(spk_variant)]),
    "spk_batch_plan": (_S, [_P, C.POINTER(spk_batch_desc), C.POINTER(spk_batch_opts), C.POINTER(_P)]),
    "spk_batch_run": (_S, [_P, _P, _D, _P, _P, _P, _P]),
    "spk_batch_tune": (_S, [_P, _P, _D, _P, _P, _P, C.POINTER(spk_tune_opts), C.POINTER(spk_tune_report)]),
    "spk_batch_info": (_S, [_P, _P, C.POINTER(_I64), C.POINTER(_I32), C.POINTER(_I64)]),
    "spk_batch_tile_modes": (_S, [_P, _P, C.POINTER(_I64), C.POINTER(_I64)]),
    "spk_batch_config": (_S, [_P, _P, C.POINTER(spk_batch_opts)]),
    "spk_batch_free": (_S, [_P, _P]),
    "spk_serve_create": (_S, [_P, C.POINTER(spk_serve_opts), C.POINTER(_P)]),
    "spk_serve_add_matrix": (_S, [_P, C.POINTER(spk_csr), C.POINTER(_I32)]),
    "spk_serve_submit": (_S, [_P, _I32, _P, _P, _P, C.POINTER(_I64)]),
    "spk_serve_poll": (_S, [_P, _P, _I32, C.POINTER(_I32)]),
    "spk_serve_drain": (_S, [_P]),
    "spk_serve_replay": (_S, [_P, _I64, _P, _P, _P, _P, _P]),
    "spk_serve_stats_get": (_S, [_P, C.POINTER(spk_serve_stats)]),
    "spk_serve_latencies": (_S, [_P, _P, _I64, C.POINTER(_I64)]),
    "spk_serve_latency_split": (_S, [_P, _P, _P, _I64, C.POINTER(_I64)]),
    "spk_serve_destroy": (_S, [_P]),
    "spk_stream_probe": (_S, [_P, _I32, _I64, _P, _P, _P, _P]),
    "spk_flush_cache": (_S, [_P, _P]),
}
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

lib = _lib


class SpkError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        self.name = STATUS.get(status, str(status))
        msg = _lib.spk_last_error().decode(errors="replace")
        super().__init__(f"{where}: {self.name}: {msg}")


def _ok(status: int, where: str) -> None:
    if status != SPK_OK:
        raise SpkError(status, where)


# ---------------------------------------------------------------- helpers --

def _torch():
    import torch
    return torch


def _dtype_code(t) -> int:
    torch = _torch()
    if t.dtype == torch.float64:
        return SPK_F64
    if t.dtype == torch.float32:
        return SPK_F32
    raise TypeError(f"unsupported dtype {t.dtype}")


def _dev(t, name: str):
    """Device pointer of a contiguous GPU tensor."""
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError(f"{name} must be a GPU tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t.data_ptr()


def _need(t, n: int, name: str):
    """The C entry points take bare pointers: a tensor shorter than the call
    reads or writes is caught here, before the pointer is passed on."""
    if t is not None and t.numel() < n:
        raise ValueError(f"{name} holds {t.numel()} elements; the call uses {n}")


def _stream(stream=None):
    if stream is not None:
        return stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
    return _torch().cuda.current_stream().cuda_stream


class Handle:
    """spk_handle: one GPU, its plan DB and scratch."""

    def __init__(self, device: int = 0, db_path: str | None = None):
        h = _P()
        _ok(_lib.spk_create(int(device), db_path.encode() if db_path else None, C.byref(h)), "spk_create")
        self.ptr = h.value
        self.device = device

    def close(self):
        if self.ptr:
            _ok(_lib.spk_destroy(self.ptr), "spk_destroy")
            self.ptr = None

    def set_plain(self, plain: bool):
        _ok(_lib.spk_set_plain(self.ptr, int(bool(plain))), "spk_set_plain")

    def info(self):
        n = _I32()
        buf = C.create_string_buffer(256)
        _ok(_lib.spk_device_info(self.ptr, C.byref(n), buf, 256), "spk_device_info")
        return int(n.value), buf.value.decode()

    def check(self, stream=None):
        _ok(_lib.spk_check(self.ptr, _stream(stream)), "spk_check")


_handles: dict[int, Handle] = {}


def default_handle(device: int | None = None) -> Handle:
    if device is None:
        device = _torch().cuda.current_device()
    if device not in _handles:
        _handles[device] = Handle(device)
    return _handles[device]


def _h(handle):
    return (handle or default_handle()).ptr


def spk_abi_version() -> int:
    return int(_lib.spk_abi_version())


def spk_status_str(s: int) -> str:
    return _lib.spk_status_str(int(s)).decode()


# ------------------------------------------------------------ vector ops --

def spk_waxpy(alpha: float, x, y, w=None, handle=None, stream=None):
    """w = alpha*x + y on the GPU; returns w."""
    if w is None:
        w = _torch().empty_like(x)
    if not (x.dtype == y.dtype == w.dtype) or not (x.numel() == y.numel() == w.numel()):
        raise ValueError("x, y, w must share dtype and size")
    _ok(_lib.spk_waxpy(_h(handle), _dtype_code(x), x.numel(), float(alpha), _dev(x, "x"), _dev(y, "y"),
                       _dev(w, "w"), _stream(stream)), "spk_waxpy")
    return w


def spk_axpy(alpha: float, x, y, handle=None, stream=None):
    """y <- alpha*x + y on the GPU; returns y."""
    if x.dtype != y.dtype or x.numel() != y.numel():
        raise ValueError("x, y must share dtype and size")
    _ok(_lib.spk_axpy(_h(handle), _dtype_code(x), x.numel(), float(alpha), _dev(x, "x"), _dev(y, "y"),
                      _stream(stream)), "spk_axpy")
    return y


def spk_dot(x, y, out=None, handle=None, stream=None):
    """sum x_i*y_i accumulated in FP64 on the GPU; returns a 1-element float64 device tensor."""
    torch = _torch()
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=x.device)
    if x.dtype != y.dtype or x.numel() != y.numel():
        raise ValueError("x, y must share dtype and size")
    _ok(_lib.spk_dot(_h(handle), _dtype_code(x), x.numel(), _dev(x, "x"), _dev(y, "y"), _dev(out, "out"),
                     _stream(stream)), "spk_dot")
    return out


def spk_dot_noalloc(x, y, out, handle=None, stream=None):
    """spk_dot on the library's fixed per-GPU scratch (allocates nothing):
    ``out`` is a caller-provided 1-element float64 device tensor."""
    if x.dtype != y.dtype or x.numel() != y.numel():
        raise ValueError("x, y must share dtype and size")
    _need(out, 1, "out")
    _ok(_lib.spk_dot_noalloc(_h(handle), _dtype_code(x), x.numel(), _dev(x, "x"), _dev(y, "y"), _dev(out, "out"),
                             _stream(stream)), "spk_dot_noalloc")
    return out


# ------------------------------------------------------------------ SpMV --

def _csr_struct(nrows, ncols, nnz, dtype_code, rp, ci, val):
    return spk_csr(int(nrows), int(ncols), int(nnz), int(dtype_code), rp, ci, val)


def spk_spmv_csr(row_ptr, col_idx, val, x, y=None, nrows=None, ncols=None, handle=None, stream=None):
    """y = A*x for a borrowed CSR (device tensors int32/int32/float)."""
    torch = _torch()
    nrows = row_ptr.numel() - 1 if nrows is None else nrows
    ncols = x.numel() if ncols is None else ncols
    if y is None:
        y = torch.empty(nrows, dtype=val.dtype, device=val.device)
    _need(row_ptr, nrows + 1, "row_ptr")
    _need(x, ncols, "x")
    _need(y, nrows, "y")
    A = _csr_struct(nrows, ncols, col_idx.numel(), _dtype_code(val), _dev(row_ptr, "row_ptr"),
                    _dev(col_idx, "col_idx"), _dev(val, "val"))
    _ok(_lib.spk_spmv_csr(_h(handle), C.byref(A), _dev(x, "x"), _dev(y, "y"), _stream(stream)), "spk_spmv_csr")
    return y


def spk_csr_structure(csr) -> dict:
    """Structure detection on a host CSR (numpy arrays; no GPU needed)."""
    rp = np.ascontiguousarray(csr.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(csr.col_idx, dtype=np.int32)
    val = np.ascontiguousarray(csr.val)
    dt = SPK_F64 if val.dtype == np.float64 else SPK_F32
    A = _csr_struct(csr.nrows, csr.ncols, ci.size, dt, rp.ctypes.data, ci.ctypes.data if ci.size else None,
                    val.ctypes.data if val.size else None)
    out = spk_structure()
    _ok(_lib.spk_csr_structure(C.byref(A), C.byref(out)), "spk_csr_structure")
    return {"formats": int(out.formats), "offsets": list(out.offsets[:out.ndiag]), "dim": int(out.dim),
            "grid": (int(out.n1), int(out.n2), int(out.n3)), "coef": list(out.coef)}


class Matrix:
    """A registered (library-owned, device-resident) CSR matrix."""

    def __init__(self, csr, handle=None, validate=True):
        """``csr``: object with nrows, ncols, row_ptr, col_idx, val (numpy arrays on the host)."""
        self.handle = handle or default_handle()
        rp = np.ascontiguousarray(csr.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(csr.col_idx, dtype=np.int32)
        val = np.ascontiguousarray(csr.val)
        if val.dtype not in (np.float64, np.float32):
            raise TypeError("values must be float64 or float32")
        self.nrows, self.ncols, self.nnz = int(csr.nrows), int(csr.ncols), int(ci.size)
        self.dtype_code = SPK_F64 if val.dtype == np.float64 else SPK_F32
        self.np_dtype = val.dtype
        self.row_ptr_host = rp
        A = _csr_struct(self.nrows, self.ncols, self.nnz, self.dtype_code, rp.ctypes.data,
                        ci.ctypes.data if ci.size else None, val.ctypes.data if val.size else None)
        m = _P()
        _ok(_lib.spk_matrix_register(self.handle.ptr, C.byref(A), 0, int(bool(validate)), C.byref(m)),
            "spk_matrix_register")
        self.ptr = m.value

    @property
    def torch_dtype(self):
        torch = _torch()
        return torch.float64 if self.dtype_code == SPK_F64 else torch.float32

    def bytes(self) -> int:
        b = _I64()
        _ok(_lib.spk_matrix_bytes(self.handle.ptr, self.ptr, C.byref(b)), "spk_matrix_bytes")
        return int(b.value)

    def formats(self) -> int:
        """Bitmask (1 << format) of the SpMV formats that apply to this matrix."""
        m = C.c_uint32()
        _ok(_lib.spk_matrix_formats(self.handle.ptr, self.ptr, C.byref(m)), "spk_matrix_formats")
        return int(m.value)

    def format_bytes(self, fmt: int, fused: bool = False) -> int:
        """Algorithmic bytes of one SpMV (or fused step) in format ``fmt``."""
        b = _I64()
        _ok(_lib.spk_matrix_format_bytes(self.handle.ptr, self.ptr, int(fmt), int(bool(fused)), C.byref(b)),
            "spk_matrix_format_bytes")
        return int(b.value)

    def release(self):
        if self.ptr:
            _ok(_lib.spk_matrix_release(self.handle.ptr, self.ptr), "spk_matrix_release")
            self.ptr = None


def spk_spmv_mat(A: Matrix, x, y=None, stream=None):
    torch = _torch()
    if y is None:
        y = torch.empty(A.nrows, dtype=A.torch_dtype, device=x.device)
    _need(x, A.ncols, "x")
    _need(y, A.nrows, "y")
    _ok(_lib.spk_spmv_mat(A.handle.ptr, A.ptr, _dev(x, "x"), _dev(y, "y"), _stream(stream)), "spk_spmv_mat")
    return y


def spk_spmv_waxpy(A: Matrix, alpha: float, x, y=None, w=None, stream=None):
    """y = A*x and w = alpha*y + x in one kernel; returns (y, w)."""
    torch = _torch()
    if y is None:
        y = torch.empty(A.nrows, dtype=A.torch_dtype, device=x.device)
    if w is None:
        w = torch.empty(A.nrows, dtype=A.torch_dtype, device=x.device)
    _need(x, A.ncols, "x")
    _need(y, A.nrows, "y")
    _need(w, A.nrows, "w")
    _ok(_lib.spk_spmv_waxpy(A.handle.ptr, A.ptr, float(alpha), _dev(x, "x"), _dev(y, "y"), _dev(w, "w"),
                            _stream(stream)), "spk_spmv_waxpy")
    return y, w


def spk_cg(A: Matrix, b, x, iters: int, hist=None, stream=None):
    """Conjugate gradients on a registered FP64 SPD matrix: ``iters``
    iterations starting from (and overwriting) ``x``.  Returns ``hist``, a
    float64 device tensor of r_k.r_k for k = 0..iters."""
    torch = _torch()
    if hist is None:
        hist = torch.empty(int(iters) + 1, dtype=torch.float64, device=x.device)
    _need(b, A.nrows, "b")
    _need(x, A.nrows, "x")
    _need(hist, int(iters) + 1, "hist")
    _ok(_lib.spk_cg(A.handle.ptr, A.ptr, _dev(b, "b"), _dev(x, "x"), int(iters), _dev(hist, "hist"),
                    _stream(stream)), "spk_cg")
    return hist


def spk_cg_tune(A: Matrix, b, iters: int, *, reps=10, warmup=2, tau=0.0, max_variants=0, record=True,
                verbose=False, formats=0, resume=False, stop_after=0) -> "spk_tune_report":
    """Tunes the SpMV+dot kernel of spk_cg on A (tile shapes, and the
    matrix-free form for grid stencils), each validated against the default
    shape's solve; records the winner for A's class."""
    o = spk_tune_opts()
    o.reps, o.warmup, o.tau, o.max_variants = reps, warmup, tau, max_variants
    o.formats = int(formats)
    o.record, o.verbose = int(record), int(verbose)
    o.resume, o.stop_after = int(resume), int(stop_after)
    rep = spk_tune_report()
    _need(b, A.nrows, "b")
    _ok(_lib.spk_cg_tune(A.handle.ptr, A.ptr, _dev(b, "b"), int(iters), C.byref(o), C.byref(rep)), "spk_cg_tune")
    return rep


# ------------------------------------------------------ variants, tuning --

def problem(op, *, A: Matrix | None = None, x=None, y=None, w=None, d_result=None, alpha=0.0, n=None, dtype=None):
    p = spk_problem()
    p.op = op
    if A is not None:
        p.A = A.ptr
        p.dtype = A.dtype_code
    elif x is not None:
        p.dtype = _dtype_code(x)
    if dtype is not None:
        p.dtype = dtype
    p.n = int(n if n is not None else (x.numel() if x is not None else 0))
    if A is not None:
        _need(x, A.ncols, "x")
        _need(y, A.nrows, "y")
        _need(w, A.nrows, "w")
    else:
        for t, name in ((x, "x"), (y, "y"), (w, "w")):
            _need(t, p.n, name)
    _need(d_result, 1, "d_result")
    p.alpha = float(alpha)
    p.x = _dev(x, "x")
    p.y = _dev(y, "y")
    p.w = _dev(w, "w")
    p.d_result = _dev(d_result, "d_result")
    return p


def spk_run(p: spk_problem, variant: spk_variant | None = None, handle=None, stream=None):
    _ok(_lib.spk_run(_h(handle), C.byref(p), C.byref(variant) if variant is not None else None, _stream(stream)),
        "spk_run")


def spk_variant_count(op: int, dtype: int) -> int:
    n = _I32()
    _ok(_lib.spk_variant_count(op, dtype, C.byref(n)), "spk_variant_count")
    return int(n.value)


def spk_variant_get(op: int, dtype: int, i: int) -> spk_variant:
    v = spk_variant()
    _ok(_lib.spk_variant_get(op, dtype, i, C.byref(v)), "spk_variant_get")
    return v


def variants(op: int, dtype: int) -> list[spk_variant]:
    return [spk_variant_get(op, dtype, i) for i in range(spk_variant_count(op, dtype))]


def spk_plain_variant(op: int, which: int = 0) -> spk_variant:
    v = spk_variant()
    _ok(_lib.spk_plain_variant(op, which, C.byref(v)), "spk_plain_variant")
    return v


def make_variant(**kw) -> spk_variant:
    v = spk_variant()
    for k, val in kw.items():
        setattr(v, k, int(val))
    return v


def spk_tune(p: spk_problem, *, reps=10, warmup=2, flush=False, max_variants=0, tau=0.0, ref=None, ref_scale=None,
             record=True, verbose=False, formats=0, handle=None, resume=False, stop_after=0) -> spk_tune_report:
    o = spk_tune_opts()
    o.reps, o.warmup, o.flush, o.max_variants, o.tau = reps, warmup, int(flush), max_variants, tau
    o.formats = int(formats)
    o.resume, o.stop_after = int(resume), int(stop_after)
    keep = []
    if ref is not None:
        r = np.ascontiguousarray(ref, dtype=np.float64)
        keep.append(r)
        o.ref_host = r.ctypes.data
    if ref_scale is not None:
        s = np.ascontiguousarray(ref_scale, dtype=np.float64)
        keep.append(s)
        o.ref_scale = s.ctypes.data
    o.record, o.verbose = int(record), int(verbose)
    rep = spk_tune_report()
    _ok(_lib.spk_tune(_h(handle), C.byref(p), C.byref(o), C.byref(rep)), "spk_tune")
    return rep


def spk_class_key(p: spk_problem, handle=None) -> str:
    buf = C.create_string_buffer(128)
    _ok(_lib.spk_class_key(_h(handle), C.byref(p), buf, 128), "spk_class_key")
    return buf.value.decode()


def spk_plan_get(key: str, handle=None) -> spk_variant | None:
    v = spk_variant()
    s = _lib.spk_plan_get(_h(handle), key.encode(), C.byref(v))
    return v if s == SPK_OK else None


def spk_plan_put(key: str, v: spk_variant, handle=None) -> None:
    _ok(_lib.spk_plan_put(_h(handle), key.encode(), C.byref(v)), "spk_plan_put")


# -------------------------------------------------------------- batching --

class Batch:
    """Many independent CSR instances driven by one (persistent, graph-replayed) launch."""

    def __init__(self, host_batch, device_arrays, persistent=True, use_graph=True, block=256, tile_nnz=2048,
                 handle=None, x_window=0):
        """``host_batch``: inputs.Batch (sizes/offsets); ``device_arrays``: (row_ptr, col_idx, val) tensors.
        The keywords fill spk_batch_opts; ``tile_nnz`` defaults to 2048 here
        (0 gives the library's 1024) and ``block=0`` takes the launch shape a
        recorded spk_batch_tune found."""
        self.handle = handle or default_handle()
        rp, ci, val = device_arrays
        self._host = [np.ascontiguousarray(a, dtype=np.int64) for a in
                      (host_batch.m, host_batch.nnz, host_batch.rp_off, host_batch.nz_off, host_batch.vec_off)]
        self._rp_host = np.ascontiguousarray(host_batch.row_ptr, dtype=np.int32)
        d = spk_batch_desc()
        d.count = host_batch.count
        d.dtype = _dtype_code(val)
        d.m, d.nnz, d.rp_off, d.nz_off, d.vec_off = (a.ctypes.data for a in self._host)
        d.row_ptr, d.col_idx, d.val = _dev(rp, "row_ptr"), _dev(ci, "col_idx"), _dev(val, "val")
        d.row_ptr_host = self._rp_host.ctypes.data
        o = spk_batch_opts(int(persistent), int(use_graph), int(block), int(tile_nnz), 0, int(x_window))
        b = _P()
        _ok(_lib.spk_batch_plan(self.handle.ptr, C.byref(d), C.byref(o), C.byref(b)), "spk_batch_plan")
        self.ptr = b.value
        self._dev = device_arrays  # keep the borrowed arrays alive

    def _check(self, x, y, w):
        rows = int(self._host[0].sum())
        for t, name in ((x, "x"), (y, "y"), (w, "w")):
            _need(t, rows, name)

    def run(self, alpha, x, y, w=None, stream=None):
        self._check(x, y, w)
        _ok(_lib.spk_batch_run(self.handle.ptr, self.ptr, float(alpha), _dev(x, "x"), _dev(y, "y"), _dev(w, "w"),
                               _stream(stream)), "spk_batch_run")

    def tune(self, alpha, x, y, w=None, reps=10, warmup=2, flush=False, record=True, verbose=False, ref=None,
             resume=False, stop_after=0):
        """spk_batch_tune; ``ref`` (optional, host FP64, one entry per vector
        element) replaces the plain kernels' y as the reference."""
        self._check(x, y, w)
        o = spk_tune_opts()
        o.reps, o.warmup, o.flush, o.record, o.verbose = reps, warmup, int(flush), int(record), int(verbose)
        o.resume, o.stop_after = int(resume), int(stop_after)
        if ref is not None:
            r = np.ascontiguousarray(ref, dtype=np.float64)
            if r.size < int(self._host[0].sum()):
                raise ValueError(f"ref holds {r.size} elements; the batch has {int(self._host[0].sum())} rows")
            o.ref_host = r.ctypes.data
        rep = spk_tune_report()
        _ok(_lib.spk_batch_tune(self.handle.ptr, self.ptr, float(alpha), _dev(x, "x"), _dev(y, "y"), _dev(w, "w"),
                                C.byref(o), C.byref(rep)), "spk_batch_tune")
        return rep

    def info(self):
        t, c, b = _I64(), _I32(), _I64()
        _ok(_lib.spk_batch_info(self.handle.ptr, self.ptr, C.byref(t), C.byref(c), C.byref(b)), "spk_batch_info")
        return {"tiles": int(t.value), "classes": int(c.value), "bytes": int(b.value)}

    def tile_modes(self, entries=False) -> dict:
        """Tiles per kernel mode as planned on the device ({mode: tiles}, modes with tiles only);
        with ``entries``, {mode: (tiles, matrix entries)}."""
        t, e = (_I64 * 65)(), (_I64 * 65)()
        _ok(_lib.spk_batch_tile_modes(self.handle.ptr, self.ptr, t, e), "spk_batch_tile_modes")
        if entries:
            return {m: (int(t[m]), int(e[m])) for m in range(65) if t[m]}
        return {m: int(t[m]) for m in range(65) if t[m]}

    def config(self) -> dict:
        o = spk_batch_opts()
        _ok(_lib.spk_batch_config(self.handle.ptr, self.ptr, C.byref(o)), "spk_batch_config")
        return {f: int(getattr(o, f)) for f, _ in o._fields_}

    def free(self):
        if self.ptr:
            _ok(_lib.spk_batch_free(self.handle.ptr, self.ptr), "spk_batch_free")
            self.ptr = None


# --------------------------------------------------------------- serving --

class Server:
    """Continuous-batching serving loop (library scheduler thread)."""

    def __init__(self, streams=4, max_inflight=256, max_batch=64, mode=0, hbm_budget=0, alpha=0.5, handle=None,
                 max_launches=0):
        self.handle = handle or default_handle()
        o = spk_serve_opts(int(streams), int(max_inflight), int(max_batch), int(mode), int(hbm_budget), float(alpha),
                           int(max_launches), 0)
        s = _P()
        _ok(_lib.spk_serve_create(self.handle.ptr, C.byref(o), C.byref(s)), "spk_serve_create")
        self.ptr = s.value
        self._keep = []

    def add_matrix(self, csr) -> int:
        rp = np.ascontiguousarray(csr.row_ptr, dtype=np.int32)
        ci = np.ascontiguousarray(csr.col_idx, dtype=np.int32)
        val = np.ascontiguousarray(csr.val)
        A = _csr_struct(csr.nrows, csr.ncols, ci.size, SPK_F64 if val.dtype == np.float64 else SPK_F32,
                        rp.ctypes.data, ci.ctypes.data if ci.size else None, val.ctypes.data if val.size else None)
        i = _I32()
        _ok(_lib.spk_serve_add_matrix(self.ptr, C.byref(A), C.byref(i)), "spk_serve_add_matrix")
        return int(i.value)

    def submit(self, mat_id: int, x: np.ndarray, y: np.ndarray, w: np.ndarray | None = None) -> int:
        self._keep.append((x, y, w))
        r = _I64()
        _ok(_lib.spk_serve_submit(self.ptr, int(mat_id), x.ctypes.data, y.ctypes.data,
                                  w.ctypes.data if w is not None else None, C.byref(r)), "spk_serve_submit")
        return int(r.value)

    def poll(self, cap=4096) -> list[int]:
        ids = np.zeros(cap, np.int64)
        n = _I32()
        _ok(_lib.spk_serve_poll(self.ptr, ids.ctypes.data, cap, C.byref(n)), "spk_serve_poll")
        return [int(v) for v in ids[:n.value]]

    def drain(self):
        _ok(_lib.spk_serve_drain(self.ptr), "spk_serve_drain")

    def replay(self, arrivals, mat_ids, xs, ys, ws=None):
        n = len(arrivals)
        arr = np.ascontiguousarray(arrivals, dtype=np.float64)
        ids = np.ascontiguousarray(mat_ids, dtype=np.int32)
        xp = (_P * n)(*[a.ctypes.data for a in xs])
        yp = (_P * n)(*[a.ctypes.data for a in ys])
        wp = (_P * n)(*[a.ctypes.data for a in ws]) if ws is not None else None
        self._keep.append((xs, ys, ws))
        _ok(_lib.spk_serve_replay(self.ptr, n, arr.ctypes.data, ids.ctypes.data, C.cast(xp, _P), C.cast(yp, _P),
                                  C.cast(wp, _P) if wp is not None else None), "spk_serve_replay")

    def stats(self) -> dict:
        s = spk_serve_stats()
        _ok(_lib.spk_serve_stats_get(self.ptr, C.byref(s)), "spk_serve_stats_get")
        return s.as_dict()

    def latencies(self) -> np.ndarray:
        cap = 1 << 22
        out = np.zeros(cap, np.float64)
        n = _I64()
        _ok(_lib.spk_serve_latencies(self.ptr, out.ctypes.data, cap, C.byref(n)), "spk_serve_latencies")
        return out[:n.value].copy()

    def latency_split(self):
        """(wait_us, run_us) per request: arrival to admission, admission to completion."""
        cap = 1 << 22
        wait = np.zeros(cap, np.float64)
        run = np.zeros(cap, np.float64)
        n = _I64()
        _ok(_lib.spk_serve_latency_split(self.ptr, wait.ctypes.data, run.ctypes.data, cap, C.byref(n)),
            "spk_serve_latency_split")
        return wait[:n.value].copy(), run[:n.value].copy()

    def close(self):
        if self.ptr:
            _ok(_lib.spk_serve_destroy(self.ptr), "spk_serve_destroy")
            self.ptr = None
            self._keep.clear()


# ----------------------------------------------------------- measurement --

def spk_stream_probe(kind: int, a, b, c, handle=None, stream=None):
    _ok(_lib.spk_stream_probe(_h(handle), int(kind), a.numel(), _dev(a, "a"), _dev(b, "b"), _dev(c, "c"),
                              _stream(stream)), "spk_stream_probe")


def spk_flush_cache(handle=None, stream=None):
    _ok(_lib.spk_flush_cache(_h(handle), _stream(stream)), "spk_flush_cache")


def to_device_csr(csr, device="cuda"):
    """Uploads an inputs.CSR (host numpy) as torch tensors (row_ptr, col_idx, val)."""
    torch = _torch()
    return (torch.from_numpy(np.ascontiguousarray(csr.row_ptr)).to(device),
            torch.from_numpy(np.ascontiguousarray(csr.col_idx)).to(device),
            torch.from_numpy(np.ascontiguousarray(csr.val)).to(device))
