"""Python binding of libcbspmv (ctypes).

Argument marshalling only: every step of the conversion and of the products
runs in the native library (host converter in C++, products in the HIP
kernels).  Functions carry the C ABI's names.  Vectors are torch tensors on
the GPU (or raw device pointers as ints); torch is used for device memory and
streams only.  Importing this module fails loudly when the library has not
been built.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcbspmv.so")
HEADER = os.path.join(os.path.dirname(_HERE), "include", "cbspmv.h")

if not os.path.exists(LIB_PATH):
    raise ImportError(
        f"{LIB_PATH} is missing: build the HIP library first (python -m paper_2605_18515_amd.build)")

# torch ships its own HIP runtime under the same soname as the system one the library links to; the
# first one loaded serves the whole process.  Loading torch first makes the library bind to torch's
# runtime (one runtime, shared streams); the other order leaves torch's HIP without a device.
try:
    import torch  # noqa: F401
except ImportError:  # the library also works without torch (raw device pointers)
    pass

_lib = ctypes.CDLL(LIB_PATH)

CB_SUCCESS, CB_ERROR_INVALID_VALUE, CB_ERROR_OUT_OF_MEMORY, CB_ERROR_HIP, CB_ERROR_NOT_SUPPORTED, \
    CB_ERROR_INTERNAL = range(6)
CB_VALUE_F64, CB_VALUE_F32, CB_VALUE_BF16 = range(3)
CB_FMT_COO, CB_FMT_CSR, CB_FMT_DENSE = range(3)
CB_LB_NONE, CB_LB_PAPER, CB_LB_CONTIGUOUS, CB_LB_PAPER_STREAM = range(4)
CB_REFINE_RESTART, CB_REFINE_REPLACE = range(2)
VALUE_TYPES = {"f64": CB_VALUE_F64, "f32": CB_VALUE_F32, "bf16": CB_VALUE_BF16}
LB_MODES = {"none": CB_LB_NONE, "paper": CB_LB_PAPER, "contiguous": CB_LB_CONTIGUOUS,
            "paper_stream": CB_LB_PAPER_STREAM}

_i32, _i64, _u32, _dbl, _p = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_double, ctypes.c_void_p


class CbOptions(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("value_type", _i32), ("col_agg", _i32), ("th1", _i32), ("th2", _i32),
                ("quantum_tiles", _i32), ("lb_mode", _i32), ("host_threads", _i32), ("th0", _dbl),
                ("wave_nnz", _i64), ("row_reduce", _i32), ("vector_f64", _i32), ("spmv_kernel", _i32),
                ("tile_dim", _i32), ("xcd_chunk", _i32), ("cols16", _i32), ("min_wave_nnz", _i64),
                ("reserved", _i64 * 2)]


class CbInfo(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("value_type", _i32), ("m", _i64), ("n", _i64), ("nnz", _i64),
                ("npanels", _i64), ("ntiles", _i64), ("tiles_coo", _i64), ("tiles_csr", _i64),
                ("tiles_dense", _i64), ("col_agg", _i32), ("lb_mode", _i32), ("super_sparse_share", _dbl),
                ("plain_tiles", _i64), ("payload_bytes", _i64), ("meta_bytes", _i64), ("restore_bytes", _i64),
                ("sched_bytes", _i64), ("nquanta", _i64), ("nwaves", _i64), ("shared_panels", _i64),
                ("prepass_panels", _i64), ("quantum_nnz_max", _i64), ("quantum_nnz_mean", _dbl),
                ("quantum_nnz_std", _dbl), ("wave_nnz_max", _i64), ("wave_nnz_mean", _dbl), ("wave_nnz_std", _dbl),
                ("spmv_bytes", _i64), ("device_bytes", _i64), ("convert_seconds", _dbl), ("on_device", _i32),
                ("reserved0", _i32), ("nbatches", _i64), ("stream_bytes", _i64), ("flat_run_mean", _dbl),
                ("row_reduce", _i32), ("vector_f64", _i32), ("spmv_kernel", _i32), ("tile_dim", _i32),
                ("xcd_chunk", _i32), ("cols16", _i32), ("reserved", _i64 * 2)]


class CbStructure(ctypes.Structure):
    _fields_ = [(n, _p) for n in ("tile_row", "tile_col", "tile_nnz", "tile_vp", "tile_type", "tile_ori", "payload",
                                  "restore_cols", "cols_offset", "quantum_ptr", "wave_ptr", "panel_shared",
                                  "prepass_list", "tile_xoff", "batch_stream", "batch_ptr", "tile_cols",
                                  "tile_cbase", "tile_c16")]


class CbCgOptions(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("max_iter", _i32), ("rtol", _dbl), ("check_every", _i32),
                ("max_refine", _i32), ("inner_rtol", _dbl), ("refine_method", _i32), ("reserved32", _i32),
                ("replace_factor", _dbl), ("reserved", _i64 * 2)]


class CbCgResult(ctypes.Structure):
    _fields_ = [("converged", _i32), ("iterations", _i32), ("refinements", _i32), ("restarts", _i32),
                ("rel_residual", _dbl), ("reserved", _i64 * 2)]


class CbServerOptions(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("max_active", _i32), ("arena_bytes", _i64), ("check_every", _i32),
                ("use_graph", _i32), ("spmm_streams", _i32), ("reserved32", _i32), ("reserved", _i64 * 4)]


class CbRequest(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("kind", _i32), ("matrix", _i32), ("k", _i32), ("alpha", _dbl),
                ("beta", _dbl), ("in_", _p), ("out", _p), ("rtol", _dbl), ("max_iter", _i32),
                ("matrix_low", _i32), ("reserved", _i64 * 4)]


class CbResponse(ctypes.Structure):
    _fields_ = [("done", _i32), ("status", _i32), ("iterations", _i32), ("converged", _i32),
                ("rel_residual", _dbl), ("latency_us", _dbl), ("queue_us", _dbl), ("replacements", _i32),
                ("restarts", _i32), ("reserved", _i64 * 1)]


class CbServerStats(ctypes.Structure):
    _fields_ = [("submitted", _i64), ("completed", _i64), ("rejected", _i64), ("spmm_done", _i64),
                ("cg_done", _i64), ("p50_us", _dbl), ("p99_us", _dbl), ("mean_us", _dbl), ("elapsed_s", _dbl),
                ("requests_per_s", _dbl), ("solves_per_s", _dbl), ("arena_peak_bytes", _i64),
                ("active_peak", _i32), ("graph_builds", _i32), ("steps", _i64), ("reserved", _i64 * 4)]


CB_REQ_SPMM, CB_REQ_CG, CB_REQ_CG_REFINE = range(3)
CB_TUNE_MAX_CANDIDATES = 16


class CbTuneOptions(ctypes.Structure):
    _fields_ = [("struct_size", _u32), ("reps", _i32), ("max_candidates", _i32), ("spmm_k", _i32),
                ("reserved", _i64 * 4)]


class CbTuneCandidate(ctypes.Structure):
    _fields_ = [("opt", CbOptions), ("us", _dbl), ("spmv_bytes", _i64), ("col_agg", _i32), ("row_reduce", _i32),
                ("tile_dim", _i32), ("spmv_kernel", _i32)]


class CbTuneReport(ctypes.Structure):
    _fields_ = [("ncandidates", _i32), ("best", _i32), ("cand", CbTuneCandidate * CB_TUNE_MAX_CANDIDATES)]


_lib.cb_tune_options_default.argtypes = [ctypes.POINTER(CbTuneOptions)]
_lib.cb_tune.argtypes = [ctypes.POINTER(_p), _i64, _i64, _i64, _p, _p, _p, ctypes.POINTER(CbOptions),
                         ctypes.POINTER(CbTuneOptions), ctypes.POINTER(CbOptions), ctypes.POINTER(CbTuneReport), _p]

_lib.cb_server_options_default.argtypes = [ctypes.POINTER(CbServerOptions)]
_lib.cb_server_create.argtypes = [ctypes.POINTER(CbServerOptions), ctypes.POINTER(_p)]
_lib.cb_server_add_matrix.argtypes = [_p, _p, ctypes.POINTER(_i32)]
_lib.cb_server_submit.argtypes = [_p, ctypes.POINTER(CbRequest), ctypes.POINTER(_i64)]
_lib.cb_server_poll.argtypes = [_p, _i64, ctypes.POINTER(CbResponse)]
_lib.cb_server_wait.argtypes = [_p, _i64, ctypes.POINTER(CbResponse)]
_lib.cb_server_stats.argtypes = [_p, ctypes.POINTER(CbServerStats)]
_lib.cb_server_destroy.argtypes = [_p]
_lib.cb_options_default.argtypes = [ctypes.POINTER(CbOptions)]
_lib.cb_cg_options_default.argtypes = [ctypes.POINTER(CbCgOptions)]
_lib.cb_cg_workspace_bytes.argtypes = [_p, _p, ctypes.POINTER(_i64)]
_lib.cb_cg.argtypes = [_p, _p, _p, _p, _i64, ctypes.POINTER(CbCgOptions), ctypes.POINTER(CbCgResult), _p]
_lib.cb_cg_refine.argtypes = [_p, _p, _p, _p, _p, _i64, ctypes.POINTER(CbCgOptions), ctypes.POINTER(CbCgResult), _p]
_lib.cb_cg_noalloc.argtypes = [_p, _p, _p, ctypes.POINTER(CbCgOptions), ctypes.POINTER(CbCgResult), _p]
CB_CG_NOALLOC_MAX_BYTES = 64 * 1024 * 1024
_lib.cb_create.argtypes = [ctypes.POINTER(_p), _i64, _i64, _i64, _p, _p, _p, ctypes.POINTER(CbOptions), _p]
_lib.cb_create_host.argtypes = [ctypes.POINTER(_p), _i64, _i64, _i64, _p, _p, _p, ctypes.POINTER(CbOptions)]
_lib.cb_spmv.argtypes = [_p, _dbl, _p, _dbl, _p, _p]
_lib.cb_spmm.argtypes = [_p, _i32, _dbl, _p, _i64, _dbl, _p, _i64, _p]
_lib.cb_destroy.argtypes = [_p]
_lib.cb_export_csr.argtypes = [_p, _p, _p, _p]
_lib.cb_get_info.argtypes = [_p, ctypes.POINTER(CbInfo)]
_lib.cb_export_structure.argtypes = [_p, ctypes.POINTER(CbStructure)]
_lib.cb_copy_probe.argtypes = [_p, _p, _i64, _p]
_lib.cb_read_probe.argtypes = [_p, _i64, _p, _p]
_lib.cb_last_error.argtypes = []
_lib.cb_last_error.restype = ctypes.c_char_p
for _f in ("cb_options_default", "cb_create", "cb_create_host", "cb_spmv", "cb_spmm", "cb_destroy", "cb_export_csr",
           "cb_get_info", "cb_export_structure", "cb_copy_probe", "cb_read_probe",
           "cb_cg_options_default", "cb_cg_workspace_bytes",
           "cb_cg", "cb_cg_refine", "cb_cg_noalloc", "cb_server_options_default", "cb_server_create", "cb_server_add_matrix",
           "cb_server_submit", "cb_server_poll", "cb_server_wait", "cb_server_stats", "cb_server_destroy",
           "cb_tune_options_default", "cb_tune"):
    getattr(_lib, _f).restype = ctypes.c_int


class CbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"cbspmv status {status}: {msg}")
        self.status = status


def cb_last_error() -> str:
    return (_lib.cb_last_error() or b"").decode()


def _check(st: int) -> None:
    if st != CB_SUCCESS:
        raise CbError(st, cb_last_error())


def header_functions() -> list[str]:
    """Names of the functions declared in include/cbspmv.h."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:cb_status_t|const char \*)\s*(cb_\w+)\s*\(", text, re.M)))


def library_handle() -> ctypes.CDLL:
    return _lib


def _stream_ptr(stream):
    if stream is None:
        try:
            import torch

            if torch.cuda.is_available():
                return torch.cuda.current_stream().cuda_stream
        except ImportError:
            pass
        return None
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream  # torch.cuda.Stream


def _require_dense(*tensors) -> None:
    for t in tensors:
        if t is not None and not isinstance(t, int) and not t.is_contiguous():
            raise ValueError(f"tensor with strides {tuple(t.stride())} is not contiguous: the library "
                             "reads and writes vectors as unit-stride arrays")


def _dev_ptr(t, dtype_name: str | None = None, numel: int | None = None, dense: bool = True):
    """Device address of a tensor handed to the C ABI.  dense: the library reads or writes it as
    one unit-stride array, so views with other strides (a column of a matrix, an expanded tensor
    whose elements share memory) are refused; the k-right-hand-side calls check their 2-D strides
    themselves and pass dense=False."""
    if t is None:
        return None
    if isinstance(t, int):
        return t
    if dense:
        _require_dense(t)
    if not t.is_cuda:
        raise ValueError("vectors must live on the GPU")
    if dtype_name is not None and str(t.dtype) != dtype_name:
        raise ValueError(f"expected {dtype_name}, got {t.dtype}")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"tensor has {t.numel()} elements, {numel} needed")
    return t.data_ptr()


def cb_options_default(**overrides) -> CbOptions:
    o = CbOptions()
    _check(_lib.cb_options_default(ctypes.byref(o)))
    for k, v in overrides.items():
        if k == "value_type" and isinstance(v, str):
            v = VALUE_TYPES[v]
        if k == "lb_mode" and isinstance(v, str):
            v = LB_MODES[v]
        if not hasattr(o, k):
            raise KeyError(k)
        setattr(o, k, v)
    return o


def _csr_args(row_ptr, col_idx, values):
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    va = np.ascontiguousarray(values, dtype=np.float64)
    return rp, ci, va


def cb_create(m, n, nnz, row_ptr, col_idx, values, opt: CbOptions | None = None, stream=None) -> int:
    rp, ci, va = _csr_args(row_ptr, col_idx, values)
    h = _p()
    _check(_lib.cb_create(ctypes.byref(h), m, n, nnz, rp.ctypes.data, ci.ctypes.data, va.ctypes.data,
                          ctypes.byref(opt) if opt is not None else None, _stream_ptr(stream)))
    return h.value


def cb_create_host(m, n, nnz, row_ptr, col_idx, values, opt: CbOptions | None = None) -> int:
    rp, ci, va = _csr_args(row_ptr, col_idx, values)
    h = _p()
    _check(_lib.cb_create_host(ctypes.byref(h), m, n, nnz, rp.ctypes.data, ci.ctypes.data, va.ctypes.data,
                               ctypes.byref(opt) if opt is not None else None))
    return h.value


def cb_destroy(A: int) -> None:
    _check(_lib.cb_destroy(A))


def cb_spmv(A: int, alpha: float, x, beta: float, y, stream=None) -> None:
    _check(_lib.cb_spmv(A, float(alpha), _dev_ptr(x), float(beta), _dev_ptr(y), _stream_ptr(stream)))


def cb_spmm(A: int, k: int, alpha: float, X, ldx: int, beta: float, Y, ldy: int, stream=None) -> None:
    _check(_lib.cb_spmm(A, int(k), float(alpha), _dev_ptr(X, dense=False), int(ldx), float(beta),
                        _dev_ptr(Y, dense=False), int(ldy), _stream_ptr(stream)))


def cb_cg_options_default(**kw) -> CbCgOptions:
    o = CbCgOptions()
    _check(_lib.cb_cg_options_default(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k) or k.startswith("reserved") or k == "struct_size":
            raise ValueError(f"unknown CG option {k}")
        setattr(o, k, v)
    return o


def cb_cg_workspace_bytes(A: int, A_low: int | None = None) -> int:
    b = _i64()
    _check(_lib.cb_cg_workspace_bytes(A, A_low, ctypes.byref(b)))
    return b.value


def _cg_result(r: CbCgResult) -> dict:
    return {"converged": bool(r.converged), "iterations": r.iterations, "refinements": r.refinements,
            "restarts": r.restarts, "rel_residual": r.rel_residual}


def cb_cg(A: int, b, x, work, work_bytes: int, opt: CbCgOptions | None = None, stream=None) -> dict:
    r = CbCgResult()
    _check(_lib.cb_cg(A, _dev_ptr(b), _dev_ptr(x), _dev_ptr(work), int(work_bytes),
                      ctypes.byref(opt) if opt is not None else None, ctypes.byref(r), _stream_ptr(stream)))
    return _cg_result(r)


def cb_cg_noalloc(A: int, b, x, opt: CbCgOptions | None = None, stream=None) -> dict:
    """cb_cg with the library's fixed device workspace (no allocation by the caller or the library)."""
    r = CbCgResult()
    _check(_lib.cb_cg_noalloc(A, _dev_ptr(b), _dev_ptr(x), ctypes.byref(opt) if opt is not None else None,
                              ctypes.byref(r), _stream_ptr(stream)))
    return _cg_result(r)


def cb_cg_refine(A: int, A_low: int, b, x, work, work_bytes: int, opt: CbCgOptions | None = None,
                 stream=None) -> dict:
    r = CbCgResult()
    _check(_lib.cb_cg_refine(A, A_low, _dev_ptr(b), _dev_ptr(x), _dev_ptr(work), int(work_bytes),
                             ctypes.byref(opt) if opt is not None else None, ctypes.byref(r), _stream_ptr(stream)))
    return _cg_result(r)


def cb_get_info(A: int) -> dict:
    info = CbInfo()
    info.struct_size = ctypes.sizeof(CbInfo)
    _check(_lib.cb_get_info(A, ctypes.byref(info)))
    return {name: getattr(info, name) for name, _ in CbInfo._fields_ if not name.startswith("reserved")}


_VDT = {CB_VALUE_F64: np.float64, CB_VALUE_F32: np.float32, CB_VALUE_BF16: np.uint16}


def cb_export_csr(A: int):
    """(row_ptr int64, col_idx int32, values) with values in the storage type
    (float64, float32, or uint16 bf16 bit patterns)."""
    info = cb_get_info(A)
    m, nnz = info["m"], info["nnz"]
    rp = np.empty(m + 1, np.int64)
    ci = np.empty(max(nnz, 1), np.int32)
    va = np.empty(max(nnz, 1), _VDT[info["value_type"]])
    _check(_lib.cb_export_csr(A, rp.ctypes.data, ci.ctypes.data, va.ctypes.data))
    return rp, ci[:nnz], va[:nnz]


def cb_export_structure(A: int) -> dict:
    info = cb_get_info(A)
    NT, P = info["ntiles"], info["npanels"]
    nrest = (info["restore_bytes"] // 4 - (P + 1) - NT) if info["col_agg"] else 0
    arrs = {
        "tile_row": np.empty(NT, np.int32), "tile_col": np.empty(NT, np.int32), "tile_nnz": np.empty(NT, np.int32),
        "tile_vp": np.empty(NT, np.int64), "tile_type": np.empty(NT, np.uint8), "tile_ori": np.empty(NT, np.int32),
        "payload": np.empty(info["payload_bytes"], np.uint8), "restore_cols": np.empty(nrest, np.int32),
        "cols_offset": np.empty(P + 1 if info["col_agg"] else 0, np.int32),
        "quantum_ptr": np.empty(info["nquanta"] + 1, np.int32), "wave_ptr": np.empty(info["nwaves"] + 1, np.int32),
        "panel_shared": np.empty(P, np.uint8), "prepass_list": np.empty(info["prepass_panels"], np.int32),
        "tile_xoff": np.empty(NT if info["col_agg"] else 0, np.int32),
        "batch_stream": np.empty(info["stream_bytes"] // 4, np.int32),
        "batch_ptr": np.empty(info["nwaves"] + 1 if info["lb_mode"] != CB_LB_PAPER else 0, np.int32),
        "tile_cols": np.empty(info["tile_dim"] * NT if info["lb_mode"] != CB_LB_PAPER and info["col_agg"] else 0, np.int32),
        "tile_cbase": np.empty(NT if info["cols16"] == 1 else 0, np.int32),
        "tile_c16": np.empty(info["tile_dim"] * NT if info["cols16"] else 0, np.uint16),
    }
    s = CbStructure(**{k: (v.ctypes.data if v.size else None) for k, v in arrs.items()})
    _check(_lib.cb_export_structure(A, ctypes.byref(s)))
    return arrs


def cb_copy_probe(src, dst, nbytes: int, stream=None) -> None:
    _check(_lib.cb_copy_probe(_dev_ptr(src), _dev_ptr(dst), int(nbytes), _stream_ptr(stream)))


def cb_read_probe(src, nbytes: int, sink, stream=None) -> None:
    _check(_lib.cb_read_probe(_dev_ptr(src), int(nbytes), _dev_ptr(sink), _stream_ptr(stream)))


class CbMatrix:
    """Owning wrapper of a cb_matrix_t handle."""

    def __init__(self, handle: int, vtype: int):
        self.handle = handle
        self.vtype = vtype
        self._info = None

    @classmethod
    def from_csr(cls, csr, device: bool = True, stream=None, **opts) -> "CbMatrix":
        o = cb_options_default(**opts)
        if device:
            h = cb_create(csr.m, csr.n, csr.nnz, csr.row_ptr, csr.col_idx, csr.values, o, stream)
        else:
            h = cb_create_host(csr.m, csr.n, csr.nnz, csr.row_ptr, csr.col_idx, csr.values, o)
        return cls(h, o.value_type)

    @property
    def info(self) -> dict:
        if self._info is None:
            self._info = cb_get_info(self.handle)
        return self._info

    @property
    def vector_dtype(self) -> str:
        return "torch.float64" if self.info["vector_f64"] else "torch.float32"

    def spmv(self, x, y, alpha: float = 1.0, beta: float = 0.0, stream=None):
        inf = self.info
        _require_dense(x, y)
        _dev_ptr(x, self.vector_dtype, inf["n"]) if inf["n"] else None
        _dev_ptr(y, self.vector_dtype, inf["m"]) if inf["m"] else None
        cb_spmv(self.handle, alpha, x, beta, y, stream)
        return y

    def spmm(self, X, Y, alpha: float = 1.0, beta: float = 0.0, stream=None):
        if X.dim() != 2 or Y.dim() != 2 or X.shape[1] != Y.shape[1]:
            raise ValueError("X (n x k) and Y (m x k) must be 2-D with the same k")
        k = X.shape[1]
        # row-major with a leading dimension of at least k: rows must not overlap (an expanded
        # tensor has row stride 0); a single row may have any row stride
        for name, T in (("X", X), ("Y", Y)):
            if T.stride(1) != 1 and k > 1:
                raise ValueError(f"{name} must be row-major (unit column stride)")
            if T.shape[0] > 1 and T.stride(0) < k:
                raise ValueError(f"{name} has row stride {T.stride(0)} < k = {k}: its rows overlap")
        inf = self.info
        if X.shape[0] != inf["n"] or Y.shape[0] != inf["m"]:
            raise ValueError("shape mismatch")
        _dev_ptr(X, self.vector_dtype, dense=False)
        _dev_ptr(Y, self.vector_dtype, dense=False)
        ldx = X.stride(0) if X.shape[0] > 1 else k
        ldy = Y.stride(0) if Y.shape[0] > 1 else k
        cb_spmm(self.handle, k, alpha, X, ldx, beta, Y, ldy, stream)
        return Y

    def export_csr(self):
        return cb_export_csr(self.handle)

    def structure(self) -> dict:
        return cb_export_structure(self.handle)

    def cg(self, b, x, work=None, stream=None, **opts) -> dict:
        """Solve A x = b by CG from the given x (device tensors of the vector type); work: a device
        uint8 tensor of at least cb_cg_workspace_bytes bytes, allocated here when None."""
        n = self.info["n"]
        _require_dense(b, x, work)
        _dev_ptr(b, self.vector_dtype)
        _dev_ptr(x, self.vector_dtype)
        if b.numel() != n or x.numel() != n:
            raise ValueError("b and x must have n elements")
        need = cb_cg_workspace_bytes(self.handle)
        work = self._workspace(work, need, x)
        return cb_cg(self.handle, b, x, work, need, cb_cg_options_default(**opts), stream)

    def cg_refine(self, low: "CbMatrix", b, x, work=None, stream=None, **opts) -> dict:
        """FP64 iterative refinement with CG on the low-precision copy `low` (float64 b and x)."""
        n = self.info["n"]
        import torch

        for t in (b, x):
            if t.dtype != torch.float64 or t.numel() != n:
                raise ValueError("b and x must be float64 device tensors with n elements")
        need = cb_cg_workspace_bytes(self.handle, low.handle)
        work = self._workspace(work, need, x)
        return cb_cg_refine(self.handle, low.handle, b, x, work, need, cb_cg_options_default(**opts), stream)

    @staticmethod
    def _workspace(work, need, like):
        import torch

        if work is None:
            return torch.empty(need, dtype=torch.uint8, device=like.device)
        if work.numel() * work.element_size() < need:
            raise ValueError(f"workspace needs {need} bytes")
        return work

    def close(self):
        if self.handle:
            cb_destroy(self.handle)
            self.handle = 0

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _struct_dict(st) -> dict:
    return {n: getattr(st, n) for n, _ in st._fields_ if not n.startswith("reserved")}


def cb_server_options_default(**kw) -> CbServerOptions:
    o = CbServerOptions()
    _check(_lib.cb_server_options_default(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k) or k.startswith("reserved") or k == "struct_size":
            raise ValueError(f"unknown server option {k}")
        setattr(o, k, v)
    return o


def check_host_vectors(dt, n: int, **vecs) -> None:
    """Host vectors of a served request: numpy arrays of dtype dt with n elements each, C-contiguous
    (the server copies them as n consecutive elements)."""
    for name, v in vecs.items():
        if not isinstance(v, np.ndarray) or v.dtype != dt or v.size != n:
            raise ValueError(f"{name} must be a {np.dtype(dt).name} array of {n} elements")
        if not v.flags.c_contiguous:
            raise ValueError(f"{name} must be C-contiguous")


class CbServer:
    """A serving loop on the current device (cb_server_*).  Host vectors given to submit_* are
    numpy arrays of the matrix's vector type; they are kept alive here until their request is
    collected with wait()."""

    def __init__(self, **opts):
        h = _p()
        _check(_lib.cb_server_create(ctypes.byref(cb_server_options_default(**opts)), ctypes.byref(h)))
        self.handle = h.value
        self._keep = {}
        self._mats = []

    def add_matrix(self, M: "CbMatrix") -> int:
        i = _i32()
        _check(_lib.cb_server_add_matrix(self.handle, M.handle, ctypes.byref(i)))
        self._mats.append(M)
        return i.value

    def _dtype(self, mid):
        return np.float64 if self._mats[mid].info["vector_f64"] else np.float32

    def _submit(self, r: CbRequest, keep) -> int:
        t = _i64()
        r.struct_size = ctypes.sizeof(CbRequest)
        _check(_lib.cb_server_submit(self.handle, ctypes.byref(r), ctypes.byref(t)))
        self._keep[t.value] = keep
        return t.value

    def submit_spmm(self, mid: int, X: np.ndarray, Y: np.ndarray, alpha: float = 1.0, beta: float = 0.0) -> int:
        dt = self._dtype(mid)
        inf = self._mats[mid].info
        if X.dtype != dt or Y.dtype != dt or not X.flags.c_contiguous or not Y.flags.c_contiguous:
            raise ValueError(f"X and Y must be C-contiguous {np.dtype(dt).name} arrays")
        k = 1 if X.ndim == 1 else X.shape[1]
        if X.size != inf["n"] * k or Y.size != inf["m"] * k:
            raise ValueError("X must be n x k and Y m x k")
        r = CbRequest(kind=CB_REQ_SPMM, matrix=mid, k=k, alpha=alpha, beta=beta, in_=X.ctypes.data,
                      out=Y.ctypes.data)
        return self._submit(r, (X, Y))

    def submit_cg(self, mid: int, b: np.ndarray, x: np.ndarray, rtol: float = 0.0, max_iter: int = 0) -> int:
        check_host_vectors(self._dtype(mid), self._mats[mid].info["n"], b=b, x=x)
        r = CbRequest(kind=CB_REQ_CG, matrix=mid, k=1, in_=b.ctypes.data, out=x.ctypes.data, rtol=rtol,
                      max_iter=max_iter)
        return self._submit(r, (b, x))

    def submit_cg_refine(self, mid: int, mid_low: int, b: np.ndarray, x: np.ndarray, rtol: float = 0.0,
                         max_iter: int = 0) -> int:
        """CG with FP64 residual replacement: mid is the FP64 handle, mid_low its FP32/BF16 copy
        (float vectors) that the steps multiply by; b and x are float64."""
        check_host_vectors(np.float64, self._mats[mid].info["n"], b=b, x=x)
        r = CbRequest(kind=CB_REQ_CG_REFINE, matrix=mid, matrix_low=mid_low, k=1, in_=b.ctypes.data,
                      out=x.ctypes.data, rtol=rtol, max_iter=max_iter)
        return self._submit(r, (b, x))

    def poll(self, ticket: int) -> dict:
        r = CbResponse()
        _check(_lib.cb_server_poll(self.handle, ticket, ctypes.byref(r)))
        return _struct_dict(r)

    def wait(self, ticket: int) -> dict:
        r = CbResponse()
        _check(_lib.cb_server_wait(self.handle, ticket, ctypes.byref(r)))
        self._keep.pop(ticket, None)
        return _struct_dict(r)

    def stats(self) -> dict:
        s = CbServerStats()
        _check(_lib.cb_server_stats(self.handle, ctypes.byref(s)))
        return _struct_dict(s)

    def close(self):
        if self.handle:
            _check(_lib.cb_server_destroy(self.handle))
            self.handle = 0
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def cb_tune_options_default(**kw) -> CbTuneOptions:
    o = CbTuneOptions()
    _check(_lib.cb_tune_options_default(ctypes.byref(o)))
    for k, v in kw.items():
        if not hasattr(o, k) or k.startswith("reserved") or k == "struct_size":
            raise ValueError(f"unknown tuner option {k}")
        setattr(o, k, v)
    return o


_OPT_NAMES = [n for n, _ in CbOptions._fields_ if not n.startswith("reserved") and n != "struct_size"]


def cb_tune(csr, stream=None, keep: bool = True, reps: int = 20, spmm_k: int = 0, **base):
    """Tunes the options for csr (cb_tune; spmm_k > 1 times cb_spmm with that many right-hand sides).
    Returns (CbMatrix or None, best options as a dict, candidates: list of dicts with the options,
    us, spmv_bytes, col_agg, row_reduce, tile_dim, spmv_kernel, best)."""
    rp, ci, va = _csr_args(csr.row_ptr, csr.col_idx, csr.values)
    b = cb_options_default(**base)
    best = CbOptions()
    rep = CbTuneReport()
    h = _p()
    _check(_lib.cb_tune(ctypes.byref(h) if keep else None, csr.m, csr.n, csr.nnz, rp.ctypes.data, ci.ctypes.data,
                        va.ctypes.data, ctypes.byref(b),
                        ctypes.byref(cb_tune_options_default(reps=reps, spmm_k=spmm_k)),
                        ctypes.byref(best), ctypes.byref(rep), _stream_ptr(stream)))
    cands = []
    for i in range(rep.ncandidates):
        c = rep.cand[i]
        cands.append({"opt": {n: getattr(c.opt, n) for n in _OPT_NAMES}, "us": c.us, "spmv_bytes": c.spmv_bytes,
                      "col_agg": c.col_agg, "row_reduce": c.row_reduce, "tile_dim": c.tile_dim,
                      "spmv_kernel": c.spmv_kernel, "best": i == rep.best})
    M = CbMatrix(h.value, best.value_type) if keep else None
    return M, {n: getattr(best, n) for n in _OPT_NAMES}, cands
