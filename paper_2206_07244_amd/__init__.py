"""opsp: row-wise SpGEMM (C = A*B, CSR, FP64) for AMD MI355X (gfx950).

Thin Python binding over the C ABI declared in ``include/opsp.h``.  It only
marshals arguments: every step of the product runs in the HIP kernels of
``libopsp.so``.  PyTorch supplies device memory and streams.  There is no
CPU fallback: if the library is missing the import of a compute entry point
raises.

Matrices are :class:`DeviceCSR` objects holding three torch tensors on a
GPU: ``rpt`` int64[rows+1], ``col`` int32[nnz], ``val`` float64[nnz].
"""
from __future__ import annotations

import ctypes
import os
import re
from ctypes import POINTER, byref, c_char_p, c_double, c_int32, c_int64, c_void_p
from typing import Optional

import numpy as np

__all__ = [
    "DeviceCSR", "Plan", "OpspError", "Config", "Stats", "spgemm", "spgemm_symbolic",
    "spgemm_numeric", "lib", "library_path", "exported_symbols", "table_sizes", "bin_bounds",
    "SYM_BINS", "NUM_BINS", "cache_release", "cache_bytes", "Batch", "Predictor",
    "row_features", "mlp_features", "mlp_forward", "mlp_grad", "mlp_adam", "spgemm_learned",
    "MLP_NPARAM", "PRED_MLP", "PRED_UPPER", "PRED_RATIO",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libopsp.so")
_HEADER = os.path.join(os.path.dirname(_HERE), "include", "opsp.h")

SYM_BINS = 9
NUM_BINS = 8
CONFIG_VERSION = 3
MLP_NPARAM = 4481
PREDICTOR_VERSION = 1
PRED_MLP, PRED_UPPER, PRED_RATIO = 0, 1, 2
DEFAULT_WEIGHTS = os.path.join(_HERE, "predictor_weights.json")


class opsp_csr(ctypes.Structure):
    _fields_ = [("rows", c_int64), ("cols", c_int64), ("nnz", c_int64),
                ("rpt", c_void_p), ("col", c_void_p), ("val", c_void_p)]


class Config(ctypes.Structure):
    """Mirror of ``opsp_config`` (zero fields = defaults)."""
    _fields_ = [("version", c_int32), ("sym_ratio", c_double), ("num_ratio", c_double),
                ("force_sym_bin", c_int32), ("force_num_bin", c_int32),
                ("sym_abort_fraction", c_double), ("b_lanes", c_int32),
                ("stage_timing", c_int32), ("validate", c_int32), ("fixed_grid", c_int32),
                ("sym_bounds", c_int64 * 7), ("num_bounds", c_int64 * 7),
                ("hash_all_rows", c_int32), ("streams", c_int32), ("group_lanes", c_int32)]

    def __init__(self, **kw):
        super().__init__()
        self.version = CONFIG_VERSION
        self.force_sym_bin = -1
        self.force_num_bin = -1
        for k, v in kw.items():
            if k in ("sym_bounds", "num_bounds"):
                arr = getattr(self, k)
                for j, x in enumerate(v):
                    arr[j] = int(x)
            else:
                setattr(self, k, v)

    def as_dict(self) -> dict:
        return {"sym_ratio": self.sym_ratio, "num_ratio": self.num_ratio,
                "sym_abort_fraction": self.sym_abort_fraction,
                "sym_bounds": list(self.sym_bounds), "num_bounds": list(self.num_bounds),
                "hash_all_rows": self.hash_all_rows, "streams": self.streams,
                "group_lanes": self.group_lanes}


class Stats(ctypes.Structure):
    """Mirror of ``opsp_stats``."""
    _fields_ = [("nprod", c_int64), ("nnz", c_int64), ("max_row_nprod", c_int64),
                ("max_row_nnz", c_int64), ("sym_bin_rows", c_int64 * SYM_BINS),
                ("num_bin_rows", c_int64 * NUM_BINS), ("ms_stage", ctypes.c_float * 8),
                ("cap_total", c_int64), ("arena_entries", c_int64),
                ("slot_overflow_rows", c_int64), ("table_overflow_rows", c_int64),
                ("retry_rows", c_int64), ("calib_scale", c_double)]

    def as_dict(self):
        return {"nprod": self.nprod, "nnz": self.nnz, "max_row_nprod": self.max_row_nprod,
                "max_row_nnz": self.max_row_nnz, "sym_bin_rows": list(self.sym_bin_rows),
                "num_bin_rows": list(self.num_bin_rows), "ms_stage": list(self.ms_stage)[:5],
                "cap_total": self.cap_total, "arena_entries": self.arena_entries,
                "slot_overflow_rows": self.slot_overflow_rows,
                "table_overflow_rows": self.table_overflow_rows, "retry_rows": self.retry_rows,
                "calib_scale": self.calib_scale}


class opsp_predictor(ctypes.Structure):
    """Mirror of ``opsp_predictor``."""
    _fields_ = [("version", c_int32), ("kind", c_int32), ("params", c_void_p),
                ("margin", c_double), ("ratio", c_double), ("cap_scale", c_double),
                ("pred_out", c_void_p), ("cap_out", c_void_p), ("calib_rows", c_int32),
                ("reserved", c_int32)]


class OpspError(RuntimeError):
    def __init__(self, code: int, where: str):
        self.code = code
        msg = lib().opsp_status_string(code).decode()
        super().__init__(f"{where}: {msg}")


_lib = None


def library_path() -> str:
    return _LIB_PATH


_variants = {}


def lib_variant(name: str):
    """A build variant of the library (``_build.VARIANTS``), loaded beside the
    product library with the same C ABI: ``"multi_access"`` is the
    read-then-swap hash probe of the hashing ablation (Section 6.3.2)."""
    if name not in _variants:
        from . import _build
        path = _build.VARIANTS[name][1]
        if not os.path.exists(path):
            raise RuntimeError(f"{path} is missing: build it with `python -m paper_2206_07244_amd._build`")
        _variants[name] = _bind(ctypes.CDLL(path))
    return _variants[name]


def lib():
    """The loaded ``libopsp.so`` (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            raise RuntimeError(
                f"{_LIB_PATH} is missing: build it with `python -m paper_2206_07244_amd._build` "
                "(there is no CPU fallback)")
        _lib = _bind(ctypes.CDLL(_LIB_PATH))
    return _lib


def _bind(L):
    """Argument and result types of every exported function."""
    P = c_void_p
    csr_p = POINTER(opsp_csr)
    L.opsp_version.restype = c_char_p
    L.opsp_version.argtypes = []
    L.opsp_status_string.restype = c_char_p
    L.opsp_status_string.argtypes = [ctypes.c_int]
    L.opsp_spgemm.restype = ctypes.c_int
    L.opsp_spgemm.argtypes = [csr_p, csr_p, csr_p, P]
    # the FP32 structs have opsp_csr's layout (val: float* instead of double*)
    L.opsp_spgemm_f32.restype = ctypes.c_int
    L.opsp_spgemm_f32.argtypes = [csr_p, csr_p, csr_p, POINTER(Config), POINTER(Stats), P]
    L.opsp_csr_f32_free.restype = ctypes.c_int
    L.opsp_csr_f32_free.argtypes = [csr_p, P]
    L.opsp_spgemm_ex.restype = ctypes.c_int
    L.opsp_spgemm_ex.argtypes = [csr_p, csr_p, csr_p, POINTER(Config), POINTER(Stats), P]
    L.opsp_spgemm_symbolic.restype = ctypes.c_int
    L.opsp_spgemm_symbolic.argtypes = [csr_p, csr_p, POINTER(Config), POINTER(c_void_p),
                                       POINTER(c_int64), P]
    L.opsp_spgemm_numeric.restype = ctypes.c_int
    L.opsp_spgemm_numeric.argtypes = [c_void_p, csr_p, csr_p, csr_p, P]
    L.opsp_spgemm_numeric_noalloc.restype = ctypes.c_int
    L.opsp_spgemm_numeric_noalloc.argtypes = [c_void_p, csr_p, csr_p, csr_p, P]
    L.opsp_plan_destroy.restype = None
    L.opsp_plan_destroy.argtypes = [c_void_p]
    L.opsp_csr_free.restype = ctypes.c_int
    L.opsp_csr_free.argtypes = [csr_p, P]
    L.opsp_batch_create.restype = ctypes.c_int
    L.opsp_batch_create.argtypes = [c_int32, csr_p, csr_p, POINTER(Config), POINTER(c_void_p), P]
    L.opsp_batch_execute.restype = ctypes.c_int
    L.opsp_batch_execute.argtypes = [c_void_p, csr_p, POINTER(Stats), P]
    L.opsp_batch_destroy.restype = None
    L.opsp_batch_destroy.argtypes = [c_void_p]
    L.opsp_spgemm_batched.restype = ctypes.c_int
    L.opsp_spgemm_batched.argtypes = [c_int32, csr_p, csr_p, csr_p, POINTER(Config),
                                      POINTER(c_void_p), P]
    L.opsp_cache_release.restype = ctypes.c_int
    L.opsp_cache_release.argtypes = []
    L.opsp_cache_bytes.restype = c_int64
    L.opsp_cache_bytes.argtypes = []
    L.opsp_cache_live_bytes.restype = c_int64
    L.opsp_cache_live_bytes.argtypes = []
    L.opsp_debug_fail_alloc.restype = None
    L.opsp_debug_fail_alloc.argtypes = [c_int64]
    L.opsp_table_sizes.restype = ctypes.c_int
    L.opsp_table_sizes.argtypes = [c_int32, POINTER(c_int64), c_int32]
    L.opsp_bin_bounds.restype = ctypes.c_int
    L.opsp_bin_bounds.argtypes = [c_int32, POINTER(c_int64), c_int32, c_double, POINTER(c_int64)]
    L.opsp_row_features.restype = ctypes.c_int
    L.opsp_row_features.argtypes = [csr_p, csr_p, P, P, P, P]
    L.opsp_mlp_features.restype = ctypes.c_int
    L.opsp_mlp_features.argtypes = [csr_p, csr_p, P, P]
    L.opsp_mlp_forward.restype = ctypes.c_int
    L.opsp_mlp_forward.argtypes = [P, P, c_int64, P, P]
    L.opsp_mlp_grad.restype = ctypes.c_int
    L.opsp_mlp_grad.argtypes = [P, P, P, c_int64, ctypes.c_float, P, P, P]
    L.opsp_mlp_adam.restype = ctypes.c_int
    L.opsp_mlp_adam.argtypes = [P, P, P, P, c_int64, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, ctypes.c_float, P, P]
    L.opsp_spgemm_learned.restype = ctypes.c_int
    L.opsp_spgemm_learned.argtypes = [csr_p, csr_p, csr_p, POINTER(opsp_predictor),
                                      POINTER(Config), POINTER(Stats), P]
    return L


def exported_symbols() -> list:
    """Function names declared in include/opsp.h."""
    with open(_HEADER) as f:
        text = f.read()
    return sorted(set(re.findall(r"\b(opsp_[a-z_0-9]+)\s*\(", text)))


def cache_release():
    """Return every cached device block of the current device to HIP."""
    _check(lib().opsp_cache_release(), "opsp_cache_release")


def cache_bytes() -> int:
    return int(lib().opsp_cache_bytes())


def cache_live_bytes() -> int:
    """Bytes the library has handed out and not taken back (see the header)."""
    return int(lib().opsp_cache_live_bytes())


def debug_fail_alloc(n: int):
    """Testing: the allocation after the next `n` successful ones fails
    (once); n < 0 switches this off."""
    lib().opsp_debug_fail_alloc(int(n))


def _check(code: int, where: str):
    if code != 0:
        raise OpspError(code, where)


# ---------------------------------------------------------------------------
# Host-side helpers (no GPU needed)
# ---------------------------------------------------------------------------

def table_sizes(step: int) -> list:
    n = SYM_BINS if step == 0 else NUM_BINS
    out = (c_int64 * n)()
    _check(lib().opsp_table_sizes(step, out, n), "opsp_table_sizes")
    return list(out)


def bin_bounds(step: int, tsizes, ratio: float) -> list:
    n = len(tsizes) + 1
    ts = (c_int64 * len(tsizes))(*tsizes)
    out = (c_int64 * max(n - 1, 1))()
    _check(lib().opsp_bin_bounds(step, ts, n, float(ratio), out), "opsp_bin_bounds")
    return list(out)[: n - 1]


# ---------------------------------------------------------------------------
# Device matrices
# ---------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def _stream_handle(stream) -> Optional[int]:
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream if hasattr(stream, "cuda_stream") else stream


class _Owner:
    """Frees library-allocated C arrays once every tensor view is gone."""

    def __init__(self, c: opsp_csr, stream):
        self.c = c
        self.stream = stream

    def __del__(self):
        try:
            if _lib is not None:
                _lib.opsp_csr_free(byref(self.c), self.stream)
        except Exception:
            pass


class _CudaArray:
    def __init__(self, ptr: int, n: int, typestr: str, owner):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr,
                                         "data": (ptr, False), "version": 2, "strides": None}
        self._owner = owner


def _wrap(ptr, n, dtype, owner, device):
    torch = _torch()
    if n == 0 or not ptr:
        return torch.empty(0, dtype=dtype, device=device)
    typestr = {torch.int64: "<i8", torch.int32: "<i4", torch.float64: "<f8", torch.float32: "<f4"}[dtype]
    t = torch.as_tensor(_CudaArray(int(ptr), int(n), typestr, owner), device=device)
    assert t.data_ptr() == int(ptr)
    return t


class DeviceCSR:
    """CSR matrix in device memory (torch tensors)."""

    def __init__(self, rows: int, cols: int, rpt, col, val):
        self.rows, self.cols = int(rows), int(cols)
        self.rpt, self.col, self.val = rpt, col, val

    @property
    def nnz(self) -> int:
        return int(self.col.numel())

    @classmethod
    def from_host(cls, A, device="cuda", dtype=np.float64) -> "DeviceCSR":
        """Upload a host CSR; ``dtype`` np.float32 rounds the values for the
        FP32 product."""
        torch = _torch()
        rpt = torch.from_numpy(np.ascontiguousarray(A.rpt, np.int64)).to(device)
        col = torch.from_numpy(np.ascontiguousarray(A.col, np.int32)).to(device)
        val = torch.from_numpy(np.ascontiguousarray(A.val, dtype)).to(device)
        return cls(A.rows, A.cols, rpt, col, val)

    def to_host(self):
        return (self.rpt.cpu().numpy(), self.col.cpu().numpy(), self.val.cpu().numpy())

    def _c(self) -> opsp_csr:
        c = opsp_csr()
        c.rows, c.cols = self.rows, self.cols
        c.nnz = int(self.rpt[-1].item() - self.rpt[0].item()) if self.rows > 0 else 0
        c.rpt = self.rpt.data_ptr()
        c.col = self.col.data_ptr() if self.col.numel() else None
        c.val = self.val.data_ptr() if self.val.numel() else None
        return c

    def _c_fast(self, nnz: int) -> opsp_csr:
        c = opsp_csr()
        c.rows, c.cols, c.nnz = self.rows, self.cols, nnz
        c.rpt = self.rpt.data_ptr()
        c.col = self.col.data_ptr() if self.col.numel() else None
        c.val = self.val.data_ptr() if self.val.numel() else None
        return c


def _adopt(c: opsp_csr, stream, device, vdtype=None) -> DeviceCSR:
    torch = _torch()
    owner = _Owner(c, stream)
    rpt = _wrap(c.rpt, c.rows + 1, torch.int64, owner, device)
    col = _wrap(c.col, c.nnz, torch.int32, owner, device)
    val = _wrap(c.val, c.nnz, vdtype or torch.float64, owner, device)
    return DeviceCSR(c.rows, c.cols, rpt, col, val)


def spgemm(A: DeviceCSR, B: DeviceCSR, config: Optional[Config] = None,
           stats: Optional[Stats] = None, stream=None) -> DeviceCSR:
    """C = A*B on the GPU (two-phase OpSparse pipeline); C is library-allocated."""
    s = _stream_handle(stream)
    Ac, Bc, Cc = A._c(), B._c(), opsp_csr()
    code = lib().opsp_spgemm_ex(byref(Ac), byref(Bc), byref(Cc),
                                byref(config) if config is not None else None,
                                byref(stats) if stats is not None else None, s)
    _check(code, "opsp_spgemm")
    return _adopt(Cc, s, A.rpt.device)


def spgemm_f32(A: DeviceCSR, B: DeviceCSR, config: Optional[Config] = None,
               stats: Optional[Stats] = None, stream=None) -> DeviceCSR:
    """C = A*B with FP32 values (``opsp_spgemm_f32``); A and B hold float32
    values (``DeviceCSR.from_host(..., dtype=np.float32)``)."""
    torch = _torch()
    assert A.val.dtype == torch.float32 and B.val.dtype == torch.float32
    s = _stream_handle(stream)
    Ac, Bc, Cc = A._c(), B._c(), opsp_csr()
    code = lib().opsp_spgemm_f32(byref(Ac), byref(Bc), byref(Cc),
                                 byref(config) if config is not None else None,
                                 byref(stats) if stats is not None else None, s)
    _check(code, "opsp_spgemm_f32")
    return _adopt(Cc, s, A.rpt.device, torch.float32)


def spgemm_raw(Ac: opsp_csr, Bc: opsp_csr, stream_handle) -> opsp_csr:
    """Lowest-overhead call used by the benchmark: returns the raw C struct
    (release with ``free_raw``)."""
    Cc = opsp_csr()
    _check(lib().opsp_spgemm(byref(Ac), byref(Bc), byref(Cc), stream_handle), "opsp_spgemm")
    return Cc


def free_raw(Cc: opsp_csr, stream_handle):
    _check(lib().opsp_csr_free(byref(Cc), stream_handle), "opsp_csr_free")


class Plan:
    """Result of the symbolic phase; reusable for numeric calls on matrices
    with the same structure."""

    def __init__(self, handle: int, nnz: int, rows: int, cols: int):
        self.handle, self.nnz, self.rows, self.cols = handle, nnz, rows, cols

    def __del__(self):
        if self.handle and _lib is not None:
            _lib.opsp_plan_destroy(self.handle)
            self.handle = None


def spgemm_symbolic(A: DeviceCSR, B: DeviceCSR, config: Optional[Config] = None,
                    stream=None) -> Plan:
    s = _stream_handle(stream)
    Ac, Bc = A._c(), B._c()
    h = c_void_p()
    nnz = c_int64()
    _check(lib().opsp_spgemm_symbolic(byref(Ac), byref(Bc),
                                      byref(config) if config is not None else None,
                                      byref(h), byref(nnz), s), "opsp_spgemm_symbolic")
    return Plan(h.value, nnz.value, A.rows, B.cols)


def spgemm_numeric(plan: Plan, A: DeviceCSR, B: DeviceCSR, out: Optional[DeviceCSR] = None,
                   stream=None) -> DeviceCSR:
    """Numeric phase.  With ``out`` (torch buffers of the right sizes) the
    result is written there; otherwise the library allocates C."""
    s = _stream_handle(stream)
    Ac, Bc = A._c(), B._c()
    Cc = opsp_csr()
    if out is not None:
        assert out.rpt.numel() == plan.rows + 1 and out.col.numel() == plan.nnz == out.val.numel()
        Cc.rpt = out.rpt.data_ptr()
        Cc.col = out.col.data_ptr() if plan.nnz else None
        Cc.val = out.val.data_ptr() if plan.nnz else None
    _check(lib().opsp_spgemm_numeric(plan.handle, byref(Ac), byref(Bc), byref(Cc), s),
           "opsp_spgemm_numeric")
    if out is not None:
        return out
    return _adopt(Cc, s, A.rpt.device)


# Bytes of the fixed device scratch behind spgemm_numeric_noalloc.
NOALLOC_SCRATCH_BYTES = 64 << 20
ERR_SCRATCH = 8


def spgemm_numeric_noalloc(plan: Plan, A: DeviceCSR, B: DeviceCSR, out: DeviceCSR,
                           stream=None) -> DeviceCSR:
    """Numeric phase into caller buffers ``out`` (rpt int64[rows+1], col
    int32[nnz], val float64[nnz]) through ``opsp_spgemm_numeric_noalloc``:
    no device allocation inside the call; the long-row bin works in the
    library's fixed per-GPU scratch (concurrent calls on one GPU race)."""
    s = _stream_handle(stream)
    Ac, Bc = A._c(), B._c()
    assert out.rpt.numel() == plan.rows + 1 and out.col.numel() == plan.nnz == out.val.numel()
    Cc = opsp_csr()
    Cc.rpt = out.rpt.data_ptr()
    Cc.col = out.col.data_ptr() if plan.nnz else None
    Cc.val = out.val.data_ptr() if plan.nnz else None
    _check(lib().opsp_spgemm_numeric_noalloc(plan.handle, byref(Ac), byref(Bc), byref(Cc), s),
           "opsp_spgemm_numeric_noalloc")
    return out


# ---------------------------------------------------------------------------
# Batched products
# ---------------------------------------------------------------------------

class Batch:
    """Many independent products C_p = A_p B_p as one block-diagonal product
    (``opsp_batch_*``).  ``execute()`` returns views into storage the batch
    owns; they stay valid until the next ``execute`` or until every view and
    the batch object are gone."""

    def __init__(self, As, Bs, config: Optional[Config] = None, stream=None):
        assert len(As) == len(Bs) and len(As) > 0
        self.As, self.Bs = list(As), list(Bs)      # keep the inputs alive
        self.count = len(As)
        self._a = (opsp_csr * self.count)(*[a._c() for a in As])
        self._b = (opsp_csr * self.count)(*[b._c() for b in Bs])
        self._s = _stream_handle(stream)
        h = c_void_p()
        _check(lib().opsp_batch_create(self.count, self._a, self._b,
                                       byref(config) if config is not None else None,
                                       byref(h), self._s), "opsp_batch_create")
        self.handle = h.value
        self.device = As[0].rpt.device

    def execute(self, stats: Optional[Stats] = None, stream=None):
        s = self._s if stream is None else _stream_handle(stream)
        C = (opsp_csr * self.count)()
        _check(lib().opsp_batch_execute(self.handle, C, byref(stats) if stats is not None else None,
                                        s), "opsp_batch_execute")
        torch = _torch()
        res = []
        for c in C:
            rpt = _wrap(c.rpt, c.rows + 1, torch.int64, self, self.device)
            lo = int(rpt[0].item()) if rpt.numel() else 0
            res.append(_BatchView(c.rows, c.cols, rpt, lo, c.nnz, c.col, c.val, self))
        return res

    def raw_execute(self, stream_handle, C=None):
        """Lowest-overhead execution (benchmark): fills a ctypes array."""
        if C is None:
            C = (opsp_csr * self.count)()
        _check(lib().opsp_batch_execute(self.handle, C, None, stream_handle), "opsp_batch_execute")
        return C

    def __del__(self):
        if getattr(self, "handle", None) and _lib is not None:
            _lib.opsp_batch_destroy(self.handle)
            self.handle = None


class _BatchView:
    """One C_p of a batch: row pointer with absolute offsets into the shared
    col/val arrays."""

    def __init__(self, rows, cols, rpt, lo, nnz, colp, valp, owner):
        self.rows, self.cols, self.rpt, self.lo, self.nnz = rows, cols, rpt, lo, nnz
        self._colp, self._valp, self._owner = colp, valp, owner

    def to_host(self):
        torch = _torch()
        rpt = self.rpt.cpu().numpy()
        n = int(self.nnz)
        if n == 0:
            return rpt - rpt[0], np.zeros(0, np.int32), np.zeros(0, np.float64)
        col = _wrap(self._colp + 4 * self.lo, n, torch.int32, self._owner, self._owner.device)
        val = _wrap(self._valp + 8 * self.lo, n, torch.float64, self._owner, self._owner.device)
        return rpt - rpt[0], col.cpu().numpy(), val.cpu().numpy()


# ---------------------------------------------------------------------------
# Row-size predictor and the one-phase product
# ---------------------------------------------------------------------------

def _ptr(t) -> Optional[int]:
    return t.data_ptr() if t is not None else None


def row_features(A: DeviceCSR, B: DeviceCSR, stream=None):
    """(a_len int32, n_prod int64, b_max int32) per row of A*B, on the device."""
    torch = _torch()
    dev = A.rpt.device
    al = torch.empty(A.rows, dtype=torch.int32, device=dev)
    npd = torch.empty(A.rows, dtype=torch.int64, device=dev)
    bm = torch.empty(A.rows, dtype=torch.int32, device=dev)
    Ac, Bc = A._c(), B._c()
    _check(lib().opsp_row_features(byref(Ac), byref(Bc), _ptr(al), _ptr(npd), _ptr(bm),
                                   _stream_handle(stream)), "opsp_row_features")
    return al, npd, bm


def mlp_features(A: DeviceCSR, B: DeviceCSR, stream=None):
    """Network inputs log2(1 + (a_len, n_prod, b_max)), float32 [rows, 3]."""
    torch = _torch()
    X = torch.empty((A.rows, 3), dtype=torch.float32, device=A.rpt.device)
    Ac, Bc = A._c(), B._c()
    _check(lib().opsp_mlp_features(byref(Ac), byref(Bc), _ptr(X), _stream_handle(stream)),
           "opsp_mlp_features")
    return X


def _params_tensor(params):
    torch = _torch()
    assert params.dtype == torch.int16 and params.numel() == MLP_NPARAM and params.is_contiguous()
    return params


def mlp_forward(params, X, stream=None):
    """y = network(X) for float32 X [n, 3] (params: int16 tensor of bf16 bits)."""
    torch = _torch()
    params = _params_tensor(params)
    X = X.contiguous()
    n = X.shape[0]
    y = torch.empty(n, dtype=torch.float32, device=X.device)
    _check(lib().opsp_mlp_forward(_ptr(params), _ptr(X), n, _ptr(y), _stream_handle(stream)),
           "opsp_mlp_forward")
    return y


def mlp_grad(params, X, target, tau: float = 0.0, stream=None):
    """(gradient float32[MLP_NPARAM], loss float32[1]) of the mean squared error
    (tau = 0) or of the mean pinball loss of level tau."""
    torch = _torch()
    params = _params_tensor(params)
    X, target = X.contiguous(), target.contiguous()
    g = torch.empty(MLP_NPARAM, dtype=torch.float32, device=X.device)
    loss = torch.empty(1, dtype=torch.float32, device=X.device)
    _check(lib().opsp_mlp_grad(_ptr(params), _ptr(X), _ptr(target), X.shape[0], float(tau), _ptr(g),
                               _ptr(loss), _stream_handle(stream)), "opsp_mlp_grad")
    return g, loss


def mlp_adam(master, m, v, grad, step: int, params, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8,
             stream=None):
    """One Adam step in place on (master, m, v); writes the bf16 copy into params."""
    _check(lib().opsp_mlp_adam(_ptr(master), _ptr(m), _ptr(v), _ptr(grad), int(step), lr, beta1,
                               beta2, eps, _ptr(_params_tensor(params)), _stream_handle(stream)),
           "opsp_mlp_adam")


class Predictor:
    """Capacity source of the one-phase product: the network (bf16 parameters
    on the device) or one of the reference rules (PRED_UPPER, PRED_RATIO)."""

    def __init__(self, kind: int = PRED_MLP, params=None, margin: float = 0.0, ratio: float = 1.0,
                 cap_scale: float = 0.0, calib_rows: int = 0):
        self.kind, self.params = kind, params
        self.margin, self.ratio, self.cap_scale = float(margin), float(ratio), float(cap_scale)
        self.calib_rows = int(calib_rows)

    @classmethod
    def load(cls, path: Optional[str] = None, device="cuda", margin: Optional[float] = None,
             calib_rows: int = 0):
        """The trained network stored by the training driver (JSON with the
        bf16 bit patterns in the packed order)."""
        import json
        torch = _torch()
        with open(path or DEFAULT_WEIGHTS) as f:
            d = json.load(f)
        bits = np.asarray(d["params_bf16"], np.uint16)
        assert bits.size == MLP_NPARAM
        t = torch.from_numpy(bits.view(np.int16).copy()).to(device)
        return cls(PRED_MLP, t, d.get("margin", 0.0) if margin is None else margin,
                   calib_rows=calib_rows)

    def struct(self, pred_out=None, cap_out=None) -> opsp_predictor:
        p = opsp_predictor()
        p.version = PREDICTOR_VERSION
        p.kind = self.kind
        p.params = _ptr(self.params) if self.params is not None else None
        p.margin, p.ratio, p.cap_scale = self.margin, self.ratio, self.cap_scale
        p.pred_out, p.cap_out = _ptr(pred_out), _ptr(cap_out)
        p.calib_rows = self.calib_rows
        return p


def spgemm_learned(A: DeviceCSR, B: DeviceCSR, predictor: Predictor,
                   config: Optional[Config] = None, stats: Optional[Stats] = None, stream=None,
                   pred_out=None, cap_out=None) -> DeviceCSR:
    """C = A*B by the one-phase method with predicted row capacities."""
    s = _stream_handle(stream)
    Ac, Bc, Cc = A._c(), B._c(), opsp_csr()
    ps = predictor.struct(pred_out, cap_out)
    code = lib().opsp_spgemm_learned(byref(Ac), byref(Bc), byref(Cc), byref(ps),
                                     byref(config) if config is not None else None,
                                     byref(stats) if stats is not None else None, s)
    _check(code, "opsp_spgemm_learned")
    return _adopt(Cc, s, A.rpt.device)
