"""Moment and cumulant tensors on MI355X (gfx950).

Thin Python binding over the C ABI of ``libcumulants.so`` (declared in
``include/cumulants.h``): argument marshalling only.  Every step of the
computation -- centring, the block moment contraction, the chunk reduction
and the cumulant recursion, unfolding -- runs in the library's HIP kernels.
Torch is used for device memory and streams.  There is no CPU fallback: if
the library is missing, importing this package raises.

Method: Domino, Gawron, Pawela, "Efficient computation of higher order
cumulant tensors" (block storage of Section 2.1, moments by Alg. 1-3,
cumulants by the recursion of Section 3.2 / Alg. 4-5).
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# CUM_LIBRARY names another build of the same library (the host-sanitizer
# build, for instance)
LIB_PATH = os.environ.get("CUM_LIBRARY") or os.path.join(_HERE, "libcumulants.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with `python paper_1701_05420_amd/build.py` "
                      "(or __graft_entry__.build()); there is no fallback implementation")

_lib = ctypes.CDLL(LIB_PATH)

PRECS = {"f64": 0, "f32": 1, "bf16x2": 2, "bf16x3": 3, "f16x2": 4}
MAX_ORDER = 10

EXPORTS = [
    "cum_layout_query", "cum_workspace_size", "cum_center", "cum_moment_blocks", "cum_cumulants",
    "cum_cumulants_noalloc", "cum_unfold",
    "cum_stored_offset", "cum_batch_create", "cum_batch_run", "cum_batch_timestamps", "cum_batch_destroy",
    "cum_plan_check", "cum_timing_enable", "cum_timing_read", "cum_autotune", "cum_set_tuning", "cum_get_tuning", "cum_get_plan_info",
    "cum_batch_autotune", "cum_stream_create", "cum_stream_update", "cum_stream_cumulants", "cum_stream_cumulants_moebius",
    "cum_stream_count",
    "cum_stream_reset", "cum_stream_destroy", "cum_status_str", "cum_last_error",
]
SHAPES = {"32x32": 0, "32x64": 2}


class PlanInfo(ctypes.Structure):
    _fields_ = [("nchunks", ctypes.c_int64), ("work_items", ctypes.c_int64), ("tiles", ctypes.c_int64),
                ("partial_entries", ctypes.c_int64), ("stored_entries", ctypes.c_int64)]


class Tuning(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("target_items", ctypes.c_int32), ("inner_b", ctypes.c_int32),
                ("ms", ctypes.c_float)]
KINDS = ["center", "moment", "reduce", "unfold", "batch"]


class Layout(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("d", ctypes.c_int32), ("b", ctypes.c_int32), ("nbar", ctypes.c_int32),
                ("b_last", ctypes.c_int32), ("nblocks", ctypes.c_int64), ("block_elems", ctypes.c_int64),
                ("elems", ctypes.c_int64)]


_I, _I64, _VP, _SZ = ctypes.c_int, ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
_lib.cum_layout_query.argtypes = [_I, _I, _I, ctypes.POINTER(Layout)]
_lib.cum_workspace_size.argtypes = [_I64, _I, _I, _I, _I, ctypes.POINTER(_SZ)]
_lib.cum_center.argtypes = [_VP, _I64, _I, _I64, _I, _VP, _VP, _VP, _SZ, _VP]
_lib.cum_moment_blocks.argtypes = [_VP, _I, _I64, _I, _I, _I, _VP, _VP, _SZ, _VP]
_lib.cum_cumulants.argtypes = [_VP, _I64, _I, _I64, _I, _I, _I, _VP, ctypes.POINTER(_VP), _VP, _SZ, _VP]
_lib.cum_cumulants_noalloc.argtypes = [_VP, _I64, _I, _I64, _I, _I, _I, _VP, ctypes.POINTER(_VP), _VP]
_lib.cum_unfold.argtypes = [_VP, _I, _I, _I, _VP, _VP]
_lib.cum_stored_offset.argtypes = [_I, _I, _I, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(_I64)]
_lib.cum_batch_create.argtypes = [_I, ctypes.POINTER(_I64), _I, _I, _I, _I, ctypes.POINTER(_VP)]
_lib.cum_batch_run.argtypes = [_VP, ctypes.POINTER(_VP), ctypes.POINTER(_VP), ctypes.POINTER(_VP), _VP]
_lib.cum_batch_timestamps.argtypes = [_VP, ctypes.POINTER(ctypes.c_uint64), ctypes.POINTER(ctypes.c_uint64),
                                      ctypes.POINTER(ctypes.c_double)]
_lib.cum_batch_destroy.argtypes = [_VP]
_lib.cum_plan_check.argtypes = [_I, _I, _I]
_lib.cum_timing_enable.argtypes = [_I]
_lib.cum_autotune.argtypes = [_VP, _I64, _I, _I64, _I, _I, _I, _VP, ctypes.POINTER(Tuning)]
_lib.cum_set_tuning.argtypes = [_I64, _I, _I, _I, _I, ctypes.POINTER(Tuning)]
_lib.cum_get_tuning.argtypes = [_I64, _I, _I, _I, _I, ctypes.POINTER(Tuning)]
_lib.cum_get_plan_info.argtypes = [_I64, _I, _I, _I, _I, ctypes.POINTER(PlanInfo)]
_lib.cum_batch_autotune.argtypes = [_VP, ctypes.POINTER(_VP), ctypes.POINTER(Tuning)]
_lib.cum_stream_create.argtypes = [_I, _I, _I, _I, _VP, ctypes.POINTER(_VP)]
_lib.cum_stream_update.argtypes = [_VP, _VP, _I64, _I64, _I, _VP]
_lib.cum_stream_cumulants.argtypes = [_VP, _VP, ctypes.POINTER(_VP), _VP]
_lib.cum_stream_cumulants_moebius.argtypes = [_VP, _VP, ctypes.POINTER(_VP), _VP]
_lib.cum_stream_count.argtypes = [_VP, ctypes.POINTER(_I64)]
_lib.cum_stream_reset.argtypes = [_VP, _VP]
_lib.cum_stream_destroy.argtypes = [_VP]
_lib.cum_timing_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]
_lib.cum_status_str.argtypes = [_I]
_lib.cum_status_str.restype = ctypes.c_char_p
_lib.cum_last_error.restype = ctypes.c_char_p
for _f in EXPORTS:
    if _f not in ("cum_status_str", "cum_last_error"):
        getattr(_lib, _f).restype = _I


class CumulantError(RuntimeError):
    def __init__(self, status: int):
        self.status = status
        msg = _lib.cum_status_str(status).decode()
        detail = _lib.cum_last_error().decode()
        super().__init__(f"{msg}: {detail}" if detail else msg)


def _check(st: int) -> None:
    if st != 0:
        raise CumulantError(st)


def _prec(prec) -> int:
    if isinstance(prec, int):
        return prec
    return PRECS[prec]


# ---------------------------------------------------------------- host-only helpers
def layout(n: int, d: int, b: int) -> dict:
    L = Layout()
    _check(_lib.cum_layout_query(n, d, b, ctypes.byref(L)))
    return {f: getattr(L, f) for f, _ in Layout._fields_}


def workspace_size(t: int, n: int, d_max: int, b: int, prec="f64") -> int:
    out = _SZ()
    _check(_lib.cum_workspace_size(t, n, d_max, b, _prec(prec), ctypes.byref(out)))
    return int(out.value)


def stored_offset(n: int, d: int, b: int, idx) -> int:
    arr = (ctypes.c_int32 * d)(*[int(i) for i in idx])
    out = _I64()
    _check(_lib.cum_stored_offset(n, d, b, arr, ctypes.byref(out)))
    return int(out.value)


def plan_check(n: int, d: int, b: int) -> None:
    _check(_lib.cum_plan_check(n, d, b))


def autotune(X, d_max: int, b: int, prec="f32", stream=None) -> dict:
    """Time the launch configurations on X and keep the fastest for this shape."""
    torch = _torch()
    _dev_check(X, torch.float64, "X")
    t, n = X.shape
    out = Tuning()
    _check(_lib.cum_autotune(X.data_ptr(), t, n, X.stride(0), d_max, b, _prec(prec), _stream(stream),
                             ctypes.byref(out)))
    return {"shape": out.shape, "target_items": out.target_items, "inner_b": out.inner_b, "ms": out.ms}


def get_tuning(t: int, n: int, d_max: int, b: int, prec) -> dict:
    """The configuration cumulants() uses for this shape (tuned, else defaults)."""
    out = Tuning()
    _check(_lib.cum_get_tuning(t, n, d_max, b, _prec(prec), ctypes.byref(out)))
    return {"shape": out.shape, "target_items": out.target_items, "inner_b": out.inner_b}


def plan_info(t: int, n: int, d_max: int, b: int, prec) -> dict:
    """How cumulants() splits the work for this shape in its current configuration."""
    out = PlanInfo()
    _check(_lib.cum_get_plan_info(t, n, d_max, b, _prec(prec), ctypes.byref(out)))
    return {f: getattr(out, f) for f, _ in PlanInfo._fields_}


def set_tuning(t: int, n: int, d_max: int, b: int, prec, shape=None, target_items=4096, inner_b=1) -> None:
    """Fix the configuration for a shape (shape=None forgets it)."""
    if shape is None:
        _check(_lib.cum_set_tuning(t, n, d_max, b, _prec(prec), None))
        return
    tune = Tuning(SHAPES[shape] if isinstance(shape, str) else int(shape), int(target_items), int(inner_b), 0.0)
    _check(_lib.cum_set_tuning(t, n, d_max, b, _prec(prec), ctypes.byref(tune)))


def timing_enable(on: bool = True) -> None:
    """Bracket every kernel launch of this thread's calls with HIP events."""
    _check(_lib.cum_timing_enable(1 if on else 0))


def timing_read() -> dict:
    """{kind: (milliseconds, launches)} since the last read (synchronises)."""
    ms = (ctypes.c_double * len(KINDS))()
    cnt = (_I64 * len(KINDS))()
    _check(_lib.cum_timing_read(ms, cnt))
    return {k: (float(ms[i]), int(cnt[i])) for i, k in enumerate(KINDS)}


# ---------------------------------------------------------------- device entry points
def _torch():
    import torch

    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_check(x, dtype, name):
    torch = _torch()
    if not isinstance(x, torch.Tensor) or not x.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {x.dtype}")


def _workspace(nbytes, ws, device):
    torch = _torch()
    if ws is not None:
        return ws  # the library checks its size
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _on(stream):
    """Allocation context of a call: tensors the call allocates (its outputs
    and a temporary workspace) belong to the stream its kernels run on, so
    torch's caching allocator does not hand them to other work before that
    stream is done with them."""
    import contextlib

    if stream is None:
        return contextlib.nullcontext()
    return _torch().cuda.stream(stream)


def center(X, prec="f64", ws=None, stream=None):
    """Column means (FP64) and centred data (FP64 for 'f64', FP32 otherwise)."""
    torch = _torch()
    _dev_check(X, torch.float64, "X")
    t, n = X.shape
    if X.stride(1) != 1:
        raise ValueError("X must have unit column stride")
    p = _prec(prec)
    with _on(stream):
        mean = torch.empty(n, dtype=torch.float64, device=X.device)
        Xc = torch.empty((t, n), dtype=torch.float64 if p == 0 else torch.float32, device=X.device)
        ws = _workspace(workspace_size(t, n, 2, 1, p), ws, X.device)
    _check(_lib.cum_center(X.data_ptr(), t, n, X.stride(0), p, mean.data_ptr(), Xc.data_ptr(), ws.data_ptr(),
                           ws.numel() * ws.element_size(), _stream(stream)))
    return mean, Xc


def moment_blocks(Xc, d: int, b: int, prec=None, ws=None, stream=None):
    """Order-d moment tensor of the data as given (no centring), block storage."""
    torch = _torch()
    if prec is None:
        prec = "f64" if Xc.dtype == torch.float64 else "f32"
    p = _prec(prec)
    _dev_check(Xc, torch.float64 if p == 0 else torch.float32, "Xc")
    if not Xc.is_contiguous():
        raise ValueError("Xc must be contiguous (t x n, leading dimension n)")
    t, n = Xc.shape
    L = layout(n, d, b)
    with _on(stream):
        M = torch.empty(L["elems"], dtype=torch.float64, device=Xc.device)
        ws = _workspace(workspace_size(t, n, d, b, p), ws, Xc.device)
    _check(_lib.cum_moment_blocks(Xc.data_ptr(), p, t, n, d, b, M.data_ptr(), ws.data_ptr(),
                                  ws.numel() * ws.element_size(), _stream(stream)))
    return M


def cumulants(X, d_max: int, b: int, prec="f64", ws=None, out=None, stream=None):
    """Mean and cumulant tensors {d: c_d in block storage} for d = 2..d_max."""
    torch = _torch()
    _dev_check(X, torch.float64, "X")
    if X.stride(1) != 1:
        raise ValueError("X must have unit column stride")
    t, n = X.shape
    p = _prec(prec)
    with _on(stream):
        mean = torch.empty(n, dtype=torch.float64, device=X.device)
        if out is None:
            out = {d: torch.empty(layout(n, d, b)["elems"], dtype=torch.float64, device=X.device)
                   for d in range(2, d_max + 1)}
        ws = _workspace(workspace_size(t, n, d_max, b, p), ws, X.device)
    ptrs = (_VP * (d_max - 1))(*[out[d].data_ptr() for d in range(2, d_max + 1)])
    _check(_lib.cum_cumulants(X.data_ptr(), t, n, X.stride(0), d_max, b, p, mean.data_ptr(), ptrs,
                              ws.data_ptr(), ws.numel() * ws.element_size(), _stream(stream)))
    return mean, out


NOALLOC_SCRATCH_BYTES = 256 << 20


def cumulants_noalloc(X, d_max: int, b: int, prec, mean, out, stream=None):
    """cumulants() through the library's allocation-free entry point: the
    caller passes the mean (n FP64) and the outputs {d: block storage}; the
    library takes its workspace from its fixed scratch.  The configuration
    must have been run once by cumulants() before."""
    torch = _torch()
    _dev_check(X, torch.float64, "X")
    if X.stride(1) != 1:
        raise ValueError("X must have unit column stride")
    t, n = X.shape
    ptrs = (_VP * (d_max - 1))(*[out[d].data_ptr() for d in range(2, d_max + 1)])
    _check(_lib.cum_cumulants_noalloc(X.data_ptr(), t, n, X.stride(0), d_max, b, _prec(prec),
                                      mean.data_ptr() if mean is not None else None, ptrs, _stream(stream)))
    return mean, out


def unfold(blocks, n: int, d: int, b: int, stream=None):
    """Dense n^d tensor from block storage (canonical stored copy per entry)."""
    torch = _torch()
    _dev_check(blocks, torch.float64, "blocks")
    with _on(stream):
        dense = torch.empty((n,) * d, dtype=torch.float64, device=blocks.device)
    _check(_lib.cum_unfold(blocks.data_ptr(), n, d, b, dense.data_ptr(), _stream(stream)))
    return dense


class Batch:
    """Many datasets (same n, uneven t_i) in one graph-captured run."""

    def __init__(self, t_list, n: int, d_max: int, b: int, prec="f32"):
        self.t = [int(x) for x in t_list]
        self.n, self.d_max, self.b, self.prec = n, d_max, b, _prec(prec)
        arr = (_I64 * len(self.t))(*self.t)
        h = _VP()
        _check(_lib.cum_batch_create(len(self.t), arr, n, d_max, b, self.prec, ctypes.byref(h)))
        self._h = h

    def run(self, X_list, out=None, means=None, stream=None):
        torch = _torch()
        ns = len(self.t)
        if len(X_list) != ns:
            raise ValueError("one array per dataset")
        for s, X in enumerate(X_list):
            _dev_check(X, torch.float64, "X")
            if tuple(X.shape) != (self.t[s], self.n) or not X.is_contiguous():
                raise ValueError(f"dataset {s} must be a contiguous {self.t[s]} x {self.n} tensor")
        with _on(stream):
            if out is None:
                out = [{d: torch.empty(layout(self.n, d, self.b)["elems"], dtype=torch.float64,
                                       device=X_list[0].device)
                        for d in range(2, self.d_max + 1)} for _ in range(ns)]
            if means is None:
                means = [torch.empty(self.n, dtype=torch.float64, device=X_list[0].device) for _ in range(ns)]
        xs = (_VP * ns)(*[X.data_ptr() for X in X_list])
        ks = (_VP * (ns * (self.d_max - 1)))(*[out[s][d].data_ptr() for s in range(ns)
                                                 for d in range(2, self.d_max + 1)])
        ms = (_VP * ns)(*[m.data_ptr() for m in means])
        _check(_lib.cum_batch_run(self._h, xs, ks, ms, _stream(stream)))
        self._keep = (X_list, out, means)
        return means, out

    def autotune(self, X_list):
        """Time the launch configurations on these datasets; keep the fastest."""
        xs = (_VP * len(X_list))(*[X.data_ptr() for X in X_list])
        out = Tuning()
        _check(_lib.cum_batch_autotune(self._h, xs, ctypes.byref(out)))
        return {"shape": out.shape, "target_items": out.target_items, "inner_b": out.inner_b, "ms": out.ms}

    def timestamps(self):
        ns = len(self.t)
        start = ctypes.c_uint64()
        ticks = (ctypes.c_uint64 * ns)()
        hz = ctypes.c_double()
        _check(_lib.cum_batch_timestamps(self._h, ctypes.byref(start), ticks, ctypes.byref(hz)))
        return int(start.value), [int(x) for x in ticks], float(hz.value)

    def close(self):
        if getattr(self, "_h", None):
            _lib.cum_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Stream:
    """A sliding window of samples: add and remove batches, read the window's
    cumulants at any time (sums about a fixed shift, FP64)."""

    def __init__(self, n: int, d_max: int, b: int, prec="f32", shift=None):
        self.n, self.d_max, self.b, self.prec = n, d_max, b, _prec(prec)
        sh = None
        if shift is not None:
            import numpy as np

            arr = np.ascontiguousarray(np.asarray(shift, dtype=np.float64))
            if arr.shape != (n,):
                raise ValueError(f"shift must hold {n} values")
            self._shift = arr
            sh = arr.ctypes.data_as(_VP)
        h = _VP()
        _check(_lib.cum_stream_create(n, d_max, b, self.prec, sh, ctypes.byref(h)))
        self._h = h

    def _update(self, X, sign, stream):
        torch = _torch()
        _dev_check(X, torch.float64, "X")
        if X.dim() != 2 or X.shape[1] != self.n or X.stride(1) != 1:
            raise ValueError(f"X must be t x {self.n} with unit column stride")
        _check(_lib.cum_stream_update(self._h, X.data_ptr(), X.shape[0], X.stride(0), sign, _stream(stream)))
        self._keep = X

    def add(self, X, stream=None):
        """Add the samples X (t x n FP64 on the device) to the window."""
        self._update(X, 1, stream)

    def remove(self, X, stream=None):
        """Remove samples X that were added before."""
        self._update(X, -1, stream)

    def count(self) -> int:
        t = _I64()
        _check(_lib.cum_stream_count(self._h, ctypes.byref(t)))
        return int(t.value)

    def cumulants(self, out=None, mean=None, stream=None, method="recursion"):
        """(mean, {d: c_d}) of the window, c_d in block storage; method
        "recursion" (centred moments, partition recursion) or "moebius" (the
        general formula on the moments about the shift)."""
        torch = _torch()
        if method not in ("recursion", "moebius"):
            raise ValueError("method is 'recursion' or 'moebius'")
        with _on(stream):
            if out is None:
                out = {d: torch.empty(layout(self.n, d, self.b)["elems"], dtype=torch.float64, device="cuda")
                       for d in range(2, self.d_max + 1)}
            if mean is None:
                mean = torch.empty(self.n, dtype=torch.float64, device="cuda")
        ks = (_VP * (self.d_max - 1))(*[out[d].data_ptr() for d in range(2, self.d_max + 1)])
        fn = _lib.cum_stream_cumulants if method == "recursion" else _lib.cum_stream_cumulants_moebius
        _check(fn(self._h, mean.data_ptr(), ks, _stream(stream)))
        return mean, out

    def reset(self, stream=None):
        _check(_lib.cum_stream_reset(self._h, _stream(stream)))

    def close(self):
        if getattr(self, "_h", None):
            _lib.cum_stream_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
