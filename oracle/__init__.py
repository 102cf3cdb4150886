"""CPU oracle for moment and cumulant tensors (TEST INFRASTRUCTURE ONLY).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The GPU library never imports, links or
calls it, and the two share no code.

Two independent implementations live here:

* ``cumoracle.c`` (loaded through ctypes): dense FP64, every entry of the full
  n^d tensors, Neumaier-compensated sample sums, the partition recursion of
  Section 3.2 (eq. cum_r) -- the oracle the GPU path is compared against;
* ``exact.py``: exact rational arithmetic on tiny integer data, by two
  different formulas (the centred recursion and the Moebius-weighted sum over
  all partitions of raw moments, eq. cumfmom of Section 5.3) -- the pins that
  the FP64 oracle is checked against.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cumoracle.c")
# ORACLE_LIBRARY names another build of the oracle (the sanitizer build)
_BUILD_PATH = os.path.join(_HERE, "liboracle.so")
_LIB_PATH = os.environ.get("ORACLE_LIBRARY") or _BUILD_PATH
_SAN_PATH = os.path.join(_HERE, "liboracle.asan.so")
_lib = None

MAXD = 10


def build(force: bool = False, sanitize: bool = False) -> str:
    """Compile the C oracle in place (gcc, OpenMP, no FP contraction); with
    sanitize, a separate build under AddressSanitizer and
    UndefinedBehaviorSanitizer."""
    path = _SAN_PATH if sanitize else _BUILD_PATH
    if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
        tmp = path + ".tmp"
        san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g"]
        subprocess.check_call(
            ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
             "-Wall", *(san if sanitize else []), "-o", tmp, _SRC])
        os.replace(tmp, path)
    return path


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp, ip, lp = ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_long)
    L, I = ctypes.c_long, ctypes.c_int
    lib.orc_center.argtypes = [dp, L, I, L, dp, dp]
    lib.orc_moment_dense.argtypes = [dp, L, I, I, dp]
    lib.orc_partitions.argtypes = [I, I, I, ip, I]
    lib.orc_cumulants_dense.argtypes = [dp, L, I, I, ctypes.POINTER(dp)]
    lib.orc_cumulant_at.argtypes = [dp, L, I, I, ip, L, dp]
    lib.orc_block_elems.argtypes = [I, I, I]
    lib.orc_block_elems.restype = L
    lib.orc_block_indices.argtypes = [I, I, I, lp, L, ip]
    lib.orc_fold.argtypes = [dp, I, I, I, dp]
    lib.orc_set_threads.argtypes = [I]
    lib.orc_max_threads.restype = I
    _lib = lib
    return lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _check(rc, what):
    if rc != 0:
        raise RuntimeError(f"oracle {what} failed with code {rc}")


def set_threads(k: int) -> None:
    _load().orc_set_threads(int(k))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def center(X: np.ndarray):
    """Column means and centred data (Def. of the centred variable, Section 1.3)."""
    lib = _load()
    X = np.ascontiguousarray(X, dtype=np.float64)
    t, n = X.shape
    mean = np.empty(n)
    Xc = np.empty((t, n))
    _check(lib.orc_center(_dp(X), t, n, n, _dp(mean), _dp(Xc)), "center")
    return mean, Xc


def moment_dense(Xc: np.ndarray, d: int) -> np.ndarray:
    """Full n^d moment tensor of the given data (Def. of the d-th moment)."""
    lib = _load()
    Xc = np.ascontiguousarray(Xc, dtype=np.float64)
    t, n = Xc.shape
    M = np.empty((n,) * d)
    _check(lib.orc_moment_dense(_dp(Xc), t, n, d, _dp(M)), "moment_dense")
    return M


def partitions(d: int, min_part: int = 2, min_parts: int = 2) -> np.ndarray:
    """Set partitions of d positions as label vectors (labels in order of
    first appearance); by default those used by the cumulant recursion."""
    lib = _load()
    cnt = lib.orc_partitions(d, min_part, min_parts, None, 0)
    if cnt < 0:
        raise ValueError("bad d")
    out = np.zeros((max(cnt, 1), d), dtype=np.int32)
    lib.orc_partitions(d, min_part, min_parts, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), cnt)
    return out[:cnt]


def cumulants_dense(X: np.ndarray, dmax: int, centred: bool = False):
    """Dense cumulant tensors {d: n^d array} for d = 2..dmax (plus the mean).

    Centres X first unless ``centred`` is set (then the mean is returned as
    None and X is taken as X~)."""
    lib = _load()
    if centred:
        mean, Xc = None, np.ascontiguousarray(X, dtype=np.float64)
    else:
        mean, Xc = center(X)
    t, n = Xc.shape
    outs = {d: np.empty((n,) * d) for d in range(2, dmax + 1)}
    arr = (ctypes.POINTER(ctypes.c_double) * (dmax - 1))(*[_dp(outs[d]) for d in range(2, dmax + 1)])
    _check(lib.orc_cumulants_dense(_dp(Xc), t, n, dmax, arr), "cumulants_dense")
    return mean, outs


def cumulant_at(Xc: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Order-d cumulant of centred data at each row of idx (count x d)."""
    lib = _load()
    Xc = np.ascontiguousarray(Xc, dtype=np.float64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    t, n = Xc.shape
    count, d = idx.shape
    out = np.empty(count)
    _check(lib.orc_cumulant_at(_dp(Xc), t, n, d, idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), count,
                               _dp(out)), "cumulant_at")
    return out


def block_elems(n: int, d: int, b: int) -> int:
    r = int(_load().orc_block_elems(n, d, b))
    if r < 0:
        raise ValueError("bad layout")
    return r


def block_indices(n: int, d: int, b: int, offsets) -> np.ndarray:
    """Multi-index stored at each block-storage offset (-1 rows for padding)."""
    lib = _load()
    offs = np.ascontiguousarray(offsets, dtype=np.int64)
    idx = np.empty((offs.size, d), dtype=np.int32)
    _check(lib.orc_block_indices(n, d, b, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_long)), offs.size,
                                 idx.ctypes.data_as(ctypes.POINTER(ctypes.c_int))), "block_indices")
    return idx


def fold(dense: np.ndarray, b: int) -> np.ndarray:
    """Dense n^d tensor read at every block-storage position (Section 2.1)."""
    lib = _load()
    dense = np.ascontiguousarray(dense, dtype=np.float64)
    d = dense.ndim
    n = dense.shape[0]
    out = np.empty(block_elems(n, d, b))
    _check(lib.orc_fold(_dp(dense), n, d, b, _dp(out)), "fold")
    return out
