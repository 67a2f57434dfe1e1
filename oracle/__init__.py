"""CPU FP64 oracle for the paper's BLAS pattern compositions.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  The GPU
library neither imports nor links it, and this package shares no code with
the GPU library.

Two independent implementations of the same definitions live here:

* ``lift_oracle.c`` (built with gcc into ``liboracle.so``): scal, asum, dot
  and gemv as the literal compositions of the paper's BLAS figure (Fig. 5),
  evaluated in binary64 with a sequential left fold for ``reduce`` -- the
  full-size numeric oracle -- BlackScholes as map(BSComputation) over
  stock prices (Section 5.2, closed-form model), and MD as a map over
  particles of a reduce over neighbour indices (Fig. 7, Lennard-Jones);
* ``patterns.py``: the paper's patterns (Tables 1 and 2) as Python functions,
  used for the rewrite-rule, derivation and low-level-expression pins.

Inputs are numpy arrays.  float32 / float16 / float64 arrays carry their own
type; bfloat16 data (which numpy lacks) is passed as its uint16 bit patterns
with ``dtype="bf16"``.  Every result is binary64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

from . import patterns  # noqa: F401  (re-exported)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lift_oracle.c")
_LIB_DEFAULT = os.path.join(_HERE, "liboracle.so")
_LIB_SAN = os.path.join(_HERE, "liboracle_san.so")
# ORACLE_LIB selects another build of the same source (the sanitizer build)
_LIB = os.environ.get("ORACLE_LIB", _LIB_DEFAULT)

F32, BF16, F16, F64 = 0, 1, 2, 3
_CODES = {"f32": F32, "bf16": BF16, "f16": F16, "f64": F64}
_NP_DT = {F32: np.float32, BF16: np.uint16, F16: np.float16, F64: np.float64}

_lock = threading.Lock()
_lib = None


def build(force: bool = True, sanitize: bool = False) -> str:
    """Compile ``liboracle.so`` with gcc (no fast-math, no FP contraction);
    with ``sanitize``, ``liboracle_san.so`` with clang's AddressSanitizer and
    UndefinedBehaviorSanitizer (the runtime the library's sanitizer build
    preloads; one process cannot hold gcc's and clang's)."""
    lib = _LIB_SAN if sanitize else _LIB_DEFAULT
    if not force and os.path.exists(lib):
        return lib
    tmp = lib + ".tmp"
    if sanitize:
        cmd = ["/opt/rocm/llvm/bin/clang", "-O1", "-g", "-std=c99", "-Wall", "-Wextra", "-fno-fast-math",
               "-ffp-contract=off", "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
               "-fno-omit-frame-pointer", "-pthread", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    else:
        cmd = ["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fno-fast-math",
               "-ffp-contract=off", "-pthread", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, lib)
    return lib


def _configure(lib):
    """Declare the C signatures on a loaded oracle library."""
    i64, dbl, i32, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_int, ctypes.c_void_p
    dp = ctypes.POINTER(ctypes.c_double)
    lib.oracle_widen.argtypes = [i64, i32, vp, dp]
    lib.oracle_scal.argtypes = [i64, dbl, i32, vp, dp]
    lib.oracle_asum.argtypes = [i64, i32, vp, dp]
    lib.oracle_dot.argtypes = [i64, i32, vp, i32, vp, dp]
    lib.oracle_dot_absmass.argtypes = [i64, i32, vp, i32, vp, dp]
    gemv_args = [i64, i64, dbl, i32, vp, i64, i32, vp, dbl, i32, vp, dp]
    lib.oracle_gemv.argtypes = gemv_args
    lib.oracle_gemv_absmass.argtypes = gemv_args
    lib.oracle_scal_par.argtypes = [i64, dbl, i32, vp, dp, i32]
    lib.oracle_asum_par.argtypes = [i64, i32, vp, dp, i32]
    lib.oracle_dot_par.argtypes = [i64, i32, vp, i32, vp, dp, i32]
    lib.oracle_blackscholes.argtypes = [i64, i32, vp, dbl, dbl, dbl, dbl, dp]
    lib.oracle_md.argtypes = [i64, vp, i64, vp, dbl, dbl, dbl, dp, dp]
    for name in ("oracle_widen", "oracle_scal", "oracle_asum", "oracle_dot",
                 "oracle_dot_absmass", "oracle_gemv", "oracle_gemv_absmass",
                 "oracle_scal_par", "oracle_asum_par", "oracle_dot_par", "oracle_blackscholes", "oracle_md"):
        getattr(lib, name).restype = ctypes.c_int
    return lib


def _load():
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=True, sanitize=_LIB == _LIB_SAN)
            _lib = _configure(ctypes.CDLL(_LIB))
    return _lib


def _code(arr: np.ndarray, dtype) -> int:
    if dtype is not None:
        code = _CODES[dtype] if isinstance(dtype, str) else int(dtype)
    elif arr.dtype == np.float32:
        code = F32
    elif arr.dtype == np.float16:
        code = F16
    elif arr.dtype == np.float64:
        code = F64
    else:
        raise TypeError(f"unsupported oracle input dtype {arr.dtype}; pass dtype='bf16' for bf16 bits")
    if arr.dtype != _NP_DT[code]:
        raise TypeError(f"array dtype {arr.dtype} does not hold code {code}")
    return code


def _flat(arr: np.ndarray) -> np.ndarray:
    if not arr.flags["C_CONTIGUOUS"]:
        raise ValueError("oracle inputs must be C-contiguous")
    return arr


def _ptr(arr: np.ndarray):
    return ctypes.c_void_p(arr.ctypes.data) if arr.size else ctypes.c_void_p(0)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed with code {rc}")


def widen(x: np.ndarray, dtype=None) -> np.ndarray:
    """Exact conversion of stored values to binary64."""
    x = _flat(x)
    code = _code(x, dtype)
    out = np.empty(x.size, dtype=np.float64)
    _check(_load().oracle_widen(x.size, code, _ptr(x), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "widen")
    return out.reshape(x.shape)


def scal(alpha: float, x: np.ndarray, dtype=None) -> np.ndarray:
    """scal(a, x) = map(mult(a), x), binary64 output."""
    x = _flat(x)
    code = _code(x, dtype)
    out = np.empty(x.size, dtype=np.float64)
    _check(_load().oracle_scal(x.size, float(alpha), code, _ptr(x),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "scal")
    return out


def asum(x: np.ndarray, dtype=None) -> float:
    """asum(x) = reduce(add, 0) o map(abs, x)."""
    x = _flat(x)
    r = ctypes.c_double()
    _check(_load().oracle_asum(x.size, _code(x, dtype), _ptr(x), ctypes.byref(r)), "asum")
    return r.value


def dot(x: np.ndarray, y: np.ndarray, dtype=None, ydtype=None) -> float:
    """dot(x, y) = reduce(add, 0) o map(mult) o zip(x, y)."""
    x, y = _flat(x), _flat(y)
    if x.size != y.size:
        raise ValueError("dot of unequal lengths")
    r = ctypes.c_double()
    _check(_load().oracle_dot(x.size, _code(x, dtype), _ptr(x), _code(y, ydtype if ydtype else dtype),
                              _ptr(y), ctypes.byref(r)), "dot")
    return r.value


def dot_absmass(x: np.ndarray, y: np.ndarray, dtype=None, ydtype=None) -> float:
    """sum |x_i y_i| -- the denominator of dot's relative error bound."""
    x, y = _flat(x), _flat(y)
    r = ctypes.c_double()
    _check(_load().oracle_dot_absmass(x.size, _code(x, dtype), _ptr(x), _code(y, ydtype if ydtype else dtype),
                                      _ptr(y), ctypes.byref(r)), "dot_absmass")
    return r.value


def _gemv(fn, alpha, A, x, beta, y, adtype, lda):
    A = _flat(A)
    if A.ndim != 2:
        raise ValueError("A must be 2-D (rows, lda) or (rows, n)")
    m = A.shape[0]
    n = x.size
    lda = A.shape[1] if lda is None else lda
    if A.shape[1] < n or lda != A.shape[1]:
        raise ValueError("A's row length must equal lda >= n")
    x = _flat(x)
    y = _flat(y)
    if y.size != m:
        raise ValueError("y must have one entry per row of A")
    out = np.empty(m, dtype=np.float64)
    rc = fn(m, n, float(alpha), _code(A, adtype), _ptr(A), lda, _code(x, None), _ptr(x),
            float(beta), _code(y, None), _ptr(y), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    _check(rc, "gemv")
    return out


def gemv(alpha: float, A: np.ndarray, x: np.ndarray, beta: float, y: np.ndarray,
         adtype=None, lda=None) -> np.ndarray:
    """y' = alpha * A x + beta * y (row-major A, leading dimension lda).

    ``A`` is a 2-D array of shape (m, lda) whose first n = len(x) columns are
    the matrix.  beta == 0 leaves y unread (BLAS convention).
    """
    return _gemv(_load().oracle_gemv, alpha, A, x, beta, y, adtype, lda)


def gemv_absmass(alpha: float, A: np.ndarray, x: np.ndarray, beta: float, y: np.ndarray,
                 adtype=None, lda=None) -> np.ndarray:
    """|alpha| sum_j |A_ij x_j| + |beta y_i| -- gemv's per-row error denominator."""
    return _gemv(_load().oracle_gemv_absmass, alpha, A, x, beta, y, adtype, lda)


# ---------------------------------------------------------------- split-join
def host_threads() -> int:
    """Threads for the split-join form: the cores this process may use,
    capped by OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    cap = os.environ.get("OMP_NUM_THREADS")
    if cap and cap.isdigit() and int(cap) > 0:
        n = min(n, int(cap))
    return max(1, min(n, 256))


def scal_par(alpha: float, x: np.ndarray, threads: int, dtype=None) -> np.ndarray:
    """scal as a map over `threads` chunks, each chunk on its own thread."""
    x = _flat(x)
    out = np.empty(x.size, dtype=np.float64)
    _check(_load().oracle_scal_par(x.size, float(alpha), _code(x, dtype), _ptr(x),
                                   out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), int(threads)), "scal_par")
    return out


def asum_par(x: np.ndarray, threads: int, dtype=None) -> float:
    """reduce(add, 0) o join o map(asum) o split: chunk sums on threads, then
    their sum in chunk order (rule 3d)."""
    x = _flat(x)
    r = ctypes.c_double()
    _check(_load().oracle_asum_par(x.size, _code(x, dtype), _ptr(x), ctypes.byref(r), int(threads)), "asum_par")
    return r.value


def dot_par(x: np.ndarray, y: np.ndarray, threads: int, dtype=None, ydtype=None) -> float:
    """dot in the same split-join form as asum_par."""
    x, y = _flat(x), _flat(y)
    if x.size != y.size:
        raise ValueError("dot of unequal lengths")
    r = ctypes.c_double()
    _check(_load().oracle_dot_par(x.size, _code(x, dtype), _ptr(x), _code(y, ydtype if ydtype else dtype),
                                  _ptr(y), ctypes.byref(r), int(threads)), "dot_par")
    return r.value


# ---------------------------------------------------------------- BlackScholes
def blackscholes(s: np.ndarray, strike: float, rate: float, volatility: float, years: float,
                 dtype=None) -> np.ndarray:
    """map(BSComputation) over stock prices: an (n, 2) array of {call, put}."""
    s = _flat(s)
    out = np.empty((s.size, 2), dtype=np.float64)
    _check(_load().oracle_blackscholes(s.size, _code(s, dtype), _ptr(s), float(strike), float(rate),
                                       float(volatility), float(years),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))), "blackscholes")
    return out


# ---------------------------------------------------------------- MD
def md(pos: np.ndarray, nbr: np.ndarray, cutoff: float, epsilon: float, sigma: float, with_mass: bool = False):
    """Forces on n particles: pos (n, 4) float32 (x, y, z, unused), nbr
    (n, k) int32 neighbour indices (outside [0, n) = empty slot).  Returns
    (n, 3) binary64 forces, and with ``with_mass`` also sum |terms| per
    component (the scale of rounding error)."""
    pos = _flat(pos)
    nbr = _flat(nbr)
    if pos.dtype != np.float32 or pos.ndim != 2 or pos.shape[1] != 4:
        raise TypeError("pos must be (n, 4) float32")
    if nbr.dtype != np.int32 or nbr.ndim != 2 or nbr.shape[0] != pos.shape[0]:
        raise TypeError("nbr must be (n, k) int32")
    n, k = pos.shape[0], nbr.shape[1]
    f = np.empty((n, 3), dtype=np.float64)
    m = np.empty((n, 3), dtype=np.float64) if with_mass else None
    dp = ctypes.POINTER(ctypes.c_double)
    _check(_load().oracle_md(n, _ptr(pos), k, _ptr(nbr), float(cutoff), float(epsilon), float(sigma),
                             f.ctypes.data_as(dp), m.ctypes.data_as(dp) if with_mass else None), "md")
    return (f, m) if with_mass else f
