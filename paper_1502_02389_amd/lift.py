"""ctypes binding of ``liblift.so`` -- argument marshalling only.

Two layers:

* ``lift_scal``, ``lift_asum``, ... : the C entry points under their own
  names, taking integers (sizes), floats and raw device addresses, returning
  the ``lift_status`` code.  Declared in ``include/lift.h``.
* ``scal``, ``asum``, ``dot``, ``gemv`` : tensor conveniences that check
  device / dtype / contiguity, allocate outputs and the per-stream workspace
  with PyTorch, and call the entry points above on the current HIP stream.
  Every step of the computation runs in the library's kernels; there is no
  fallback: without the built library these raise.
"""
from __future__ import annotations

import ctypes
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
# LIFT_LIB selects another build of the library (the CPU sanitizer build)
LIB_PATH = os.environ.get("LIFT_LIB", os.path.join(HERE, "liblift.so"))

LIFT_OK, LIFT_EINVAL, LIFT_EWORKSPACE, LIFT_EHIP, LIFT_EUNSUPPORTED = 0, -1, -2, -3, -4
LIFT_F32, LIFT_BF16, LIFT_F16, LIFT_F64 = 0, 1, 2, 3
LIFT_ACC_F32, LIFT_ACC_F32_COMP, LIFT_ACC_F32_F64COMBINE = 0, 1, 2
LIFT_INTERLEAVE_DEFAULT, LIFT_INTERLEAVE_STRIDE, LIFT_INTERLEAVE_CHUNK = 0, 1, 2
LIFT_LANES_TREE, LIFT_LANES_SEQ, LIFT_LANES_RUNS_TREE, LIFT_LANES_RUNS_SEQ = 0, 1, 2, 3

ACC = {"f32": LIFT_ACC_F32, "comp": LIFT_ACC_F32_COMP, "f64combine": LIFT_ACC_F32_F64COMBINE}


class LiftError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = _lib().lift_status_string(status).decode() if _LIB is not None else str(status)
        extra = ""
        if status == LIFT_EHIP:
            extra = f" (hipError {_lib().lift_last_hip_error()})"
        super().__init__(f"{what}: {msg}{extra} [{status}]")


class lift_knobs(ctypes.Structure):
    _fields_ = [
        ("block", ctypes.c_int32),
        ("vec_bytes", ctypes.c_int32),
        ("unroll", ctypes.c_int32),
        ("rows_per_wave", ctypes.c_int32),
        ("split", ctypes.c_int64),
        ("wg_per_cu", ctypes.c_int32),
        ("row_split", ctypes.c_int32),
        ("lanes_per_item", ctypes.c_int32),
        ("interleave", ctypes.c_int32),
        ("lane_form", ctypes.c_int32),
    ]


def knobs(block=0, vec_bytes=0, unroll=0, rows_per_wave=0, split=0, wg_per_cu=0, row_split=0, lanes_per_item=0,
          interleave=0, lane_form=0):
    """A lift_knobs struct; every field 0 selects the library's default for it
    (interleave: LIFT_INTERLEAVE_STRIDE / LIFT_INTERLEAVE_CHUNK, 0 = default;
    lane_form: a LIFT_LANES_* value, 0 = reorder-stride lanes and a tree).
    Field meanings and allowed values are those of lift_knobs in lift.h."""
    return lift_knobs(block, vec_bytes, unroll, rows_per_wave, split, wg_per_cu, row_split, lanes_per_item,
                      interleave, lane_form)


LIFT_KIND_ASUM, LIFT_KIND_DOT, LIFT_KIND_GEMV = 0, 1, 2


class lift_problem(ctypes.Structure):
    _fields_ = [
        ("kind", ctypes.c_int32),
        ("reserved", ctypes.c_int32),
        ("m", ctypes.c_int64),
        ("n", ctypes.c_int64),
        ("lda", ctypes.c_int64),
        ("a", ctypes.c_void_p),
        ("b", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("alpha", ctypes.c_float),
        ("beta", ctypes.c_float),
    ]


_LIB = None
_LOCK = threading.Lock()

_i64, _f32, _vp, _sz, _i32 = ctypes.c_int64, ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int
_kp = ctypes.POINTER(lift_knobs)

SIGNATURES = {
    "lift_scal": (_i32, [_i64, _f32, _vp, _vp, _vp]),
    "lift_asum": (_i32, [_i64, _vp, _vp, _vp, _sz, _vp]),
    "lift_dot": (_i32, [_i64, _vp, _vp, _vp, _vp, _sz, _vp]),
    "lift_gemv": (_i32, [_i64, _i64, _f32, _vp, _i64, _vp, _f32, _vp, _vp]),
    "lift_workspace_bytes": (_sz, []),
    "lift_max_workgroups": (ctypes.c_int32, []),
    "lift_scal_ex": (_i32, [_i64, _f32, _vp, _vp, _kp, _vp]),
    "lift_asum_ex": (_i32, [_i64, _i32, _vp, _i32, _i32, _vp, _vp, _sz, _kp, _vp]),
    "lift_dot_ex": (_i32, [_i64, _i32, _vp, _vp, _i32, _i32, _vp, _vp, _sz, _kp, _vp]),
    "lift_gemv_ex": (_i32, [_i64, _i64, _f32, _i32, _vp, _i64, _vp, _f32, _vp, _i32, _kp, _vp]),
    "lift_blackscholes": (_i32, [_i64, _vp, _f32, _f32, _f32, _f32, _vp, _vp]),
    "lift_blackscholes_ex": (_i32, [_i64, _vp, _f32, _f32, _f32, _f32, _vp, _kp, _vp]),
    "lift_md": (_i32, [_i64, _vp, _i64, _vp, _f32, _f32, _f32, _vp, _vp]),
    "lift_md_ex": (_i32, [_i64, _vp, _i64, _vp, _f32, _f32, _f32, _vp, _kp, _vp]),
    "lift_status_string": (ctypes.c_char_p, [_i32]),
    "lift_last_hip_error": (_i32, []),
    "lift_version": (ctypes.c_char_p, []),
    "lift_time_next_launch": (_i32, [_vp, _vp]),
    "lift_batch_create": (_i32, [ctypes.POINTER(lift_problem), ctypes.c_int32, _i32, _i32, _i32, _kp,
                                 ctypes.POINTER(ctypes.c_void_p)]),
    "lift_batch_run": (_i32, [_vp, _vp]),
    "lift_batch_capture": (_i32, [_vp, _vp, ctypes.POINTER(ctypes.c_void_p)]),
    "lift_batch_info": (_i32, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                               ctypes.POINTER(ctypes.c_int64)]),
    "lift_batch_destroy": (None, [_vp]),
    "lift_stream_read": (_i32, [_i64, _vp, _vp, _kp, _vp]),
    "lift_stream_copy": (_i32, [_i64, _vp, _vp, _kp, _vp]),
    "lift_stamp_next_launch": (_i32, [_vp, _i64, ctypes.POINTER(ctypes.c_int32)]),
    "lift_dot_ex_noalloc": (_i32, [_i64, _i32, _vp, _vp, _i32, _i32, _vp, _kp, _vp]),
    "lift_default_knobs": (_i32, [ctypes.c_char_p, _i32, _i32, _i64, _i64, ctypes.c_char_p, ctypes.c_int32, _kp]),
}


def _lib():
    global _LIB
    if _LIB is None:
        with _LOCK:
            if _LIB is None:
                if not os.path.exists(LIB_PATH):
                    raise ImportError(
                        f"{LIB_PATH} is not built; run `python -m paper_1502_02389_amd.build` "
                        "(there is no CPU fallback)")
                lib = ctypes.CDLL(LIB_PATH)
                for name, (res, args) in SIGNATURES.items():
                    fn = getattr(lib, name)
                    fn.restype = res
                    fn.argtypes = args
                _LIB = lib
    return _LIB


def library():
    """The loaded ctypes library (loads it on first use)."""
    return _lib()


# ---------------------------------------------------------------- C entry points


def lift_scal(n, alpha, x, out, stream=0):
    return _lib().lift_scal(n, alpha, x, out, stream)


def lift_asum(n, x, result, ws, ws_bytes, stream=0):
    return _lib().lift_asum(n, x, result, ws, ws_bytes, stream)


def lift_dot(n, x, y, result, ws, ws_bytes, stream=0):
    return _lib().lift_dot(n, x, y, result, ws, ws_bytes, stream)


def lift_gemv(m, n, alpha, A, lda, x, beta, y, stream=0):
    return _lib().lift_gemv(m, n, alpha, A, lda, x, beta, y, stream)


def lift_workspace_bytes():
    return _lib().lift_workspace_bytes()


def lift_max_workgroups():
    return _lib().lift_max_workgroups()


def _kptr(k):
    return ctypes.byref(k) if k is not None else None


def lift_scal_ex(n, alpha, x, out, knobs=None, stream=0):
    return _lib().lift_scal_ex(n, alpha, x, out, _kptr(knobs), stream)


def lift_asum_ex(n, xt, x, acc, rt, result, ws, ws_bytes, knobs=None, stream=0):
    return _lib().lift_asum_ex(n, xt, x, acc, rt, result, ws, ws_bytes, _kptr(knobs), stream)


def lift_dot_ex(n, xt, x, y, acc, rt, result, ws, ws_bytes, knobs=None, stream=0):
    return _lib().lift_dot_ex(n, xt, x, y, acc, rt, result, ws, ws_bytes, _kptr(knobs), stream)


def lift_dot_ex_noalloc(n, xt, x, y, acc, rt, result, knobs=None, stream=0):
    return _lib().lift_dot_ex_noalloc(n, xt, x, y, acc, rt, result, _kptr(knobs), stream)


def lift_gemv_ex(m, n, alpha, at, A, lda, x, beta, y, acc, knobs=None, stream=0):
    return _lib().lift_gemv_ex(m, n, alpha, at, A, lda, x, beta, y, acc, _kptr(knobs), stream)


def lift_blackscholes(n, s, strike, rate, volatility, years, call_put, stream=0):
    return _lib().lift_blackscholes(n, s, strike, rate, volatility, years, call_put, stream)


def lift_blackscholes_ex(n, s, strike, rate, volatility, years, call_put, knobs=None, stream=0):
    return _lib().lift_blackscholes_ex(n, s, strike, rate, volatility, years, call_put, _kptr(knobs), stream)


def lift_md(n, pos, k, nbr, cutoff, epsilon, sigma, force, stream=0):
    return _lib().lift_md(n, pos, k, nbr, cutoff, epsilon, sigma, force, stream)


def lift_md_ex(n, pos, k, nbr, cutoff, epsilon, sigma, force, knobs=None, stream=0):
    return _lib().lift_md_ex(n, pos, k, nbr, cutoff, epsilon, sigma, force, _kptr(knobs), stream)


def lift_stream_read(n, x, sink, knobs=None, stream=0):
    return _lib().lift_stream_read(n, x, sink, _kptr(knobs), stream)


def lift_stream_copy(n, x, out, knobs=None, stream=0):
    return _lib().lift_stream_copy(n, x, out, _kptr(knobs), stream)


def lift_default_knobs(op, storage, acc, elements, arch=None, cus=0, row_length=0):
    """(source, knobs dict) of a call without knobs: source 2 = LIFT_FORCE_CONFIG,
    1 = the tuned table, 0 = the defaults (all-zero knobs); arch None = the
    current device; row_length: gemv's n.  Raises LiftError on a negative
    status."""
    k = lift_knobs()
    st = _lib().lift_default_knobs(op.encode(), storage, acc, elements, row_length, arch.encode() if arch else None,
                                   cus, ctypes.byref(k))
    if st < 0:
        raise LiftError(st, "lift_default_knobs")
    return st, {f: getattr(k, f) for f, _ in lift_knobs._fields_}


def lift_stamp_next_launch(stamps, capacity):
    """Arm the stamped instances for the next asum / dot launch or batch run
    (see lift_stamp_next_launch in lift.h); returns (status, clock rate in kHz)."""
    khz = ctypes.c_int32(0)
    st = _lib().lift_stamp_next_launch(stamps, capacity, ctypes.byref(khz) if stamps else None)
    return st, khz.value


def lift_status_string(status):
    return _lib().lift_status_string(status).decode()


def lift_last_hip_error():
    return _lib().lift_last_hip_error()


def lift_version():
    return _lib().lift_version().decode()


def lift_time_next_launch(start, stop):
    return _lib().lift_time_next_launch(start, stop)


def lift_batch_create(probs, count, storage, acc, rt, knobs, out):
    """probs: ctypes array of lift_problem; out: ctypes.c_void_p receiving the handle."""
    return _lib().lift_batch_create(probs, count, storage, acc, rt, _kptr(knobs), ctypes.byref(out))


def lift_batch_run(batch, stream=0):
    return _lib().lift_batch_run(batch, stream)


def lift_batch_capture(batch, stream, exec_out):
    """exec_out: ctypes.c_void_p receiving the hipGraphExec_t."""
    return _lib().lift_batch_capture(batch, stream, ctypes.byref(exec_out))


def lift_batch_info(batch):
    t, g, b = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
    st = _lib().lift_batch_info(batch, ctypes.byref(t), ctypes.byref(g), ctypes.byref(b))
    return st, t.value, g.value, b.value


def lift_batch_destroy(batch):
    _lib().lift_batch_destroy(batch)


class HipEvents:
    """Raw HIP events (hipEventCreate) for lift_time_next_launch, via ctypes."""

    def __init__(self, count):
        self._hip = ctypes.CDLL("libamdhip64.so")
        self._hip.hipEventCreate.argtypes = [ctypes.POINTER(ctypes.c_void_p)]
        self._hip.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p, ctypes.c_void_p]
        self._hip.hipEventDestroy.argtypes = [ctypes.c_void_p]
        self.events = []
        for _ in range(count):
            ev = ctypes.c_void_p()
            if self._hip.hipEventCreate(ctypes.byref(ev)) != 0:
                raise RuntimeError("hipEventCreate failed")
            self.events.append(ev.value)

    def elapsed_ms(self, a, b):
        ms = ctypes.c_float()
        err = self._hip.hipEventElapsedTime(ctypes.byref(ms), self.events[a], self.events[b])
        if err != 0:
            raise RuntimeError(f"hipEventElapsedTime failed ({err})")
        return ms.value

    def close(self):
        for ev in self.events:
            self._hip.hipEventDestroy(ev)
        self.events = []


# ---------------------------------------------------------------- tensor layer


def _torch():
    import torch

    return torch


_WS = {}
_WS_LOCK = threading.Lock()


def _stream_handle(device):
    torch = _torch()
    return torch.cuda.current_stream(device).cuda_stream


def workspace(device, stream=None):
    """The zero-initialised workspace for (device, stream), allocated once.

    Every asum/dot call leaves it zeroed again, so it is reused without a
    memset; concurrent streams get their own.
    """
    torch = _torch()
    device = torch.device(device)
    handle = _stream_handle(device) if stream is None else stream
    key = (device.index, handle)
    with _WS_LOCK:
        ws = _WS.get(key)
        if ws is None:
            ws = torch.zeros(lift_workspace_bytes(), dtype=torch.uint8, device=device)
            _WS[key] = ws
    return ws


_DT = None


def _dtype_code(t):
    torch = _torch()
    global _DT
    if _DT is None:
        _DT = {torch.float32: LIFT_F32, torch.bfloat16: LIFT_BF16, torch.float16: LIFT_F16,
               torch.float64: LIFT_F64}
    try:
        return _DT[t]
    except KeyError:
        raise TypeError(f"unsupported dtype {t}") from None


def _check_tensor(t, name, dtypes):
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a GPU (got {t.device}); there is no CPU path")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


def _ok(status, what):
    if status != LIFT_OK:
        raise LiftError(status, what)


def scal(alpha, x, out=None, knobs=None):
    """out = alpha * x (binary32); ``out`` may be ``x`` for in-place."""
    torch = _torch()
    _check_tensor(x, "x", (torch.float32,))
    if out is None:
        out = torch.empty_like(x)
    _check_tensor(out, "out", (torch.float32,))
    if out.numel() != x.numel():
        raise ValueError("out must match x")
    s = _stream_handle(x.device)
    _ok(lift_scal_ex(x.numel(), float(alpha), x.data_ptr(), out.data_ptr(), knobs, s), "lift_scal")
    return out


def _reduce(which, x, y, acc, result_dtype, knobs):
    torch = _torch()
    _check_tensor(x, "x", (torch.float32, torch.bfloat16, torch.float16))
    if y is not None:
        _check_tensor(y, "y", (x.dtype,))
        if y.numel() != x.numel():
            raise ValueError("x and y must have the same length")
        if y.device != x.device:
            raise ValueError("x and y must be on the same device")
    result = torch.empty((), dtype=result_dtype, device=x.device)
    ws = workspace(x.device)
    s = _stream_handle(x.device)
    accc = ACC[acc] if isinstance(acc, str) else int(acc)
    rt = _dtype_code(result_dtype)
    if which == "asum":
        st = lift_asum_ex(x.numel(), _dtype_code(x.dtype), x.data_ptr(), accc, rt, result.data_ptr(),
                          ws.data_ptr(), ws.numel(), knobs, s)
    else:
        st = lift_dot_ex(x.numel(), _dtype_code(x.dtype), x.data_ptr(), y.data_ptr(), accc, rt,
                         result.data_ptr(), ws.data_ptr(), ws.numel(), knobs, s)
    _ok(st, f"lift_{which}")
    return result


def asum(x, acc="f32", result_dtype=None, knobs=None):
    """sum |x_i| as a 0-d device tensor (binary32 unless result_dtype=float64)."""
    torch = _torch()
    return _reduce("asum", x, None, acc, result_dtype or torch.float32, knobs)


def dot(x, y, acc="f32", result_dtype=None, knobs=None):
    """sum x_i y_i as a 0-d device tensor."""
    torch = _torch()
    return _reduce("dot", x, y, acc, result_dtype or torch.float32, knobs)


def blackscholes(s, strike, rate, volatility, years, out=None, knobs=None):
    """map(BSComputation) over binary32 stock prices: an (n, 2) tensor of
    {call, put} per price (``out`` may be given, (n, 2) float32)."""
    torch = _torch()
    _check_tensor(s, "s", (torch.float32,))
    n = s.numel()
    if out is None:
        out = torch.empty((n, 2), dtype=torch.float32, device=s.device)
    _check_tensor(out, "out", (torch.float32,))
    if out.numel() != 2 * n:
        raise ValueError("out must hold two floats per price")
    st = _stream_handle(s.device)
    _ok(lift_blackscholes_ex(n, s.data_ptr(), float(strike), float(rate), float(volatility), float(years),
                             out.data_ptr(), knobs, st), "lift_blackscholes")
    return out


def md(pos, nbr, cutoff, epsilon, sigma, out=None, knobs=None):
    """Forces on n particles from their neighbour lists: pos (n, 4) float32,
    nbr (n, k) int32 (outside [0, n) = empty slot); returns (n, 4) float32
    (fx, fy, fz, 0)."""
    torch = _torch()
    _check_tensor(pos, "pos", (torch.float32,))
    _check_tensor(nbr, "nbr", (torch.int32,))
    if pos.dim() != 2 or pos.shape[1] != 4:
        raise ValueError("pos must be (n, 4)")
    if nbr.dim() != 2 or nbr.shape[0] != pos.shape[0]:
        raise ValueError("nbr must be (n, k)")
    n, k = pos.shape[0], nbr.shape[1]
    if out is None:
        out = torch.empty((n, 4), dtype=torch.float32, device=pos.device)
    _check_tensor(out, "out", (torch.float32,))
    if out.numel() != 4 * n:
        raise ValueError("out must be (n, 4)")
    st = _stream_handle(pos.device)
    _ok(lift_md_ex(n, pos.data_ptr(), k, nbr.data_ptr(), float(cutoff), float(epsilon), float(sigma),
                   out.data_ptr(), knobs, st), "lift_md")
    return out


def gemv(alpha, A, x, beta, y, acc="f32", knobs=None, lda=None):
    """y <- alpha * A x + beta * y in place (row-major A, rows of length lda).

    ``A`` is (m, lda) with the matrix in its first n = len(x) columns.
    """
    torch = _torch()
    _check_tensor(A, "A", (torch.float32, torch.bfloat16, torch.float16))
    _check_tensor(x, "x", (torch.float32,))
    _check_tensor(y, "y", (torch.float32,))
    if A.dim() != 2:
        raise ValueError("A must be 2-D")
    m, n = A.shape[0], x.numel()
    lda = A.shape[1] if lda is None else lda
    if A.shape[1] != lda or lda < n:
        raise ValueError("A must be (m, lda) with lda >= len(x)")
    if y.numel() != m:
        raise ValueError("y must have one entry per row of A")
    s = _stream_handle(A.device)
    accc = ACC[acc] if isinstance(acc, str) else int(acc)
    _ok(lift_gemv_ex(m, n, float(alpha), _dtype_code(A.dtype), A.data_ptr(), lda, x.data_ptr(),
                     float(beta), y.data_ptr(), accc, knobs, s), "lift_gemv")
    return y


# ---------------------------------------------------------------- batched form


class Batch:
    """Many asum / dot / gemv problems run as two persistent kernels (reduction
    tiles, then gemv tiles) on one stream.

    ``problems`` is a list of tuples:
      ("asum", x)                       -> result written to a 0-d tensor
      ("dot", x, y)
      ("gemv", alpha, A, x, beta, y)    -> y updated in place (A is (m, lda))
    All x / y / A of reductions and A of gemv share one storage dtype; gemv x
    and y are float32.  The tensors are kept alive by the batch; results
    live in ``self.results`` (one 0-d tensor per reduction, None for gemv).
    """

    def __init__(self, problems, acc="f32", result_dtype=None, knobs=None, device=None):
        torch = _torch()
        self._hip = None
        self.handle = ctypes.c_void_p()
        self.keep = []
        self.results = []
        dev = torch.device(device) if device is not None else None
        storage = None
        arr = (lift_problem * max(1, len(problems)))()
        rdt = result_dtype or torch.float32
        for i, pr in enumerate(problems):
            kind = pr[0]
            q = arr[i]
            if kind in ("asum", "dot"):
                x = pr[1]
                _check_tensor(x, "x", (torch.float32, torch.bfloat16, torch.float16))
                dev = dev or x.device
                storage = storage or x.dtype
                if x.dtype != storage:
                    raise TypeError("every problem of a batch uses one storage dtype")
                res = torch.zeros((), dtype=rdt, device=dev)
                q.kind = LIFT_KIND_ASUM if kind == "asum" else LIFT_KIND_DOT
                q.n = x.numel()
                q.a = x.data_ptr() or None
                q.out = res.data_ptr()
                self.keep.append(x)
                if kind == "dot":
                    y = pr[2]
                    _check_tensor(y, "y", (storage,))
                    if y.numel() != x.numel():
                        raise ValueError("dot operands differ in length")
                    q.b = y.data_ptr() or None
                    self.keep.append(y)
                self.results.append(res)
            elif kind == "gemv":
                alpha, A, x, beta, y = pr[1:6]
                _check_tensor(A, "A", (torch.float32, torch.bfloat16, torch.float16))
                _check_tensor(x, "x", (torch.float32,))
                _check_tensor(y, "y", (torch.float32,))
                dev = dev or A.device
                storage = storage or A.dtype
                if A.dtype != storage:
                    raise TypeError("every problem of a batch uses one storage dtype")
                q.kind = LIFT_KIND_GEMV
                q.m, q.n, q.lda = A.shape[0], x.numel(), A.shape[1]
                q.a, q.b, q.out = A.data_ptr() or None, x.data_ptr() or None, y.data_ptr() or None
                q.alpha, q.beta = float(alpha), float(beta)
                self.keep += [A, x, y]
                self.results.append(None)
            else:
                raise ValueError(f"unknown problem kind {kind!r}")
        storage = storage or torch.float32
        self.device = dev or torch.device("cuda", torch.cuda.current_device())
        with torch.cuda.device(self.device):
            st = lift_batch_create(arr, len(problems), _dtype_code(storage), ACC[acc] if isinstance(acc, str)
                                   else int(acc), _dtype_code(rdt), knobs, self.handle)
        _ok(st, "lift_batch_create")
        _, self.tiles, self.grid, self.bytes = lift_batch_info(self.handle)
        self.graphs = []

    def run(self, stream=None):
        s = _stream_handle(self.device) if stream is None else stream
        _ok(lift_batch_run(self.handle, s), "lift_batch_run")

    def capture(self, stream):
        """Capture one run into a HIP graph on `stream` (a non-default
        torch.cuda.Stream or raw handle); returns a replayable GraphRun."""
        h = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        ex = ctypes.c_void_p()
        _ok(lift_batch_capture(self.handle, h, ex), "lift_batch_capture")
        g = GraphRun(ex.value)
        self.graphs.append(g)
        return g

    def close(self):
        for g in self.graphs:
            g.close()
        self.graphs = []
        if self.handle:
            lift_batch_destroy(self.handle)
            self.handle = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class GraphRun:
    """An instantiated HIP graph (hipGraphExec_t) replayed with hipGraphLaunch."""

    def __init__(self, exec_handle):
        self.exec = exec_handle
        self._hip = ctypes.CDLL("libamdhip64.so")
        self._hip.hipGraphLaunch.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
        self._hip.hipGraphExecDestroy.argtypes = [ctypes.c_void_p]

    def launch(self, stream):
        h = stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream)
        err = self._hip.hipGraphLaunch(self.exec, h)
        if err != 0:
            raise RuntimeError(f"hipGraphLaunch failed ({err})")

    def close(self):
        if self.exec:
            self._hip.hipGraphExecDestroy(self.exec)
            self.exec = None
