"""Thin ctypes binding of libtde.so (include/tde.h).

Argument marshalling only: every step of the estimator runs in the library's
HIP kernels. PyTorch provides device memory (``Tensor.data_ptr()``) and the
current HIP stream. The functions keep the C names; ``Context`` adds
conveniences that allocate outputs and workspaces with torch.

Importing this module needs the built ``libtde.so`` (``python -m
paper_2509_19974_amd.build``); there is no fallback of any kind.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtde.so")

TDE_OK = 0
TDE_ERR_ARG = -1
TDE_ERR_RANGE = -2
TDE_ERR_WS = -3
TDE_ERR_HIP = -4
TDE_ERR_UNSUPPORTED = -5
TDE_ERR_IO = -6

TDE_I32, TDE_I64 = 0, 1
TDE_PATH_AUTO, TDE_PATH_MFMA, TDE_PATH_POPC, TDE_PATH_NTT, TDE_PATH_MFMA_I8 = 0, 1, 2, 3, 4
TDE_MODE_FULL, TDE_MODE_LEARNED = 0, 1
TDE_QUANT_UNIFORM, TDE_QUANT_MULAW, TDE_QUANT_GAUSS = 0, 1, 2

TDE_FLAG_NONFINITE_X = 1
TDE_FLAG_NONFINITE_Y = 2
TDE_FLAG_ZERO_X = 4
TDE_FLAG_ZERO_Y = 8
TDE_FLAG_FALLBACK = 16
TDE_FLAG_REFINED = 32
TDE_FLAG_REFINE_PARTIAL = 64
TDE_FLAG_SCALE_EXACT = 128
TDE_FLAG_REFINE_EXACT = 256
TDE_FLAG_REFINE_NONFINITE = 512

PEAK_DTYPE = np.dtype([("lag", "<i8"), ("rmax", "<i8"), ("n_ties", "<i4"), ("flags", "<i4")])
QSTAT_DTYPE = np.dtype([("inv_step", "<f4"), ("flags", "<i4"), ("n_nonfinite", "<i8"), ("n_zero", "<i8"),
                        ("sum_q", "<i8"), ("sum_q2", "<i8")])


class tde_pair(ctypes.Structure):
    _fields_ = [("x", ctypes.c_void_p), ("y", ctypes.c_void_p), ("nx", ctypes.c_int64), ("ny", ctypes.c_int64),
                ("lag_lo", ctypes.c_int64), ("lag_hi", ctypes.c_int64), ("bits", ctypes.c_int32),
                ("inv_step_x", ctypes.c_float), ("inv_step_y", ctypes.c_float), ("r_dtype", ctypes.c_int32),
                ("r_out", ctypes.c_void_p)]


class tde_opts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("path", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("topk", ctypes.c_int32), ("model", ctypes.c_void_p), ("margin", ctypes.c_float),
                ("quantizer", ctypes.c_int32)]


class TDEError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{msg} (status {status})")
        self.status = status


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libtde.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    try:
        # torch carries its own HIP runtime; loading it first makes libtde
        # bind to that one instead of bringing a second copy into the process
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(path):
        raise RuntimeError(f"libtde.so not built: {path} missing (run python -m paper_2509_19974_amd.build)")
    lib = ctypes.CDLL(path)
    i64, i32, f32, vp, sz = ctypes.c_int64, ctypes.c_int, ctypes.c_float, ctypes.c_void_p, ctypes.c_size_t
    sig = {
        "tde_create": (i32, [ctypes.POINTER(vp), i32]),
        "tde_destroy": (None, [vp]),
        "tde_status_string": (ctypes.c_char_p, [i32]),
        "tde_last_error": (ctypes.c_char_p, []),
        "tde_quantize_workspace_size": (sz, [i64]),
        "tde_quantize": (i32, [vp, vp, i64, i32, f32, vp, vp, vp, sz, vp]),
        "tde_quantize_ex": (i32, [vp, vp, i64, i32, i32, f32, vp, vp, vp, sz, vp]),
        "tde_quantizer_thresholds": (i32, [i32, i32, vp]),
        "tde_xcorr_workspace_size": (sz, [i64, i64, i32, i32, i64, i64, i32]),
        "tde_mfma_operand_bits": (i32, [i32, i32, i32]),
        "tde_mfma_tile_lags": (i32, [i64, i64, i32, i32, i64, i64, i32]),
        "tde_xcorr_int": (i32, [vp, vp, i64, vp, i64, i32, i32, i64, i64, vp, i32, i32, vp, sz, vp]),
        "tde_xcorr_int_noalloc": (i32, [vp, vp, i64, vp, i64, i32, i32, i64, i64, vp, i32, i32, vp]),
        "tde_argmax_workspace_size": (sz, [i64]),
        "tde_argmax_lag": (i32, [vp, vp, i32, i64, i64, vp, vp, sz, vp]),
        "tde_estimate_workspace_size": (sz, [ctypes.POINTER(tde_pair), i64, ctypes.POINTER(tde_opts)]),
        "tde_estimate_batch": (i32, [vp, ctypes.POINTER(tde_pair), i64, ctypes.POINTER(tde_opts), vp, vp, sz, vp]),
        "tde_model_create": (i32, [vp, i32, i32, ctypes.c_uint64, ctypes.POINTER(vp)]),
        "tde_model_destroy": (None, [vp]),
        "tde_model_num_params": (i64, [vp]),
        "tde_model_get_params": (i32, [vp, vp, i64]),
        "tde_model_set_params": (i32, [vp, vp, i64]),
        "tde_model_gradients": (i32, [vp, vp, i64]),
        "tde_model_save": (i32, [vp, ctypes.c_char_p]),
        "tde_model_load": (i32, [vp, ctypes.c_char_p]),
        "tde_model_prepare_workspace_size": (sz, [ctypes.POINTER(tde_pair), i64]),
        "tde_model_prepare": (i32, [vp, vp, ctypes.POINTER(tde_pair), i64, vp, vp, sz, vp]),
        "tde_model_forward": (i32, [vp, vp, vp, i64, vp, i32, vp, vp, vp]),
        "tde_train_step": (i32, [vp, vp, vp, vp, i64, f32, ctypes.POINTER(f32), vp]),
        "tde_refine_workspace_size": (sz, [i32]),
        "tde_stream_create": (i32, [vp, vp, i64, i32, f32, f32, i64, i32, ctypes.POINTER(vp), vp]),
        "tde_stream_push": (i32, [vp, vp, i64, vp, i32, vp, vp, vp]),
        "tde_stream_finish": (i32, [vp, vp, i32, vp, vp, vp]),
        "tde_stream_position": (i64, [vp]),
        "tde_stream_destroy": (None, [vp]),
        "tde_refine_ties": (i32, [vp, vp, i64, vp, i64, vp, i32, i64, i64, vp, i32, vp, sz, vp]),
        "tde_tune": (i32, [vp, i32, vp]),
        "tde_tune_query": (i32, [i64, i64, i32, i32, i64, i64]),
        "tde_tune_save": (i32, [ctypes.c_char_p]),
        "tde_tune_load": (i32, [ctypes.c_char_p]),
        "tde_tune_reset": (i32, []),
        "tde_timing_enable": (i32, [vp, i32]),
        "tde_timing_read": (i32, [vp, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int):
    if status != TDE_OK:
        msg = load_library().tde_last_error().decode(errors="replace")
        raise TDEError(status, msg)


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream) -> int | None:
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


# ----------------------------------------------------- C-named functions --

def tde_create(device: int = 0) -> int:
    h = ctypes.c_void_p()
    _check(load_library().tde_create(ctypes.byref(h), device))
    return h.value


def tde_destroy(ctx: int) -> None:
    load_library().tde_destroy(ctx)


def tde_status_string(status: int) -> str:
    return load_library().tde_status_string(status).decode()


def tde_last_error() -> str:
    return load_library().tde_last_error().decode(errors="replace")


def tde_quantize_workspace_size(n: int) -> int:
    return int(load_library().tde_quantize_workspace_size(n))


def tde_quantize(ctx, x, n, bits, inv_step, q, stat=None, ws=None, ws_bytes=0, stream=None, quantizer=0):
    _check(load_library().tde_quantize_ex(ctx, _ptr(x), n, bits, quantizer, float(inv_step), _ptr(q), _ptr(stat),
                                          _ptr(ws), ws_bytes, _stream(stream)))


def tde_quantizer_thresholds(quantizer: int, bits: int) -> np.ndarray:
    out = np.zeros(7, np.float32)
    k = int(load_library().tde_quantizer_thresholds(quantizer, bits, out.ctypes.data))
    if k < 0:
        _check(k)
    return out[:k]


def tde_xcorr_workspace_size(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi, path=TDE_PATH_AUTO) -> int:
    return int(load_library().tde_xcorr_workspace_size(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi, path))


def tde_mfma_tile_lags(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi, path=TDE_PATH_AUTO) -> int:
    """Lags per matrix-core tile (4096 or 8192) for this correlation."""
    st = load_library().tde_mfma_tile_lags(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi, path)
    if st < 0:
        _check(st)
    return int(st)


def tde_mfma_operand_bits(kmax_u, kmax_v, path=TDE_PATH_MFMA) -> int:
    st = int(load_library().tde_mfma_operand_bits(kmax_u, kmax_v, path))
    if st < 0:
        _check(st)
    return st


def tde_xcorr_int(ctx, u, nu, v, nv, kmax_u, kmax_v, lag_lo, lag_hi, r, r_dtype, path=TDE_PATH_AUTO, ws=None,
                  ws_bytes=0, stream=None):
    _check(load_library().tde_xcorr_int(ctx, _ptr(u), nu, _ptr(v), nv, kmax_u, kmax_v, lag_lo, lag_hi, _ptr(r),
                                        r_dtype, path, _ptr(ws), ws_bytes, _stream(stream)))


def tde_argmax_workspace_size(nlags: int) -> int:
    return int(load_library().tde_argmax_workspace_size(nlags))


def tde_argmax_lag(ctx, r, r_dtype, lag_lo, lag_hi, out, ws=None, ws_bytes=0, stream=None):
    _check(load_library().tde_argmax_lag(ctx, _ptr(r), r_dtype, lag_lo, lag_hi, _ptr(out), _ptr(ws), ws_bytes,
                                         _stream(stream)))


def make_pairs(pairs) -> ctypes.Array:
    arr = (tde_pair * len(pairs))()
    for i, p in enumerate(pairs):
        arr[i] = p
    return arr


def tde_estimate_workspace_size(pairs_arr, npairs, opts: tde_opts) -> int:
    return int(load_library().tde_estimate_workspace_size(pairs_arr, npairs, ctypes.byref(opts)))


def tde_estimate_batch(ctx, pairs_arr, npairs, opts: tde_opts, out, ws, ws_bytes, stream=None):
    _check(load_library().tde_estimate_batch(ctx, pairs_arr, npairs, ctypes.byref(opts), _ptr(out), _ptr(ws),
                                             ws_bytes, _stream(stream)))


class Stream:
    """Correlation of a stream against a template, block by block
    (tde_stream): push float32 device blocks, then finish."""

    def __init__(self, ctx: "Context", x, bits: int, inv_step_y: float, max_block: int, inv_step_x: float = 0.0,
                 path: int = TDE_PATH_AUTO, stream=None):
        self.ctx = ctx
        self.nx = x.numel()
        h = ctypes.c_void_p()
        _check(load_library().tde_stream_create(ctx.handle, _ptr(x), x.numel(), bits, float(inv_step_x),
                                                float(inv_step_y), max_block, path, ctypes.byref(h),
                                                _stream(stream)))
        self.handle = h.value

    def close(self):
        if self.handle:
            load_library().tde_stream_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def position(self) -> int:
        return int(load_library().tde_stream_position(self.handle))

    def push(self, y, want_r=False, r_dtype=TDE_I64, stream=None):
        """Returns (r or None, block peak bytes, running peak bytes) on the device."""
        torch = self.ctx.torch
        r = (torch.empty(y.numel(), dtype=torch.int32 if r_dtype == TDE_I32 else torch.int64, device=self.ctx.device)
             if want_r else None)
        pk = self.ctx._bytes(2 * PEAK_DTYPE.itemsize)
        _check(load_library().tde_stream_push(self.handle, _ptr(y), y.numel(), _ptr(r), r_dtype, _ptr(pk),
                                              _ptr(pk) + PEAK_DTYPE.itemsize, _stream(stream)))
        return r, pk[:PEAK_DTYPE.itemsize], pk[PEAK_DTYPE.itemsize:]

    def finish(self, want_r=False, r_dtype=TDE_I64, stream=None):
        torch = self.ctx.torch
        n = self.nx - 1
        r = (torch.empty(max(n, 1), dtype=torch.int32 if r_dtype == TDE_I32 else torch.int64, device=self.ctx.device)
             if want_r else None)
        pk = self.ctx._bytes(2 * PEAK_DTYPE.itemsize)
        pk.zero_()
        _check(load_library().tde_stream_finish(self.handle, _ptr(r), r_dtype, _ptr(pk),
                                                _ptr(pk) + PEAK_DTYPE.itemsize, _stream(stream)))
        return (r[:n] if r is not None else None), pk[:PEAK_DTYPE.itemsize], pk[PEAK_DTYPE.itemsize:]


class Model:
    """Learned lag-window proposer (tde_model) on the context's device."""

    def __init__(self, ctx: "Context", ld: int = 16384, nbins: int = 512, seed: int = 1):
        self.ctx = ctx
        self.ld, self.nbins = ld, nbins
        h = ctypes.c_void_p()
        _check(load_library().tde_model_create(ctx.handle, ld, nbins, seed, ctypes.byref(h)))
        self.handle = h.value

    def close(self):
        if self.handle:
            load_library().tde_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def num_params(self) -> int:
        return int(load_library().tde_model_num_params(self.handle))

    def get_params(self) -> np.ndarray:
        a = np.empty(self.num_params, np.float32)
        _check(load_library().tde_model_get_params(self.handle, a.ctypes.data, a.size))
        return a

    def set_params(self, a) -> None:
        a = np.ascontiguousarray(a, dtype=np.float32)
        _check(load_library().tde_model_set_params(self.handle, a.ctypes.data, a.size))

    def gradients(self) -> np.ndarray:
        a = np.empty(self.num_params, np.float32)
        _check(load_library().tde_model_gradients(self.handle, a.ctypes.data, a.size))
        return a

    def save(self, path: str) -> None:
        _check(load_library().tde_model_save(self.handle, path.encode()))

    def load(self, path: str) -> None:
        _check(load_library().tde_model_load(self.handle, path.encode()))

    def prepare(self, specs, stream=None):
        """Decimated bf16 inputs (int16 tensor [B][2][ld], bf16 bit patterns)."""
        torch = self.ctx.torch
        arr, _, _ = self.ctx.batch_plan(specs)
        n = len(arr)
        wsb = int(load_library().tde_model_prepare_workspace_size(arr, n))
        ws = self.ctx._bytes(wsb)
        out = torch.empty((n, 2, self.ld), dtype=torch.int16, device=self.ctx.device)
        _check(load_library().tde_model_prepare(self.ctx.handle, self.handle, arr, n, _ptr(out), _ptr(ws), wsb,
                                                _stream(stream)))
        return out

    def forward(self, xdec, topk: int = 0, stream=None):
        torch = self.ctx.torch
        B = xdec.shape[0]
        logits = torch.empty((B, self.nbins), dtype=torch.float32, device=self.ctx.device)
        top = torch.empty((B, max(topk, 1)), dtype=torch.int32, device=self.ctx.device) if topk else None
        margin = torch.empty(B, dtype=torch.float32, device=self.ctx.device) if topk else None
        _check(load_library().tde_model_forward(self.ctx.handle, self.handle, _ptr(xdec), B, _ptr(logits), topk,
                                                _ptr(top), _ptr(margin), _stream(stream)))
        return logits, top, margin

    def train_step(self, xdec, labels, lr: float, stream=None, want_loss: bool = True) -> float:
        """One Adam step; returns the mean loss (the call then waits for the
        stream), or nan with want_loss=False (no wait)."""
        loss = ctypes.c_float(0.0)
        _check(load_library().tde_train_step(self.ctx.handle, self.handle, _ptr(xdec), _ptr(labels), xdec.shape[0],
                                             float(lr), ctypes.byref(loss) if want_loss else None, _stream(stream)))
        return float(loss.value) if want_loss else float("nan")


def tde_tune(ctx, max_log_n: int = 22, stream=None) -> None:
    _check(load_library().tde_tune(ctx, max_log_n, _stream(stream)))


def tde_tune_query(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi) -> int:
    st = load_library().tde_tune_query(nu, nv, kmax_u, kmax_v, lag_lo, lag_hi)
    if st < 0:
        _check(st)
    return st


def tde_tune_save(path: str) -> None:
    _check(load_library().tde_tune_save(path.encode()))


def tde_tune_load(path: str) -> None:
    _check(load_library().tde_tune_load(path.encode()))


def tde_tune_reset() -> None:
    _check(load_library().tde_tune_reset())


def tde_timing_enable(ctx, on: bool) -> None:
    _check(load_library().tde_timing_enable(ctx, 1 if on else 0))


TDE_STAGES = 7


def tde_timing_read(ctx):
    """Returns (ms, count) lists for the stages quantize, engine, argmax,
    whole call, proposer."""
    ms = (ctypes.c_double * TDE_STAGES)()
    cnt = (ctypes.c_int64 * TDE_STAGES)()
    _check(load_library().tde_timing_read(ctx, ms, cnt))
    return list(ms), list(cnt)


# ------------------------------------------------------------ conveniences --

def kmax_of_bits(bits: int) -> int:
    return 1 if bits == 1 else (1 << (bits - 1)) - 1


def decode_peaks(buf) -> np.ndarray:
    """Device uint8 tensor of n*24 bytes -> numpy structured array."""
    raw = buf.detach().cpu().numpy().tobytes()
    return np.frombuffer(raw, dtype=PEAK_DTYPE).copy()


def decode_qstat(buf) -> np.ndarray:
    raw = buf.detach().cpu().numpy().tobytes()
    return np.frombuffer(raw, dtype=QSTAT_DTYPE).copy()


class Context:
    """Owns a tde_ctx on one device; methods allocate with torch and call the C ABI."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = torch.device("cuda", device)
        self.handle = tde_create(device)

    def close(self):
        if self.handle:
            tde_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _bytes(self, n):
        return self.torch.empty(max(int(n), 1), dtype=self.torch.uint8, device=self.device)

    def quantize(self, x, bits: int, inv_step: float = 0.0, stream=None, quantizer: int = 0):
        """Returns (q int8 tensor, qstat record)."""
        torch = self.torch
        n = x.numel()
        q = torch.empty(n, dtype=torch.int8, device=self.device)
        stat = self._bytes(QSTAT_DTYPE.itemsize)
        wsb = tde_quantize_workspace_size(n)
        ws = self._bytes(wsb)
        tde_quantize(self.handle, x, n, bits, inv_step, q, stat, ws, wsb, stream, quantizer)
        return q, stat

    def xcorr(self, u, v, kmax_u, kmax_v, lag_lo, lag_hi, r_dtype=TDE_I64, path=TDE_PATH_AUTO, stream=None):
        torch = self.torch
        L = lag_hi - lag_lo + 1
        r = torch.empty(L, dtype=torch.int32 if r_dtype == TDE_I32 else torch.int64, device=self.device)
        wsb = tde_xcorr_workspace_size(u.numel(), v.numel(), kmax_u, kmax_v, lag_lo, lag_hi, path)
        ws = self._bytes(wsb)
        tde_xcorr_int(self.handle, u, u.numel(), v, v.numel(), kmax_u, kmax_v, lag_lo, lag_hi, r, r_dtype, path,
                      ws, wsb, stream)
        return r

    def argmax(self, r, lag_lo, lag_hi, stream=None):
        r_dtype = TDE_I32 if r.dtype == self.torch.int32 else TDE_I64
        out = self._bytes(PEAK_DTYPE.itemsize)
        wsb = tde_argmax_workspace_size(lag_hi - lag_lo + 1)
        ws = self._bytes(wsb)
        tde_argmax_lag(self.handle, r, r_dtype, lag_lo, lag_hi, out, ws, wsb, stream)
        return out

    def refine(self, x, y, r, lag_lo, lag_hi, peak, max_ties=4096, stream=None):
        """Algorithm 1, tie-refinement step on a peak record (uint8 tensor of 24 bytes,
        updated in place); r is the pair's full correlation (int32/int64)."""
        r_dtype = TDE_I32 if r.dtype == self.torch.int32 else TDE_I64
        wsb = int(load_library().tde_refine_workspace_size(max_ties))
        ws = self._bytes(wsb)
        _check(load_library().tde_refine_ties(self.handle, _ptr(x), x.numel(), _ptr(y), y.numel(), _ptr(r), r_dtype,
                                              lag_lo, lag_hi, _ptr(peak), max_ties, _ptr(ws), wsb, _stream(stream)))
        return peak

    def batch_plan(self, specs, path=TDE_PATH_AUTO, mode=TDE_MODE_FULL, use_graph=0, model=None, topk=8,
                   margin=0.0, quantizer=TDE_QUANT_UNIFORM):
        """specs: list of dicts with x, y (device float32 tensors), lag_lo, lag_hi,
        bits, optional inv_step_x/y, r_out, r_dtype. Returns (pairs array, opts,
        workspace bytes)."""
        pairs = []
        for s in specs:
            p = tde_pair()
            p.x, p.y = _ptr(s["x"]), _ptr(s["y"])
            p.nx, p.ny = s["x"].numel(), s["y"].numel()
            p.lag_lo, p.lag_hi = int(s["lag_lo"]), int(s["lag_hi"])
            p.bits = int(s["bits"])
            p.inv_step_x = float(s.get("inv_step_x", 0.0))
            p.inv_step_y = float(s.get("inv_step_y", 0.0))
            r_out = s.get("r_out")
            p.r_out = _ptr(r_out) if r_out is not None else None
            p.r_dtype = int(s.get("r_dtype", TDE_I64))
            pairs.append(p)
        arr = make_pairs(pairs)
        opts = tde_opts(mode, path, int(use_graph), int(topk), model.handle if model is not None else None,
                        float(margin), int(quantizer))
        wsb = tde_estimate_workspace_size(arr, len(pairs), opts)
        if wsb == 0:
            raise TDEError(TDE_ERR_ARG, tde_last_error())
        return arr, opts, wsb

    def estimate_batch(self, specs, path=TDE_PATH_AUTO, ws=None, out=None, stream=None, plan=None):
        arr, opts, wsb = plan if plan is not None else self.batch_plan(specs, path)
        n = len(arr)
        if out is None:
            out = self._bytes(n * PEAK_DTYPE.itemsize)
        if ws is None:
            ws = self._bytes(wsb)
        tde_estimate_batch(self.handle, arr, n, opts, out, ws, wsb, stream)
        return out
