"""Python binding of libapx (ctypes).  Argument marshalling only: every step of the convolution
runs in the HIP kernels of libapx.so.  PyTorch provides device memory and streams.

The functions mirror the C ABI of include/apx.h with the same names; tensors are passed as
device pointers.  The library must be built (paper_1201_3018_amd/build.py); importing this module
without it raises, there is no other code path.
"""
from __future__ import annotations

import ctypes
import math
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libapx.so")

APX_OK, APX_E_INVALID, APX_E_BOUND, APX_E_NOMEM, APX_E_DEVICE, APX_E_UNSUPPORTED = 0, -1, -2, -3, -4, -5
APX_FULL_FP32, APX_SYM, APX_ASYM2, APX_ASYM3, APX_AUTO_SNR, APX_FULL_FP64 = 0, 1, 2, 3, 4, 5
APX_CORE_AUTO, APX_CORE_TIME, APX_CORE_FFT, APX_CORE_INT8 = 0, 1, 2, 3
APX_CONV, APX_XCORR = 0, 1
APX_FLAG_NONFINITE, APX_FLAG_ZERO = 1, 2
APX_FB_F16X3, APX_FB_BF16X3 = 0, 1
APX_MARGINAL_LAPLACE, APX_MARGINAL_WEIBULL = 0, 1

MODE_NAMES = {APX_FULL_FP32: "full", APX_SYM: "sym", APX_ASYM2: "asym2", APX_ASYM3: "asym3",
              APX_AUTO_SNR: "auto", APX_FULL_FP64: "full64"}

# Every exported symbol of include/apx.h.
EXPORTS = ("apx_create", "apx_destroy", "apx_geometry", "apx_kernel_create", "apx_kernel_destroy", "apx_run",
           "apx_debug_fields", "apx_calibrate", "apx_conv", "apx_xcorr", "apx_kernel_describe", "apx_batch_create",
           "apx_batch_run", "apx_batch_blocks", "apx_batch_describe", "apx_batch_destroy", "apx_xcorr_argmax_batch",
           "apx_fbank_create", "apx_fbank_run", "apx_fbank_describe", "apx_fbank_destroy", "apx_workspace_bytes",
           "apx_run_auto", "apx_server_create", "apx_server_submit", "apx_server_poll", "apx_server_drain",
           "apx_server_stats", "apx_server_destroy", "apx_server_now", "apx_fit_marginal", "apx_status_str",
           "apx_last_error", "apx_many_create", "apx_many_run", "apx_many_describe", "apx_many_destroy", "apx_run_auto_noalloc",
           "apx_tune", "apx_tune_describe")


class apx_params(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("core", ctypes.c_int32), ("Sq", ctypes.c_int32), ("Kq", ctypes.c_int32),
                ("snr_min_db", ctypes.c_double), ("calib_db", ctypes.c_double), ("allow_unsafe", ctypes.c_int32),
                ("fft_variant", ctypes.c_int32), ("sigma_s", ctypes.c_double), ("sigma_k", ctypes.c_double)]


class apx_block_info(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int32), ("flags", ctypes.c_int32), ("Sq", ctypes.c_int32), ("Kq", ctypes.c_int32),
                ("rmax", ctypes.c_int64), ("cs", ctypes.c_double), ("smax", ctypes.c_double), ("rms", ctypes.c_double),
                ("snr_pred_db", ctypes.c_double)]


BLOCK_INFO_DTYPE = np.dtype([("mode", "<i4"), ("flags", "<i4"), ("Sq", "<i4"), ("Kq", "<i4"), ("rmax", "<i8"),
                             ("cs", "<f8"), ("smax", "<f8"), ("rms", "<f8"), ("snr_pred_db", "<f8")])
assert BLOCK_INFO_DTYPE.itemsize == ctypes.sizeof(apx_block_info)


class apx_tuned(ctypes.Structure):
    _fields_ = [("core", ctypes.c_int32), ("fft_variant", ctypes.c_int32), ("W_block", ctypes.c_int32),
                ("tile", ctypes.c_int32), ("ps_per_output", ctypes.c_double)]


class apx_server_config(ctypes.Structure):
    _fields_ = [("hbm_budget", ctypes.c_int64), ("n_streams", ctypes.c_int32), ("max_inflight", ctypes.c_int32)]


class apx_request(ctypes.Structure):
    _fields_ = [("kernel_key", ctypes.c_uint64), ("k", ctypes.c_void_p), ("N", ctypes.c_int32), ("op", ctypes.c_int32),
                ("s", ctypes.c_void_p), ("L", ctypes.c_int64), ("r_out", ctypes.c_void_p),
                ("snr_min_db", ctypes.c_double), ("W_block", ctypes.c_int32), ("mode", ctypes.c_int32)]


class apx_completion(ctypes.Structure):
    _fields_ = [("ticket", ctypes.c_uint64), ("status", ctypes.c_int32), ("core", ctypes.c_int32),
                ("W_block", ctypes.c_int32), ("N", ctypes.c_int32), ("L", ctypes.c_int64),
                ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double)]


class apx_server_counters(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "failed", "rejected", "kernel_hits",
                                              "kernel_misses", "evictions", "peak_bytes", "reserved_bytes")] + \
               [("cached_kernels", ctypes.c_int32), ("pad", ctypes.c_int32), ("launches", ctypes.c_int64)]


class ApxError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"apx status {status}: {msg}")
        self.status = status


_lib = None


def lib() -> ctypes.CDLL:
    """Load libapx.so (in-tree).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python {os.path.join(HERE, 'build.py')}`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dp = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        L.apx_create.argtypes = [ctypes.c_int, ctypes.POINTER(vp)]
        L.apx_destroy.argtypes = [vp]
        L.apx_geometry.argtypes = [i64, i32, i32, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i64)]
        L.apx_kernel_create.argtypes = [vp, vp, i32, i32, i32, ctypes.POINTER(apx_params), vp, ctypes.POINTER(vp)]
        L.apx_kernel_destroy.argtypes = [vp]
        L.apx_run.argtypes = [vp, vp, vp, i64, vp, vp, vp]
        L.apx_debug_fields.argtypes = [vp, vp, vp, i64, vp, vp]
        L.apx_calibrate.argtypes = [vp, vp, vp, i64, i32, i32, vp, ctypes.POINTER(dp)]
        L.apx_conv.argtypes = [vp, vp, i64, vp, i32, i32, ctypes.POINTER(apx_params), vp, vp, vp]
        L.apx_xcorr.argtypes = [vp, vp, i64, vp, i32, i32, ctypes.POINTER(apx_params), vp, vp, vp]
        L.apx_kernel_describe.argtypes = [vp, ctypes.c_char_p, i32]
        pvp, pi64, pi32 = ctypes.POINTER(vp), ctypes.POINTER(i64), ctypes.POINTER(i32)
        L.apx_batch_create.argtypes = [vp, i32, pvp, pi64, pvp, pi32, ctypes.POINTER(apx_params), i32, vp, pvp]
        L.apx_batch_run.argtypes = [vp, vp, vp, vp, vp]
        L.apx_batch_blocks.argtypes = [vp, pi32, pi32, pi32]
        L.apx_batch_describe.argtypes = [vp, ctypes.c_char_p, i32]
        L.apx_batch_destroy.argtypes = [vp]
        L.apx_xcorr_argmax_batch.argtypes = [vp, i32, pvp, pi64, pvp, pi32, ctypes.POINTER(apx_params), vp, vp, vp]
        L.apx_fbank_create.argtypes = [vp, vp, i32, i32, i32, vp, pvp]
        L.apx_fbank_run.argtypes = [vp, vp, vp, i32, i64, i64, vp, i64, vp]
        L.apx_fbank_describe.argtypes = [vp, ctypes.c_char_p, i32]
        L.apx_fbank_destroy.argtypes = [vp]
        L.apx_workspace_bytes.argtypes = []
        L.apx_workspace_bytes.restype = ctypes.c_size_t
        L.apx_run_auto.argtypes = [vp, vp, vp, i64, vp, vp, dp, i32, vp, vp]
        L.apx_run_auto_noalloc.argtypes = [vp, vp, vp, i64, vp, vp, dp, i32, vp]
        L.apx_server_create.argtypes = [vp, ctypes.POINTER(apx_server_config), pvp]
        L.apx_server_submit.argtypes = [vp, ctypes.POINTER(apx_request), ctypes.POINTER(ctypes.c_uint64)]
        L.apx_server_poll.argtypes = [vp, ctypes.POINTER(apx_completion), i32, pi32, i32]
        L.apx_server_drain.argtypes = [vp]
        L.apx_server_stats.argtypes = [vp, ctypes.POINTER(apx_server_counters)]
        L.apx_server_destroy.argtypes = [vp]
        L.apx_server_now.argtypes = []
        L.apx_server_now.restype = dp
        L.apx_fit_marginal.argtypes = [vp, vp, i64, i32, ctypes.POINTER(ctypes.c_double), vp]
        L.apx_tune.argtypes = [vp, vp, i32, i32, i32, ctypes.POINTER(apx_params), i64, vp, ctypes.POINTER(apx_tuned)]
        L.apx_tune_describe.argtypes = [vp, ctypes.c_char_p, i32]
        L.apx_many_create.argtypes = [vp, vp, i32, pvp, pi64, pvp, pvp, vp, pvp]
        L.apx_many_run.argtypes = [vp, vp, vp]
        L.apx_many_describe.argtypes = [vp, ctypes.c_char_p, i32]
        L.apx_many_destroy.argtypes = [vp]
        L.apx_status_str.argtypes = [ctypes.c_int]
        L.apx_status_str.restype = ctypes.c_char_p
        L.apx_last_error.restype = ctypes.c_char_p
        for name in EXPORTS:
            if name not in ("apx_status_str", "apx_last_error", "apx_workspace_bytes", "apx_server_now"):
                getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(st: int):
    if st != APX_OK:
        raise ApxError(st, lib().apx_last_error().decode(errors="replace"))


FFT_AUTO, FFT_BLOCK, FFT_WAVE, FFT_GROUP, FFT_MULTIPASS = 0, 1, 2, 3, 4


def params(mode=APX_FULL_FP32, core=APX_CORE_AUTO, Sq=0, Kq=0, snr_min_db=0.0, calib_db=float("nan"),
           allow_unsafe=False, fft_variant=FFT_AUTO, sigma_s=0.0, sigma_k=0.0) -> apx_params:
    return apx_params(int(mode), int(core), int(Sq), int(Kq), float(snr_min_db), float(calib_db),
                      1 if allow_unsafe else 0, int(fft_variant), float(sigma_s), float(sigma_k))


def _dev_ptr(t, dtype_name: str):
    import torch
    want = {"float32": torch.float32, "float64": torch.float64, "uint8": torch.uint8}[dtype_name]
    if not t.is_cuda or t.dtype != want or not t.is_contiguous():
        raise ValueError(f"expected a contiguous {dtype_name} device tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ------------------------------------------------------------------------------- C ABI mirror
def apx_create(device: int = 0) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().apx_create(device, ctypes.byref(h)))
    return h


def apx_destroy(ctx):
    _check(lib().apx_destroy(ctx))


def apx_geometry(L: int, N: int, W_block: int):
    """(N_odd, W, P) of the overlap-save partition."""
    no, w, p = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int64()
    _check(lib().apx_geometry(L, N, W_block, ctypes.byref(no), ctypes.byref(w), ctypes.byref(p)))
    return no.value, w.value, p.value


def apx_kernel_create(ctx, k, W_block: int, prm: apx_params, op: int = APX_CONV, stream=None):
    h = ctypes.c_void_p()
    _check(lib().apx_kernel_create(ctx, _dev_ptr(k, "float32"), k.numel(), op, W_block, ctypes.byref(prm),
                                   _stream(stream), ctypes.byref(h)))
    return h


def apx_kernel_destroy(kern):
    _check(lib().apx_kernel_destroy(kern))


def apx_run(ctx, kern, s, out, info=None, stream=None):
    _check(lib().apx_run(ctx, kern, _dev_ptr(s, "float32"), s.numel(), _dev_ptr(out, "float32"),
                         None if info is None else _dev_ptr(info, "uint8"), _stream(stream)))


def apx_debug_fields(ctx, kern, s, fields, stream=None):
    _check(lib().apx_debug_fields(ctx, kern, _dev_ptr(s, "float32"), s.numel(), _dev_ptr(fields, "float64"),
                                  _stream(stream)))


def apx_calibrate(ctx, kern, s, block: int = 0, Q: int = 8, stream=None) -> float:
    off = ctypes.c_double()
    _check(lib().apx_calibrate(ctx, kern, _dev_ptr(s, "float32"), s.numel(), block, Q, _stream(stream),
                               ctypes.byref(off)))
    return off.value


def apx_fit_marginal(ctx, x, model: int, stream=None):
    """(scale, shape, sigma, samples used) of the marginal fit of the device samples x."""
    out = (ctypes.c_double * 4)()
    _check(lib().apx_fit_marginal(ctx, _dev_ptr(x, "float32"), x.numel(), int(model), out, _stream(stream)))
    return tuple(out)


def apx_workspace_bytes() -> int:
    return int(lib().apx_workspace_bytes())


def apx_run_auto(ctx, kern, s, out, snr_min_db: float, calib_block: int, workspace, info=None, stream=None):
    _check(lib().apx_run_auto(ctx, kern, _dev_ptr(s, "float32"), s.numel(), _dev_ptr(out, "float32"),
                              None if info is None else _dev_ptr(info, "uint8"), float(snr_min_db), int(calib_block),
                              _dev_ptr(workspace, "uint8"), _stream(stream)))


def apx_run_auto_noalloc(ctx, kern, s, out, snr_min_db: float, calib_block: int, info=None, stream=None):
    _check(lib().apx_run_auto_noalloc(ctx, kern, _dev_ptr(s, "float32"), s.numel(), _dev_ptr(out, "float32"),
                                      None if info is None else _dev_ptr(info, "uint8"), float(snr_min_db),
                                      int(calib_block), _stream(stream)))


def apx_kernel_describe(kern) -> str:
    buf = ctypes.create_string_buffer(512)
    _check(lib().apx_kernel_describe(kern, buf, 512))
    return buf.value.decode()


def apx_conv(ctx, s, k, W_block: int, prm: apx_params, out, info=None, stream=None):
    _check(lib().apx_conv(ctx, _dev_ptr(s, "float32"), s.numel(), _dev_ptr(k, "float32"), k.numel(), W_block,
                          ctypes.byref(prm), _dev_ptr(out, "float32"),
                          None if info is None else _dev_ptr(info, "uint8"), _stream(stream)))


def apx_xcorr(ctx, s, k, W_block: int, prm: apx_params, out, info=None, stream=None):
    _check(lib().apx_xcorr(ctx, _dev_ptr(s, "float32"), s.numel(), _dev_ptr(k, "float32"), k.numel(), W_block,
                           ctypes.byref(prm), _dev_ptr(out, "float32"),
                           None if info is None else _dev_ptr(info, "uint8"), _stream(stream)))


def _pair_arrays(refs, tmpls):
    n = len(refs)
    if len(tmpls) != n:
        raise ValueError("one template per reference")
    rp = (ctypes.c_void_p * n)(*[_dev_ptr(r, "float32").value for r in refs])
    tp = (ctypes.c_void_p * n)(*[_dev_ptr(k, "float32").value for k in tmpls])
    L = (ctypes.c_int64 * n)(*[r.numel() for r in refs])
    N = (ctypes.c_int32 * n)(*[k.numel() for k in tmpls])
    return n, rp, L, tp, N


def apx_batch_create(ctx, refs, tmpls, prm: apx_params, logW: int = 0, stream=None):
    n, rp, L, tp, N = _pair_arrays(refs, tmpls)
    h = ctypes.c_void_p()
    _check(lib().apx_batch_create(ctx, n, rp, L, tp, N, ctypes.byref(prm), logW, _stream(stream), ctypes.byref(h)))
    return h


def apx_batch_run(ctx, batch, lag_out, val_out, stream=None):
    import torch
    if not (lag_out.is_cuda and lag_out.dtype == torch.int64 and lag_out.is_contiguous()):
        raise ValueError("lag_out must be a contiguous int64 device tensor")
    _check(lib().apx_batch_run(ctx, batch, ctypes.c_void_p(lag_out.data_ptr()), _dev_ptr(val_out, "float32"),
                               _stream(stream)))


def apx_batch_blocks(batch, n: int):
    wb = (ctypes.c_int32 * n)()
    lw, ni = ctypes.c_int32(), ctypes.c_int32()
    _check(lib().apx_batch_blocks(batch, wb, ctypes.byref(lw), ctypes.byref(ni)))
    return np.array(wb[:], dtype=np.int64), lw.value, ni.value


def apx_batch_describe(batch) -> str:
    buf = ctypes.create_string_buffer(4096)
    _check(lib().apx_batch_describe(batch, buf, 4096))
    return buf.value.decode()


def apx_batch_destroy(batch):
    _check(lib().apx_batch_destroy(batch))


def apx_xcorr_argmax_batch(ctx, refs, tmpls, prm: apx_params, lag_out, val_out, stream=None):
    import torch
    n, rp, L, tp, N = _pair_arrays(refs, tmpls)
    if not (lag_out.is_cuda and lag_out.dtype == torch.int64 and lag_out.is_contiguous()):
        raise ValueError("lag_out must be a contiguous int64 device tensor")
    _check(lib().apx_xcorr_argmax_batch(ctx, n, rp, L, tp, N, ctypes.byref(prm), ctypes.c_void_p(lag_out.data_ptr()),
                                        _dev_ptr(val_out, "float32"), _stream(stream)))


def apx_tune(ctx, k, W_block: int, prm: apx_params, op: int = APX_CONV, L_hint: int = 0, stream=None) -> dict:
    """Time every core / FFT implementation (and block size when W_block = 0) for taps k (device
    tensor) on a signal of L_hint samples and record the fastest in the context's table."""
    t = apx_tuned()
    _check(lib().apx_tune(ctx, _dev_ptr(k, "float32"), k.numel(), int(op), int(W_block), ctypes.byref(prm),
                          int(L_hint), _stream(stream), ctypes.byref(t)))
    return {"core": t.core, "fft_variant": t.fft_variant, "W_block": t.W_block, "tile": t.tile,
            "ps_per_output": t.ps_per_output}


def apx_tune_describe(ctx) -> str:
    buf = ctypes.create_string_buffer(16384)
    _check(lib().apx_tune_describe(ctx, buf, 16384))
    return buf.value.decode()


def apx_many_create(ctx, kern, signals, outs, infos=None, stream=None):
    """signals / outs / infos: lists of device tensors (infos entries may be None)."""
    n = len(signals)
    vp = ctypes.c_void_p
    sp = (vp * n)(*[_dev_ptr(x, "float32") for x in signals])
    op = (vp * n)(*[_dev_ptr(x, "float32") for x in outs])
    Ls = (ctypes.c_int64 * n)(*[int(x.numel()) for x in signals])
    ip = None
    if infos is not None:
        ip = (vp * n)(*[None if x is None else x.data_ptr() for x in infos])
    h = vp()
    _check(lib().apx_many_create(ctx, kern, n, sp, Ls, op, ip, _stream(stream), ctypes.byref(h)))
    return h


def apx_many_run(ctx, many, stream=None):
    _check(lib().apx_many_run(ctx, many, _stream(stream)))


def apx_many_describe(many) -> str:
    buf = ctypes.create_string_buffer(1024)
    _check(lib().apx_many_describe(many, buf, 1024))
    return buf.value.decode()


def apx_many_destroy(many):
    _check(lib().apx_many_destroy(many))


def apx_fbank_create(ctx, h, prec: int = APX_FB_F16X3, stream=None):
    """h: (F, N) contiguous FP32 device tensor."""
    if h.dim() != 2:
        raise ValueError("h must be (F, N)")
    out = ctypes.c_void_p()
    _check(lib().apx_fbank_create(ctx, _dev_ptr(h, "float32"), h.shape[0], h.shape[1], prec, _stream(stream),
                                  ctypes.byref(out)))
    return out


def apx_fbank_run(ctx, fb, x, L: int, y, stream=None):
    """x: (C, ldx) FP32 device tensor; y: (C * F, ldy) FP32 device tensor."""
    if x.dim() != 2 or y.dim() != 2:
        raise ValueError("x must be (C, ldx) and y (C*F, ldy)")
    _check(lib().apx_fbank_run(ctx, fb, _dev_ptr(x, "float32"), x.shape[0], L, x.shape[1], _dev_ptr(y, "float32"),
                               y.shape[1], _stream(stream)))


def apx_fbank_describe(fb) -> str:
    buf = ctypes.create_string_buffer(512)
    _check(lib().apx_fbank_describe(fb, buf, 512))
    return buf.value.decode()


def apx_fbank_destroy(fb):
    _check(lib().apx_fbank_destroy(fb))


# ------------------------------------------------------------------------------- conveniences
class Context:
    def __init__(self, device: int = 0):
        self.device = device
        self.h = apx_create(device)

    def close(self):
        if self.h:
            apx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Kernel:
    """A prepared kernel (companded / packed taps and spectra resident on the device)."""

    def __init__(self, ctx: Context, k, W_block: int, mode=APX_FULL_FP32, core=APX_CORE_AUTO, Sq=0, Kq=0,
                 snr_min_db=0.0, calib_db=float("nan"), op=APX_CONV, allow_unsafe=False, fft_variant=FFT_AUTO,
                 sigma_s=0.0, sigma_k=0.0, stream=None):
        self.ctx = ctx
        self.N = int(k.numel())
        self.W_block = W_block
        self.op = op
        self.prm = params(mode, core, Sq, Kq, snr_min_db, calib_db, allow_unsafe, fft_variant, sigma_s, sigma_k)
        self.h = apx_kernel_create(ctx.h, k, W_block, self.prm, op, stream)
        if W_block == 0:  # the block size the library chose (tuned, or its default rule)
            import re
            self.W_block = int(re.search(r"W_block=(\d+)", self.describe()).group(1))

    def geometry(self, L: int):
        return apx_geometry(L, self.N, self.W_block)

    def run(self, s, out=None, info: bool = False, stream=None):
        import torch
        if out is None:
            out = torch.empty(s.numel() + self.N - 1, dtype=torch.float32, device=s.device)
        inf = None
        if info:
            P = self.geometry(s.numel())[2]
            inf = torch.empty(P * BLOCK_INFO_DTYPE.itemsize, dtype=torch.uint8, device=s.device)
        apx_run(self.ctx.h, self.h, s, out, inf, stream)
        return (out, inf) if info else out

    def fields(self, s, stream=None):
        import torch
        f = torch.empty(s.numel() + self.N - 1, dtype=torch.float64, device=s.device)
        apx_debug_fields(self.ctx.h, self.h, s, f, stream)
        return f

    def describe(self) -> str:
        return apx_kernel_describe(self.h)

    def run_auto(self, s, snr_min_db: float, out=None, calib_block: int = 0, workspace=None, stream=None):
        """APX_AUTO_SNR run with this call's target and a calibration measured on the device on
        block `calib_block` of s (apx_run_auto)."""
        import torch
        if out is None:
            out = torch.empty(s.numel() + self.N - 1, dtype=torch.float32, device=s.device)
        if workspace is None:
            workspace = torch.empty(apx_workspace_bytes(), dtype=torch.uint8, device=s.device)
        apx_run_auto(self.ctx.h, self.h, s, out, snr_min_db, calib_block, workspace, None, stream)
        return out

    def calibrate(self, s, block: int = 0, Q: int = 8, stream=None) -> float:
        return apx_calibrate(self.ctx.h, self.h, s, block, Q, stream)

    def close(self):
        if self.h:
            apx_kernel_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Many:
    """Many signals through one prepared kernel in one launch (apx_many_*).  The signal and
    output tensors are kept referenced for the handle's lifetime."""

    def __init__(self, kernel: "Kernel", signals, outs=None, info: bool = False, stream=None):
        import torch
        self.ctx = kernel.ctx
        self.kernel = kernel
        self.signals = list(signals)
        if outs is None:
            outs = [torch.empty(x.numel() + kernel.N - 1, dtype=torch.float32, device=x.device) for x in self.signals]
        self.outs = list(outs)
        self.infos = None
        if info:
            self.infos = [torch.empty(kernel.geometry(x.numel())[2] * BLOCK_INFO_DTYPE.itemsize, dtype=torch.uint8,
                                      device=x.device) for x in self.signals]
        self.h = apx_many_create(self.ctx.h, kernel.h, self.signals, self.outs, self.infos, stream)

    def run(self, stream=None):
        apx_many_run(self.ctx.h, self.h, stream)
        return self.outs

    def describe(self) -> str:
        return apx_many_describe(self.h)

    def close(self):
        if self.h:
            apx_many_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def block_info(info_tensor) -> np.ndarray:
    """Device block-report bytes -> numpy structured array (synchronizes)."""
    return np.frombuffer(info_tensor.cpu().numpy().tobytes(), dtype=BLOCK_INFO_DTYPE)


class Batch:
    """Batched cross-correlation matching of (reference, template) pairs in one persistent launch.
    Keeps the tensors alive: the library holds their device pointers."""

    def __init__(self, ctx: Context, refs, tmpls, mode=APX_SYM, Sq=0, Kq=0, allow_unsafe=False, logW: int = 0,
                 stream=None):
        self.ctx = ctx
        self.refs, self.tmpls = list(refs), list(tmpls)
        self.n = len(self.refs)
        self.prm = params(mode, APX_CORE_FFT, Sq, Kq, 0.0, float("nan"), allow_unsafe)
        self.h = apx_batch_create(ctx.h, self.refs, self.tmpls, self.prm, logW, stream)

    def run(self, lag=None, val=None, stream=None):
        import torch
        dev = self.refs[0].device
        if lag is None:
            lag = torch.empty(self.n, dtype=torch.int64, device=dev)
        if val is None:
            val = torch.empty(self.n, dtype=torch.float32, device=dev)
        apx_batch_run(self.ctx.h, self.h, lag, val, stream)
        return lag, val

    def blocks(self):
        """(W_block per pair, log2 FFT length, work items)."""
        return apx_batch_blocks(self.h, self.n)

    def describe(self) -> str:
        return apx_batch_describe(self.h)

    def close(self):
        if self.h:
            apx_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FilterBank:
    """F <= 32 filters of N <= 512 taps on split-precision matrix cores (see apx_fbank_*)."""

    def __init__(self, ctx: Context, h, prec=APX_FB_F16X3, stream=None):
        self.ctx = ctx
        self.F, self.N = int(h.shape[0]), int(h.shape[1])
        self.h = apx_fbank_create(ctx.h, h, prec, stream)

    def run(self, x, y=None, L: Optional[int] = None, ldy: Optional[int] = None, stream=None):
        """x: (C, ldx); returns y viewed as (C, F, ldy) with L + N - 1 valid samples per row."""
        import torch
        C = x.shape[0]
        L = x.shape[1] if L is None else L
        Lout = L + self.N - 1
        if y is None:
            ldy = Lout if ldy is None else ldy
            y = torch.empty(C * self.F, ldy, dtype=torch.float32, device=x.device)
        y2 = y.view(C * self.F, -1)
        apx_fbank_run(self.ctx.h, self.h, x, L, y2, stream)
        return y2.view(C, self.F, -1)

    def describe(self) -> str:
        return apx_fbank_describe(self.h)

    def close(self):
        if self.h:
            apx_fbank_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _host_ptr(a):
    """Host address of a contiguous float32 numpy array or CPU tensor."""
    if isinstance(a, np.ndarray):
        if a.dtype != np.float32 or not a.flags["C_CONTIGUOUS"]:
            raise ValueError("expected a contiguous float32 array")
        return a.ctypes.data
    if a.is_cuda or not a.is_contiguous() or str(a.dtype) != "torch.float32":
        raise ValueError("expected a contiguous float32 CPU tensor")
    return a.data_ptr()


class Server:
    """Request loop with admission by HBM budget and resident kernels (apx_server_*).  Keeps the
    host buffers of every outstanding request alive until its completion is polled."""

    def __init__(self, ctx: Context, hbm_budget: int = 32 << 30, n_streams: int = 8, max_inflight: int = 64):
        self.ctx = ctx
        cfg = apx_server_config(int(hbm_budget), int(n_streams), int(max_inflight))
        h = ctypes.c_void_p()
        _check(lib().apx_server_create(ctx.h, ctypes.byref(cfg), ctypes.byref(h)))
        self.h = h
        self.keep = {}
        self._buf = (apx_completion * 1024)()

    @staticmethod
    def now() -> float:
        return float(lib().apx_server_now())

    def submit(self, key: int, k, s, r_out, snr_min_db: float = 40.0, op: int = APX_CONV, mode: int = APX_AUTO_SNR,
               W_block: int = 0, L: Optional[int] = None) -> int:
        """k: N taps, s: input (first L samples used), r_out: L + N - 1 outputs; host memory
        (numpy float32 or CPU tensors, pinned ones overlap their copies)."""
        N = int(k.shape[0])
        L = int(s.shape[0]) if L is None else int(L)
        if r_out.shape[0] < L + N - 1:
            raise ValueError("r_out too short")
        req = apx_request(int(key), _host_ptr(k), N, int(op), _host_ptr(s), L, _host_ptr(r_out), float(snr_min_db),
                          int(W_block), int(mode))
        t = ctypes.c_uint64()
        st = lib().apx_server_submit(self.h, ctypes.byref(req), ctypes.byref(t))
        if st != APX_OK:
            raise ApxError(st, "request refused")
        self.keep[t.value] = (k, s, r_out)
        return t.value

    def poll(self, wait_ms: int = 0, max_n: int = 1024):
        n = ctypes.c_int32()
        _check(lib().apx_server_poll(self.h, self._buf, min(max_n, 1024), ctypes.byref(n), int(wait_ms)))
        out = []
        for i in range(n.value):
            c = self._buf[i]
            out.append({"ticket": c.ticket, "status": c.status, "core": c.core, "W_block": c.W_block, "N": c.N,
                        "L": c.L, "t_submit": c.t_submit, "t_admit": c.t_admit, "t_done": c.t_done})
            self.keep.pop(c.ticket, None)
        return out

    def drain(self):
        _check(lib().apx_server_drain(self.h))

    def stats(self) -> dict:
        c = apx_server_counters()
        _check(lib().apx_server_stats(self.h, ctypes.byref(c)))
        return {n: getattr(c, n) for n, _ in apx_server_counters._fields_ if n != "pad"}

    def close(self):
        if self.h:
            _check(lib().apx_server_destroy(self.h))
            self.h = None
            self.keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
