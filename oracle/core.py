"""Oracle for packed approximate overlap-save convolution -- TEST INFRASTRUCTURE ONLY.

Only tests/, __graft_entry__.smoke() and the CPU-baseline leg of bench.py may import
this module.  It imports nothing from the product package and the product never
imports it.  Everything is FP64 (or exact int64) on the CPU.

Paper: Anam & Andreopoulos, "Throughput Scaling Of Convolution For Error-Tolerant
Multimedia Applications" (arXiv 1201.3018).

Two levels live here.

* Plain definitions -- what the packed method computes exactly whenever its unpacking
  is error-free (Table 1, "Companding range"):
    conv_direct            eq. (1), FP64
    Partition              overlap-save blocks of Section II / Section III, placement eq. (17)
    compand                eq. (2) with c = Q / ||x||_inf
    conv_blocked           per-block integer convolution of companded data, eq. (16)
* The paper's own steps, in its order, used to show that the method reaches the plain
  definition inside the Table 1 bounds:
    pack_sym_signal/kernel eqs. (4), (5), (6)
    unpack_sym             eqs. (11)-(15)
    pack_asym / unpack_asym eqs. (7), (8)
    conv_blocked_paper     Section III.A-C end to end, time-domain or FFT core
* Distortion model and selection: snr_model_db (eqs. 18, 19), select_mode and
  calibrate (Section IV.D).

Readings taken where the paper is silent, ambiguous or garbled (each one is restated at
the function that uses it):
  R1  eq. (5) as printed puts eps^-1 on the odd taps; with (9), (14), (15) the decoded
      fields are then not convolution outputs.  For convolution the packed kernel is
      k~[2n+1] + eps^-1 k~[2n] (eps^-1 on the even taps).
  R2  even N: one zero tap is appended (Section III opening); the output keeps L+N-1 samples.
  R3  [[.]] is round-half-to-even; c*x is one FP64 multiply of the FP32 sample widened.
  R4  block w covers s_in[Ww-2, Ww-2+W_block) for w >= 1 and s_in[0, W_block) for w = 0;
      P = ceil(L/W); block 0 keeps its first W+N-1 outputs, block w keeps local outputs
      [N+1, N+1+W) (this is eq. 17 with W_start from eq. 10).
  R6  eps = fl(1/(2 R_max)) but eps^-1 is the exact integer 2 R_max.
  R7  the system constant u_sys eps^-1 in R_safe becomes a half eps-digit, eps/2, and
      R_safe is added as (R eps + eps/2) followed by the exact integer R (1 + 2R).
  R9  asymmetric packing: part stride T = ceil(W/M); block w >= 1 packs parts at offsets
      2 + qT, block 0 at offsets qT (its part 0 is valid from the first word); unpacking
      takes balanced base-2R digits one after the other.
  R11 Table 1's SNR expression swaps the roles of S_q and K_q relative to eqs. (18), (19);
      the model here is eqs. (18), (19) with sigma_v = ||x||_inf / (Q sqrt 12).
  R12 sigma is the square root of the (uncentred) second moment of the block or kernel.
  R13 S_q = K_q = floor(sqrt(bound / N)) is "the maximum S_q and K_q" a packing allows.
  R14 calibration: offset = measured - model SNR at S_q = K_q = 8 on one block.
  R15 candidate order for the SNR-driven choice: symmetric, asymmetric M=2, full precision.
"""
from __future__ import annotations

import ctypes
import math
import os
from dataclasses import dataclass, field
from typing import List, Optional, Sequence

import numpy as np

# Table 1, "Companding range" row: error-free packing limits under FP64.
SYM_BOUND = 97667
ASYM2_BOUND = 43165096
ASYM3_BOUND = 97667

FULL, SYM, ASYM2, ASYM3 = "full", "sym", "asym2", "asym3"
PACKED_MODES = (SYM, ASYM2, ASYM3)
BOUND = {SYM: SYM_BOUND, ASYM2: ASYM2_BOUND, ASYM3: ASYM3_BOUND}

# ----------------------------------------------------------------------------------------
# C loops
# ----------------------------------------------------------------------------------------
_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


def _lib():
    global _LIB
    if _LIB is None:
        from . import build as _b
        path = os.path.join(_HERE, "liborc.so")
        if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_b.SRC):
            _b.build()
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER
        i64 = ctypes.c_int64
        lib.orc_conv_f64.argtypes = [P(ctypes.c_double), i64, P(ctypes.c_double), i64, P(ctypes.c_double)]
        lib.orc_conv_i64_range.argtypes = [P(i64), i64, P(i64), i64, i64, i64, P(i64)]
        lib.orc_conv_i64_blocks.argtypes = [P(i64), i64, i64, P(i64), i64, P(i64), P(i64), P(i64), P(i64)]
        lib.orc_num_threads.restype = ctypes.c_int
        _LIB = lib
    return _LIB


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def num_threads() -> int:
    return int(_lib().orc_num_threads())


# ----------------------------------------------------------------------------------------
# Eq. (1): linear convolution
# ----------------------------------------------------------------------------------------
def conv_direct(s, k) -> np.ndarray:
    """r[m] = sum_n s[m-n] k[n], 0 <= m < L+N-1, in FP64 (eq. 1)."""
    s = np.ascontiguousarray(s, dtype=np.float64)
    k = np.ascontiguousarray(k, dtype=np.float64)
    L, N = s.size, k.size
    r = np.empty(L + N - 1, dtype=np.float64)
    _lib().orc_conv_f64(_p(s, ctypes.c_double), L, _p(k, ctypes.c_double), N, _p(r, ctypes.c_double))
    return r


def conv_int_range(sq, kq, m0: int, m1: int) -> np.ndarray:
    """Exact int64 convolution outputs m in [m0, m1) of integer sequences (eq. 1 on s~, k~)."""
    sq = np.ascontiguousarray(sq, dtype=np.int64)
    kq = np.ascontiguousarray(kq, dtype=np.int64)
    out = np.empty(max(0, m1 - m0), dtype=np.int64)
    if out.size:
        _lib().orc_conv_i64_range(_p(sq, ctypes.c_int64), sq.size, _p(kq, ctypes.c_int64), kq.size,
                                  m0, m1, _p(out, ctypes.c_int64))
    return out


def xcorr_direct(s, k) -> np.ndarray:
    """Cross-correlation c[l] = sum_n s[l+n] k[n] for l in [-(N-1), L-1], returned at index
    l + N - 1 (textbook definition, FP64, plain loops; used for the applications of Section IV
    where correlation replaces the convolution call)."""
    s = np.asarray(s, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    L, N = s.size, k.size
    out = np.zeros(L + N - 1, dtype=np.float64)
    for lag in range(-(N - 1), L):
        acc = 0.0
        for n in range(N):
            i = lag + n
            if 0 <= i < L:
                acc += s[i] * k[n]
        out[lag + N - 1] = acc
    return out


def xcorr(s, k) -> np.ndarray:
    """Cross-correlation through the convolution of eq. (1) with the time-reversed kernel."""
    return conv_direct(s, np.asarray(k, dtype=np.float64)[::-1])


def argmax_lag(c: np.ndarray, N: int):
    """Largest correlation value and its lag l = index - (N-1); ties go to the smallest lag."""
    i = int(np.argmax(c))
    return i - (N - 1), c[i]


def argmax_lag_finite(c: np.ndarray, N: int):
    """argmax_lag over the entries that are not NaN (-0 equals +0, ties to the smallest lag);
    (None, nan) when every entry is NaN.  The matching step of the correlation applications
    (Section IV.B) picks the lag of the largest correlation."""
    c = np.asarray(c)
    ok = np.nonzero(~np.isnan(c))[0]
    if ok.size == 0:
        return None, float("nan")
    j = int(np.argmax(c[ok]))
    return int(ok[j]) - (N - 1), c[ok[j]]


# ----------------------------------------------------------------------------------------
# Overlap-save partition (Section II, Section III opening, eqs. 10 and 17)
# ----------------------------------------------------------------------------------------
@dataclass
class Partition:
    L: int
    N: int          # kernel taps as given
    N_odd: int      # taps after padding an even kernel with one zero (R2)
    W_block: int
    W: int          # outputs per block, W_block = W + N + 1
    P: int          # number of blocks
    starts: np.ndarray

    @property
    def out_len(self) -> int:
        return self.L + self.N - 1

    def window(self, s, w: int) -> np.ndarray:
        """The block s of Section II: W_block samples from start_w, zero past the input end."""
        b = np.zeros(self.W_block, dtype=np.asarray(s).dtype)
        a = int(self.starts[w])
        e = min(a + self.W_block, self.L)
        if e > a:
            b[: e - a] = s[a:e]
        return b

    def keep(self, w: int):
        """Local output range [j_lo, j_hi) of block w's convolution kept by eq. (17), and the
        r_out index of j_lo.  The range is clipped so that it ends at the output length."""
        N = self.N_odd
        if w == 0:
            j_lo, j_hi, o = 0, self.W + N - 1, 0
        else:
            j_lo, j_hi, o = N + 1, N + 1 + self.W, N - 1 + self.W * w
        j_hi = min(j_hi, j_lo + max(0, self.out_len - o))
        return j_lo, j_hi, o


def partition(L: int, N: int, W_block: int) -> Partition:
    """Blocks of W_block = W + N + 1 samples producing W outputs each, W >= 2N and even
    (Section III opening).  Block w >= 1 starts at W w - 2 so that eq. (17) places its
    local outputs [N+1, N+1+W) at r_out[N-1+Ww ...] (reading R4)."""
    if L < 1 or N < 1 or N > L:
        raise ValueError("need 1 <= N <= L")
    N_odd = N if N % 2 == 1 else N + 1
    W = W_block - N_odd - 1
    if W < 2 * N_odd or W % 2 != 0:
        raise ValueError(f"W = W_block - N - 1 = {W} must be even and >= 2N = {2 * N_odd}")
    P = max(1, -(-L // W))
    starts = np.array([0] + [W * w - 2 for w in range(1, P)], dtype=np.int64)
    return Partition(L, N, N_odd, W_block, W, P, starts)


def pad_kernel(k) -> np.ndarray:
    """Reading R2: an even-length kernel gets one trailing zero tap."""
    k = np.asarray(k)
    if k.size % 2 == 0:
        k = np.concatenate([k, np.zeros(1, dtype=k.dtype)])
    return k


# ----------------------------------------------------------------------------------------
# Eqs. (2), (3), (6): companding, range, packing coefficient
# ----------------------------------------------------------------------------------------
def compand(x, Q: int):
    """Uniform companding, eq. (2): c = Q / ||x||_inf, x~ = [[c x]] (round half to even,
    reading R3).  An all-zero x gives c = 0 and x~ = 0."""
    x = np.asarray(x, dtype=np.float64)
    m = float(np.max(np.abs(x))) if x.size else 0.0
    if m == 0.0:
        return 0.0, np.zeros(x.size, dtype=np.int64)
    c = float(Q) / m
    return c, np.rint(c * x).astype(np.int64)


def r_max(N: int, S: int, K: int) -> int:
    """Companding range, eq. (3): R_max = [[N S_q K_q]]."""
    return int(N) * int(S) * int(K)


def epsilon(R: int) -> float:
    """Packing coefficient, eq. (6): eps = (2 R_max)^-1 (reading R6: eps^-1 stays the integer 2R)."""
    return 1.0 / (2.0 * R)


def max_q(mode: str, N_odd: int) -> int:
    """Reading R13: largest S_q = K_q with N S_q K_q inside the mode's Table 1 bound."""
    return math.isqrt(BOUND[mode] // N_odd)


# ----------------------------------------------------------------------------------------
# Plain definition of the per-block quantized convolution (eqs. 2, 16, 17)
# ----------------------------------------------------------------------------------------
@dataclass
class BlockParams:
    mode: str
    S: int = 0
    K: int = 0
    cs: float = 0.0
    smax: float = 0.0
    rms: float = 0.0
    snr_pred_db: float = math.inf


def block_stats(b) -> tuple:
    """||b||_inf and the root of the uncentred second moment (reading R12)."""
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(b))), float(math.sqrt(np.sum(b * b) / b.size))


def kernel_stats(k) -> tuple:
    k = np.asarray(k, dtype=np.float64)
    return float(np.max(np.abs(k))), float(math.sqrt(np.sum(k * k) / k.size))


def conv_blocked(s, k, W_block: int, params: Sequence[BlockParams], out_dtype=np.float32,
                 return_fields: bool = False):
    """Overlap-save convolution with per-block companding (plain definition).

    For each block w with window b (reading R4):
      packed modes: c_s = S/||b||_inf, s~ = [[c_s b]], k~ = [[c_k k]], r~ = s~ * k~ in exact
                    int64, r = (c_s c_k)^-1 r~ in FP64 (eq. 16: the inverse is formed once per
                    block and multiplies r~), cast to out_dtype;
      full:         r = b * k in FP64 (eq. 1 on the block);
    kept outputs are placed by eq. (17).  A block whose window holds a NaN or infinity gives
    NaN outputs (the companding factor is undefined there).  With return_fields, also returns the int64 r~ at
    every output position (0 for full-precision blocks) and the per-block c_s.
    """
    s = np.asarray(s)
    part = partition(s.size, np.asarray(k).size, W_block)
    kp = pad_kernel(np.asarray(k, dtype=np.float64))
    N = part.N_odd
    out = np.zeros(part.out_len, dtype=np.float64)
    fields = np.zeros(part.out_len, dtype=np.int64) if return_fields else None
    cks = {}
    packed_ws = [w for w in range(part.P) if params[w].mode != FULL]
    full_ws = [w for w in range(part.P) if params[w].mode == FULL]

    # integer blocks, grouped by K (the kernel is companded once per K, Section IV "Initialization")
    by_k = {}
    for w in packed_ws:
        by_k.setdefault(params[w].K, []).append(w)
    for K, ws in by_k.items():
        ck, kq = compand(kp, K)
        cks[K] = ck
        wins = np.zeros((len(ws), W_block), dtype=np.int64)
        css = np.zeros(len(ws))
        m0 = np.zeros(len(ws), dtype=np.int64)
        m1 = np.zeros(len(ws), dtype=np.int64)
        off = np.zeros(len(ws), dtype=np.int64)
        pos = 0
        for i, w in enumerate(ws):
            win = part.window(s, w)
            if not np.all(np.isfinite(win)):
                win = np.zeros_like(win)       # outputs set to NaN below
            cs, sq = compand(win, params[w].S)
            css[i] = cs
            params[w].cs = cs
            wins[i] = sq
            j_lo, j_hi, _ = part.keep(w)
            m0[i], m1[i], off[i] = j_lo, j_hi, pos
            pos += max(0, j_hi - j_lo)
        rq = np.empty(pos, dtype=np.int64)
        _lib().orc_conv_i64_blocks(_p(wins, ctypes.c_int64), len(ws), W_block, _p(kq, ctypes.c_int64),
                                   N, _p(m0, ctypes.c_int64), _p(m1, ctypes.c_int64), _p(off, ctypes.c_int64),
                                   _p(rq, ctypes.c_int64))
        for i, w in enumerate(ws):
            j_lo, j_hi, o = part.keep(w)
            n = j_hi - j_lo
            seg = rq[off[i]: off[i] + n]
            if not np.all(np.isfinite(part.window(s, w))):
                out[o: o + n] = np.nan
            elif css[i] == 0.0 or ck == 0.0:
                out[o: o + n] = 0.0
            else:
                out[o: o + n] = (1.0 / (css[i] * ck)) * seg.astype(np.float64)   # eq. (16)
            if return_fields:
                fields[o: o + n] = seg
    for w in full_ws:
        j_lo, j_hi, o = part.keep(w)
        win = part.window(s, w)
        if not np.all(np.isfinite(win)):
            out[o: o + (j_hi - j_lo)] = np.nan
            continue
        r = conv_direct(win, kp)
        out[o: o + (j_hi - j_lo)] = r[j_lo:j_hi]
    out = out.astype(out_dtype)
    if return_fields:
        return out, fields, cks
    return out


def fixed_params(s, k, W_block: int, mode: str, S: int, K: int) -> List[BlockParams]:
    """Every block in one mode at fixed S_q, K_q (Section IV.A-C usage)."""
    part = partition(np.asarray(s).size, np.asarray(k).size, W_block)
    ps = []
    for w in range(part.P):
        smax, rms = block_stats(part.window(s, w))
        ps.append(BlockParams(mode, S if mode != FULL else 0, K if mode != FULL else 0, 0.0, smax, rms))
    return ps


# ----------------------------------------------------------------------------------------
# Distortion model and SNR-constrained selection (eqs. 18, 19; Section IV.D)
# ----------------------------------------------------------------------------------------
def snr_model_db(sigma_s: float, smax: float, sigma_k: float, kmax: float, S: int, K: int,
                 N: int = 1) -> float:
    """Expected SNR of the companded convolution against full precision.

    sigma_v = ||x||_inf / (Q sqrt 12) for uniform rounding noise (text after eq. 19);
    D_r = N [(sigma_s sigma_vk)^2 + (sigma_k sigma_vs)^2 + (sigma_vk sigma_vs)^2]  (eq. 18);
    SNR = 10 log10(N (sigma_s sigma_k)^2 / D_r)                                     (eq. 19).
    Reading R11: this is the form derived from (18), (19), not Table 1's printed one.
    A zero signal or kernel is reproduced exactly: +inf.
    """
    if sigma_s == 0.0 or sigma_k == 0.0:
        return math.inf
    svs = smax / (S * math.sqrt(12.0))
    svk = kmax / (K * math.sqrt(12.0))
    D = N * ((sigma_s * svk) ** 2 + (sigma_k * svs) ** 2 + (svk * svs) ** 2)
    return 10.0 * math.log10(N * (sigma_s * sigma_k) ** 2 / D)


def select_mode(smax: float, rms: float, kmax: float, krms: float, N_odd: int, target_db: float,
                calib_db: float = 0.0, candidates=(SYM, ASYM2)) -> BlockParams:
    """Section IV.D: the first packing (fastest first, reading R15) whose calibrated model SNR
    at its maximum S_q = K_q (reading R13) meets the target; otherwise full precision."""
    for mode in candidates:
        q = max_q(mode, N_odd)
        if q < 1:
            continue
        snr = snr_model_db(rms, smax, krms, kmax, q, q) + calib_db
        if snr >= target_db:
            return BlockParams(mode, q, q, 0.0, smax, rms, snr)
    return BlockParams(FULL, 0, 0, 0.0, smax, rms, math.inf)


def auto_params(s, k, W_block: int, target_db: float, calib_db: float = 0.0,
                candidates=(SYM, ASYM2)) -> List[BlockParams]:
    part = partition(np.asarray(s).size, np.asarray(k).size, W_block)
    kmax, krms = kernel_stats(k)
    ps = []
    for w in range(part.P):
        smax, rms = block_stats(part.window(s, w))
        ps.append(select_mode(smax, rms, kmax, krms, part.N_odd, target_db, calib_db, candidates))
    return ps


def measured_snr_db(r, r_ref) -> float:
    """10 log10(sum r_ref^2 / sum (r - r_ref)^2), both FP64."""
    r = np.asarray(r, dtype=np.float64)
    r_ref = np.asarray(r_ref, dtype=np.float64)
    e = float(np.sum((r - r_ref) ** 2))
    p = float(np.sum(r_ref ** 2))
    if e == 0.0:
        return math.inf
    return 10.0 * math.log10(p / e)


def block_snr_db(s, k, W_block: int, r_out) -> np.ndarray:
    """Measured SNR of r_out per block against the FP64 direct convolution."""
    part = partition(np.asarray(s).size, np.asarray(k).size, W_block)
    ref = conv_direct(s, k)
    res = np.zeros(part.P)
    for w in range(part.P):
        j_lo, j_hi, o = part.keep(w)
        res[w] = measured_snr_db(np.asarray(r_out)[o: o + j_hi - j_lo], ref[o: o + j_hi - j_lo])
    return res


def calibrate(s, k, W_block: int, block: int = 0, Q: int = 8) -> float:
    """Reading R14: offset = measured - model SNR at S_q = K_q = Q on one block's kept outputs."""
    part = partition(np.asarray(s).size, np.asarray(k).size, W_block)
    b = part.window(s, block)
    kp = pad_kernel(np.asarray(k, dtype=np.float64))
    cs, sq = compand(b, Q)
    ck, kq = compand(kp, Q)
    j_lo, j_hi, _ = part.keep(block)
    ref = conv_direct(b, kp)[j_lo:j_hi]
    rq = conv_int_range(sq, kq, j_lo, j_hi).astype(np.float64) / (cs * ck)
    smax, rms = block_stats(b)
    kmax, krms = kernel_stats(k)
    return measured_snr_db(rq, ref) - snr_model_db(rms, smax, krms, kmax, Q, Q)


# ----------------------------------------------------------------------------------------
# The paper's packing / unpacking steps (Section III.A-C)
# ----------------------------------------------------------------------------------------
def pack_sym_signal(sq, eps: float) -> np.ndarray:
    """Eq. (4): s-[m] = s~[2m] + eps s~[2m+1] (even-length block)."""
    sq = np.asarray(sq, dtype=np.float64)
    return sq[..., 0::2] + eps * sq[..., 1::2]


def pack_sym_kernel(kq, two_r: int) -> np.ndarray:
    """Eq. (5) for convolution, reading R1: k-[n] = k~[2n+1] + eps^-1 k~[2n], with eps^-1 = 2R
    exactly and k~[N] = 0 for the odd kernel; ceil(N/2) words."""
    kq = np.asarray(kq, dtype=np.float64)
    if kq.size % 2:
        kq = np.concatenate([kq, [0.0]])
    return kq[1::2] + float(two_r) * kq[0::2]


def pack_sym_kernel_printed(kq, two_r: int) -> np.ndarray:
    """Eq. (5) exactly as printed: k~[2n] + eps^-1 k~[2n+1] (kept to show reading R1)."""
    kq = np.asarray(kq, dtype=np.float64)
    if kq.size % 2:
        kq = np.concatenate([kq, [0.0]])
    return kq[0::2] + float(two_r) * kq[1::2]


def unpack_sym(rbar, R: int, w_start: int, m_hi: int) -> np.ndarray:
    """Eqs. (11)-(15) for m in [w_start, m_hi) along the last axis; returns
    r~[2 w_start .. 2 m_hi) as int64.

    u = r- + R_safe                                       (11), reading R7 for R_safe
    side_eps   = R (m = w_start) or eps^-1 (u[m-1] - floor u[m-1])   (12)
    side_epsinv = floor(eps u[m])                          (13)
    r~[2m]   = floor(side_epsinv + side_eps - 2R)          (14)
    r~[2m+1] = floor(floor(u[m]) - eps^-1 side_epsinv - R) (15)
    """
    rbar = np.asarray(rbar, dtype=np.float64)
    eps = epsilon(R)
    two_r = float(2 * R)
    u = (rbar[..., w_start:m_hi] + (R * eps + eps / 2.0)) + float(R * (1 + 2 * R))
    fl = np.floor(u)
    side_epsinv = np.floor(eps * u)
    side_eps = np.empty_like(u)
    side_eps[..., 1:] = two_r * (u[..., :-1] - fl[..., :-1])
    side_eps[..., 0] = float(R)
    even = np.floor(side_epsinv + side_eps - 2.0 * R)
    odd = np.floor(fl - two_r * side_epsinv - R)
    out = np.empty(rbar.shape[:-1] + (2 * (m_hi - w_start),), dtype=np.int64)
    out[..., 0::2] = even.astype(np.int64)
    out[..., 1::2] = odd.astype(np.int64)
    return out


def asym_layout(part: Partition, w: int, M: int):
    """Reading R9: part stride T and the window offset of each part for block w."""
    T = -(-part.W // M)
    base = 0 if w == 0 else 2
    return T, [base + q * T for q in range(M)]


def pack_asym(sq, M: int, eps: float, offs, length: int) -> np.ndarray:
    """Eq. (7): s-[m] = sum_q eps^q s~[off_q + m], zero outside the block."""
    sq = np.asarray(sq, dtype=np.float64)
    out = np.zeros(length, dtype=np.float64)
    for q in range(M):
        seg = np.zeros(length)
        a = offs[q]
        lo, hi = max(0, -a), min(length, sq.size - a)
        if hi > lo:
            seg[lo:hi] = sq[a + lo: a + hi]
        out = out + (eps ** q) * seg
    return out


def unpack_asym(rbar, R: int, M: int) -> np.ndarray:
    """Reading R9 for the cited M-step unpacking: balanced base-2R digits, d_0 = [[x]],
    then x <- (x - d_0) 2R, repeated M times.  Returns an (M, len) int64 array."""
    x = np.asarray(rbar, dtype=np.float64).copy()
    two_r = float(2 * R)
    out = np.zeros((M, x.size), dtype=np.int64)
    for q in range(M):
        d = np.rint(x)
        out[q] = d.astype(np.int64)
        x = (x - d) * two_r
    return out


def _packed_core(a, b, core: str) -> np.ndarray:
    """Tier-2 core on packed words: sequential FP64 time-domain sum, or an FFT (numpy's) of a
    size holding the whole linear result."""
    if core == "td":
        return conv_direct(a, b)
    n = a.size + b.size - 1
    F = 1
    while F < n:
        F *= 2
    return np.fft.irfft(np.fft.rfft(a, F) * np.fft.rfft(b, F), F)[:n]


def conv_blocked_paper(s, k, W_block: int, mode: str, S: int, K: int, core: str = "td",
                       allow_unsafe: bool = False):
    """The method end to end (Section III.A-C): compand (2), pack (4)/(5) or (7), packed block
    convolution (9) or (8), unpack (11)-(15) or the M-step digit unpacking, inverse companding
    (16), placement (17).  Returns (r_out float32, r~ fields int64 at each output position)."""
    s = np.asarray(s)
    part = partition(s.size, np.asarray(k).size, W_block)
    N = part.N_odd
    R = r_max(N, S, K)
    if not allow_unsafe and R > BOUND[mode]:
        raise ValueError(f"R_max = {R} exceeds the {mode} bound {BOUND[mode]}")
    eps = epsilon(R)
    kp = pad_kernel(np.asarray(k, dtype=np.float64))
    ck, kq = compand(kp, K)
    fields = np.zeros(part.out_len, dtype=np.int64)
    out = np.zeros(part.out_len, dtype=np.float64)
    kbar = pack_sym_kernel(kq, 2 * R) if mode == SYM else kq.astype(np.float64)
    for w in range(part.P):
        b = part.window(s, w)
        cs, sq = compand(b, S)
        j_lo, j_hi, o = part.keep(w)
        if mode == SYM:
            sbar = pack_sym_signal(sq, eps)
            rbar = _packed_core(sbar, kbar, core)
            w_start = 0 if w == 0 else (N - 1) // 2          # eq. (10)
            dec = unpack_sym(rbar, R, w_start, W_block // 2)  # r~[2 w_start .. W_block)
            local = np.zeros(W_block, dtype=np.int64)
            local[2 * w_start:] = dec
        else:
            M = 2 if mode == ASYM2 else 3
            T, offs = asym_layout(part, w, M)
            length = T + N - 1
            sbar = pack_asym(sq, M, eps, offs, length)
            rbar = _packed_core(sbar, kq.astype(np.float64), core)[:length]
            digits = unpack_asym(rbar, R, M)
            local = np.zeros(W_block + M * T, dtype=np.int64)
            for q in range(M):
                m_lo = 0 if (w == 0 and q == 0) else N - 1
                idx = np.arange(m_lo, length)
                local[offs[q] + idx] = digits[q, m_lo:length]
        seg = local[j_lo:j_hi]
        fields[o: o + seg.size] = seg
        if cs != 0.0 and ck != 0.0:
            out[o: o + seg.size] = (1.0 / (cs * ck)) * seg.astype(np.float64)     # eq. (16)
    return out.astype(np.float32), fields


def xcorr_blocked(s, k, W_block: int, mode: str, S: int = 0, K: int = 0, out_dtype=np.float32):
    """Cross-correlation c[l] = sum_n s[l+n] k[n] (index l + N - 1) through the blocked
    companded convolution of conv_blocked with the time-reversed kernel, every block in `mode`
    at S_q, K_q (0 = the largest the mode allows, reading R13); FP64 blocks for FULL."""
    s = np.asarray(s, dtype=np.float32)
    kr = np.ascontiguousarray(np.asarray(k, dtype=np.float32)[::-1])
    N_odd = kr.size if kr.size % 2 else kr.size + 1
    if mode != FULL:
        S = S or max_q(mode, N_odd)
        K = K or max_q(mode, N_odd)
    return conv_blocked(s, kr, W_block, fixed_params(s, kr, W_block, mode, S, K), out_dtype=out_dtype)


def int_fields(s, k, W_block: int, S: int, K: int):
    """r~ at every output position under fixed (S_q, K_q), plain definition."""
    ps = fixed_params(s, k, W_block, SYM, S, K)
    _, f, _ = conv_blocked(s, k, W_block, ps, return_fields=True)
    return f
