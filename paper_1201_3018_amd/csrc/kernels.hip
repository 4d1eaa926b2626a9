// Device kernels of libapx (gfx950).
//
// Per overlap-save block (Section II) one workgroup of 256 threads:
//   block statistics (||s||_inf, root second moment) by wave shuffles + LDS,
//   mode / bit allocation (fixed, or the calibrated model of eqs. 18-19, Section IV.D),
//   companding (eq. 2) fused with packing (eqs. 4, 7) into LDS,
//   packed convolution core: register-blocked time-domain FMA loop, or LDS Stockham FFT with
//   the resident kernel spectrum,
//   unpacking (the digits of eq. 9 / eq. 8) fused with inverse companding (eq. 16) and the
//   placement of eq. (17).
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <type_traits>

#include "fft.h"
#include "internal.h"
#include "items.h"

namespace apx {

// ------------------------------------------------------------------------------------------
// small helpers
// ------------------------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T ld_uniform(const T* p, int i) {
    // read-only kernel data indexed uniformly across the wave: constant address space lets the
    // compiler use scalar loads
    return ((const __attribute__((address_space(4))) T*)p)[i];
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ int wave_or(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

// Wave reductions by DPP lane moves (VALU only, no LDS round trips), the result read from lane
// 63 into a scalar: pairs and quads by quad permutes, rows of 16 by rotations of 4 and 8, then
// row 0 into row 1 and row 2 into row 3 (broadcast of lane 15 of each), then rows 0-1 into rows
// 2-3 (broadcast of lane 31).  Lanes outside a move's row mask take 0, the identity of both
// operations here (the maximum is over non-negative values).
template <int CTRL, int ROWS>
__device__ __forceinline__ int dpp_i(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_d(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = dpp_i<CTRL, ROWS>((int)(b & 0xffffffffLL)), hi = dpp_i<CTRL, ROWS>((int)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
__device__ __forceinline__ double wave_sum_dpp(double v) {
    v += dpp_d<0xb1, 0xf>(v);   // quad_perm [1,0,3,2]
    v += dpp_d<0x4e, 0xf>(v);   // quad_perm [2,3,0,1]
    v += dpp_d<0x124, 0xf>(v);  // row_ror:4
    v += dpp_d<0x128, 0xf>(v);  // row_ror:8
    v += dpp_d<0x142, 0xa>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_d<0x143, 0xc>(v);  // row_bcast:31 into rows 2 and 3
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), 63), hi = __builtin_amdgcn_readlane((int)(b >> 32), 63);
    return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// maximum of non-negative floats
__device__ __forceinline__ float wave_max_dpp(float v) {
    v = fmaxf(v, __int_as_float(dpp_i<0xb1, 0xf>(__float_as_int(v))));
    v = fmaxf(v, __int_as_float(dpp_i<0x4e, 0xf>(__float_as_int(v))));
    v = fmaxf(v, __int_as_float(dpp_i<0x124, 0xf>(__float_as_int(v))));
    v = fmaxf(v, __int_as_float(dpp_i<0x128, 0xf>(__float_as_int(v))));
    v = fmaxf(v, __int_as_float(dpp_i<0x142, 0xa>(__float_as_int(v))));
    v = fmaxf(v, __int_as_float(dpp_i<0x143, 0xc>(__float_as_int(v))));
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

struct BlockStats {
    double smax, sumsq;
    int nonfinite;
};

// ||b||_inf, sum b^2 and a non-finite flag over s[start, start + n), all threads get the result.
__device__ BlockStats block_stats(const float* __restrict__ s, int64_t start, int n) {
    __shared__ double red_m[NT / 64], red_s[NT / 64];
    __shared__ int red_f[NT / 64];
    double m = 0.0, q = 0.0;
    int nf = 0;
    constexpr int CH = 8;  // loads in flight per thread
    for (int base = 0; base < n; base += NT * CH) {
        float xs[CH];
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int i = base + threadIdx.x + NT * c;
            xs[c] = (i < n) ? s[start + i] : 0.0f;
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const float x = xs[c];
            if (!isfinite(x)) {
                nf = 1;
            } else {
                double d = (double)x;
                m = fmax(m, fabs(d));
                q += d * d;
            }
        }
    }
    m = wave_max(m);
    q = wave_sum(q);
    nf = wave_or(nf);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red_m[wv] = m;
        red_s[wv] = q;
        red_f[wv] = nf;
    }
    __syncthreads();
    BlockStats r;
    r.smax = red_m[0];
    r.sumsq = red_s[0];
    r.nonfinite = red_f[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) {
        r.smax = fmax(r.smax, red_m[i]);
        r.sumsq += red_s[i];
        r.nonfinite |= red_f[i];
    }
    __syncthreads();
    return r;
}

// SNR of eqs. (18)-(19) as a ratio (the tap count cancels), uniform rounding noise
// sigma_v = ||x||_inf / (Q sqrt 12).
__device__ __forceinline__ double snr_ratio(double rms, double smax, double krms, double kmax, int S, int K) {
    const double r12 = 3.4641016151377545870548926830117447;
    double svs = smax / ((double)S * r12);
    double svk = kmax / ((double)K * r12);
    double a = rms * svk, b = krms * svs, c = svk * svs;
    double D = a * a + b * b + c * c;
    double p = rms * krms;
    return (p * p) / D;
}

// One unit of work: a block (or the first outputs of block 0 for the FFT core).
struct Item {
    int64_t start;  // window start in s
    int nwin;       // window samples present (W_block clipped at the input end)
    int nvalid;     // samples used by the packing (window, or the prefix cut)
    int j_lo, j_hi; // kept local outputs of the block convolution
    int64_t o0;     // r_out index of local output j_lo
    int64_t w;      // block index
};

__device__ __forceinline__ Item make_item(const RunArgs& a, int64_t item, bool fft) {
    Item it;
    const int N = a.N;
    bool prefix = item >= a.P;
    it.w = prefix ? 0 : item;
    it.start = it.w == 0 ? 0 : (int64_t)a.W * it.w - 2;
    int64_t rem = a.L - it.start;
    it.nwin = (int)(rem < a.W_block ? rem : a.W_block);
    it.nvalid = it.nwin;
    if (prefix) {
        // first N+1 outputs of block 0: only its first N+1 samples matter, the rest is zero so
        // that the cyclic FFT result has no wrap-around there
        it.j_lo = 0;
        it.j_hi = N + 1;
        it.o0 = 0;
        if (it.nvalid > N + 1) it.nvalid = N + 1;
    } else if (it.w == 0) {
        it.j_lo = fft ? N + 1 : 0;
        it.j_hi = a.W + N - 1;
        it.o0 = it.j_lo;
    } else {
        it.j_lo = N + 1;
        it.j_hi = N + 1 + a.W;
        it.o0 = (int64_t)N - 1 + (int64_t)a.W * it.w;
    }
    int64_t room = a.out_len - it.o0;
    if (room < 0) room = 0;
    if ((int64_t)(it.j_hi - it.j_lo) > room) it.j_hi = it.j_lo + (int)room;
    if (it.j_hi < it.j_lo) it.j_hi = it.j_lo;
    return it;
}

struct Choice {
    int mode;
    int S, K;
    int64_t R;
    double cs;
    double inv;       // (c_s c_k)^-1 of eq. (16), formed once per block
    double snr_db;
    int flags;
};

// ks_in: the taps' state (*a.ks), which a kernel may load early
__device__ __forceinline__ Choice choose(const RunArgs& a, const BlockStats& st, const KState& ks_in) {
    Choice c;
    KState ks = ks_in;
    // eq. (18)'s sigmas: each block's and the taps' root second moments, or source-level values
    const double rms = a.sigma_s > 0.0 ? a.sigma_s : sqrt(st.sumsq / (double)a.W_block);
    // the block's mean square (rms^2) for the division-free comparison below
    const double ms = a.sigma_s > 0.0 ? a.sigma_s * a.sigma_s : st.sumsq * a.inv_wb;
    const bool kzero = ks.krms == 0.0;
    if (a.sigma_k > 0.0) ks.krms = a.sigma_k;
    c.flags = 0;
    c.snr_db = INFINITY;
    c.mode = a.mode;
    if (a.mode == MD_AUTO) {
        double thr = a.thr_lin, calib = a.calib_db;
        if (a.calib_dev) {  // this call's calibration: offset and threshold ratio
            calib = a.calib_dev[0];
            thr = a.calib_dev[1];
        }
        c.mode = MD_FULL32;
        // model SNR ratio of eqs. (18)-(19), p^2 / D with p^2 = ms krms^2 and
        // D = ms svk^2 + krms^2 svs^2 + svk^2 svs^2, compared as p^2 >= thr D (no division)
        const double k2 = ks.krms * ks.krms;
#pragma unroll
        for (int m = MD_SYM; m <= MD_ASYM2; ++m) {
            if (!((a.cand_mask >> m) & 1) || a.S[m] < 1) continue;
            if (st.smax == 0.0 || kzero) {
                c.mode = m;
                break;
            }
            const double svs = st.smax * a.qs_inv[m], svk = ks.kmax * a.qk_inv[m];
            const double D = ms * (svk * svk) + k2 * (svs * svs) + (svk * svs) * (svk * svs);
            if (ms * k2 >= thr * D) {
                c.mode = m;
                if (a.info) c.snr_db = 10.0 * log10(ms * k2 / D) + calib;  // reported only
                break;
            }
        }
    }
    if (c.mode >= MD_SYM && c.mode <= MD_ASYM3) {
        // select without a runtime array index (that would copy the arguments to scratch)
        const bool s1 = c.mode == MD_SYM, s2 = c.mode == MD_ASYM2;
        c.S = s1 ? a.S[1] : (s2 ? a.S[2] : a.S[3]);
        c.K = s1 ? a.K[1] : (s2 ? a.K[2] : a.K[3]);
        c.R = s1 ? a.R[1] : (s2 ? a.R[2] : a.R[3]);
        const double ck = s1 ? ks.ck[1] : (s2 ? ks.ck[2] : ks.ck[3]);
        c.cs = st.smax == 0.0 ? 0.0 : (double)c.S / st.smax;
        c.inv = 1.0 / (c.cs * ck);
        if (a.info && a.mode != MD_AUTO && st.smax != 0.0 && !kzero)
            c.snr_db = 10.0 * log10(snr_ratio(rms, st.smax, ks.krms, ks.kmax, c.S, c.K));
    } else {
        c.S = c.K = 0;
        c.R = 0;
        c.cs = 0.0;
        c.inv = 0.0;
    }
    if (st.nonfinite || ks.nonfinite) c.flags |= APX_FLAG_NONFINITE;
    if (st.smax == 0.0 || ks.kmax == 0.0) c.flags |= APX_FLAG_ZERO;
    return c;
}

__device__ __forceinline__ Choice choose(const RunArgs& a, const BlockStats& st) { return choose(a, st, *a.ks); }

__device__ __forceinline__ void write_info(const RunArgs& a, const Item& it, const Choice& c, const BlockStats& st,
                                           bool is_report, bool lead = threadIdx.x == 0) {
    if (a.info && is_report && lead) {
        apx_block_info b;
        b.mode = c.mode;
        b.flags = c.flags;
        b.Sq = c.S;
        b.Kq = c.K;
        b.rmax = c.R;
        b.cs = c.cs;
        b.smax = st.smax;
        b.rms = sqrt(st.sumsq / (double)a.W_block);
        b.snr_pred_db = c.snr_db;
        a.info[it.w] = b;
    }
}

// Uniform outputs (all zero, or all NaN) for a block that needs no arithmetic.
__device__ __forceinline__ void fill_block(const RunArgs& a, const Item& it, float v) {
    for (int j = it.j_lo + threadIdx.x; j < it.j_hi; j += NT) {
        a.out[it.o0 + (j - it.j_lo)] = v;
        if (a.fields) a.fields[it.o0 + (j - it.j_lo)] = 0.0;
    }
}

// STREAM: the non-temporal store (out_store), for the FFT cores' rows of consecutive outputs
template <bool STREAM = false>
__device__ __forceinline__ void put(const RunArgs& a, const Item& it, int j, double rt, double inv) {
    const int64_t o = it.o0 + (j - it.j_lo);
    rt += 0.0;  // a zero digit is +0, as the integer it stands for
    if (a.fields) a.fields[o] = rt;
    if (STREAM) out_store(&a.out[o], (float)(inv * rt));  // eq. (16)
    else a.out[o] = (float)(inv * rt);
}

// Where the outputs of a block go.  StoreSink writes r_out (and the debug fields), StreamSink
// the same with the non-temporal hint (the FFT cores); ArgmaxSink keeps, per thread, the largest
// output seen and its r_out index (ties: smallest index).
template <bool STREAM>
struct OutSink {
    __device__ __forceinline__ void put(const RunArgs& a, const Item& it, int j, double rt, double inv) {
        apx::put<STREAM>(a, it, j, rt, inv);
    }
    __device__ __forceinline__ void put32(const RunArgs& a, const Item& it, int j, float v) {
        const int64_t o = it.o0 + (j - it.j_lo);
        if (STREAM) out_store(&a.out[o], v);
        else a.out[o] = v;
        if (a.fields) a.fields[o] = 0.0;
    }
};
using StoreSink = OutSink<false>;
using StreamSink = OutSink<true>;
// The one-workgroup FFT cores stream the asymmetric modes' outputs (rows of one digit each:
// 3-6% faster on the paper sweep's shapes) and store the symmetric and FP32 ones plainly (the
// hint measured 0-3% slower there)
template <int MODE>
using AsymSink = typename std::conditional<MODE == MD_ASYM2 || MODE == MD_ASYM3, StreamSink, StoreSink>::type;

// Order-preserving 64-bit key of (value, index): larger value first, then smaller index.
// -0 counts as +0; NaN never enters.  Key 0 means "no finite output".
__device__ __forceinline__ unsigned long long argmax_key(float v, int64_t o) {
    const unsigned int b = __float_as_uint(v + 0.0f);
    const unsigned int u = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    return ((unsigned long long)u << 32) | (unsigned long long)(0xFFFFFFFFu - (unsigned int)o);
}

struct ArgmaxSink {
    float bv = 0.0f;
    int64_t bo = -1;  // -1: no finite output seen
    // the order of argmax_key: larger value, then smaller index; -0 equals +0; NaN never enters
    __device__ __forceinline__ void consider(int64_t o, float v) {
        if (v == v && (bo < 0 || v > bv || (v == bv && o < bo))) {
            bv = v;
            bo = o;
        }
    }
    __device__ __forceinline__ unsigned long long key() const { return bo < 0 ? 0ull : argmax_key(bv, bo); }
    __device__ __forceinline__ void put(const RunArgs& a, const Item& it, int j, double rt, double inv) {
        consider(it.o0 + (j - it.j_lo), (float)(inv * (rt + 0.0)));  // eq. (16), as stored by StoreSink
    }
    __device__ __forceinline__ void put32(const RunArgs& a, const Item& it, int j, float v) {
        consider(it.o0 + (j - it.j_lo), v);
    }
};

// Companded sample s~[i] of the item's window (eq. 2); zero outside [0, nvalid).
__device__ __forceinline__ double sq_at(const RunArgs& a, const Item& it, double cs, int i) {
    if (i < 0 || i >= it.nvalid) return 0.0;
    return rint(cs * (double)a.s[it.start + i]);
}

// ------------------------------------------------------------------------------------------
// Unpacking (exact integer digits of the packed results)
// ------------------------------------------------------------------------------------------
// Symmetric packing: rb = 2R Dm + B + eps De with |B| <= R, |Dm|, |De| < R (eq. 9).  The side-eps
// digit is read from the fraction, the rest split into base and side-eps^-1 digits by a
// balanced division by 2R.  At |B| = R the integer part 2R Dm + B is the same for (Dm, R) and
// (Dm + 1, -R): the word does not tell them apart.  The split then takes the one with the
// smaller |Dm|, which is wrong whenever the true Dm and B have opposite signs; this tie is the
// case the no-overlap condition excludes (every product of a window at full scale with one
// sign).  Everywhere else the digits are unique and equal eqs. (11)-(15) where those are exact.
struct SymDigits {
    double Dm, B, De;
};
__device__ __forceinline__ SymDigits sym_split(double rb, double two_r, double inv_two_r, double R) {
    SymDigits d;
    double I = rint(rb);
    d.De = rint((rb - I) * two_r);
    double q = rint(I * inv_two_r);  // off by at most one; the range corrections below undo it
    double B = I - q * two_r;
    if (B > R) {
        q += 1.0;
        B -= two_r;
    }
    if (B < -R) {
        q -= 1.0;
        B += two_r;
    }
    if (B == R && q < 0.0) {
        q += 1.0;
        B -= two_r;
    }
    if (B == -R && q > 0.0) {
        q -= 1.0;
        B += two_r;
    }
    d.Dm = q;
    d.B = B;
    return d;
}

// Decode and store the kept outputs of a symmetric-packed block.  rbar(m) returns the packed
// result at word m (m >= -1; word -1 is zero).
template <typename Fn, typename Sink = StoreSink>
__device__ __forceinline__ void sym_unpack_store(const RunArgs& a, const Item& it, const Choice& c, Fn rbar,
                                                 Sink&& sk = Sink{}) {
    const double two_r = (double)(2 * c.R), R = (double)c.R, inv_two_r = 1.0 / two_r;
    const int m_lo = it.j_lo >> 1, m_hi = (it.j_hi + 1) >> 1;
    for (int m = m_lo + threadIdx.x; m < m_hi; m += NT) {
        SymDigits cur = sym_split(rbar(m), two_r, inv_two_r, R);
        const int j0 = 2 * m, j1 = 2 * m + 1;
        if (j0 >= it.j_lo && j0 < it.j_hi) {
            double de_prev = (m >= 1) ? sym_split(rbar(m - 1), two_r, inv_two_r, R).De : 0.0;
            sk.put(a, it, j0, cur.Dm + de_prev, c.inv);
        }
        if (j1 >= it.j_lo && j1 < it.j_hi) sk.put(a, it, j1, cur.B, c.inv);
    }
}

// Asymmetric packing: rb = sum_q eps^q d_q, balanced base-2R digits taken one after the other.
template <int MM, typename Fn, typename Sink = StoreSink>
__device__ __forceinline__ void asym_unpack_store(const RunArgs& a, const Item& it, const Choice& c, int Tit,
                                                  int base_off, int m_first0, int m_first, int m_end, Fn rbar,
                                                  Sink&& sk = Sink{}) {
    const double two_r = (double)(2 * c.R);
    for (int m = m_first0 + threadIdx.x; m < m_end; m += NT) {
        double x = rbar(m);
#pragma unroll
        for (int q = 0; q < MM; ++q) {
            double d = rint(x);
            x = (x - d) * two_r;
            if (q > 0 && m < m_first) continue;
            const int j = base_off + q * Tit + m;
            if (j >= it.j_lo && j < it.j_hi) sk.put(a, it, j, d, c.inv);
        }
    }
}

// ------------------------------------------------------------------------------------------
// Time-domain core
// ------------------------------------------------------------------------------------------
constexpr int RB = 8;    // most consecutive outputs per thread (margins of the LDS buffers)
constexpr int KUN = 8;   // tap arrays are zero padded to a multiple of 8

// r[m - mlo] = sum_n x[m - n] kt[n] for m in [mlo, mhi).  x: LDS, logical index i at x[i],
// valid (zero filled) for i in [mlo - npad - 8, mhi + RB).  Each thread owns C consecutive
// outputs m0 .. m0+C-1 (the tile, 4 or 8) and walks the taps in steps of C: step n0 reads
// x[m0 - n0 - C .. m0 - n0 + C - 1], the chunk x[m0 - n0 .. m0 - n0 + C - 1] it shares with the
// previous step stays in registers, so one chunk of C samples is read per C^2 FMAs (the two chunk
// registers swap roles every step).  C = 8 reads less LDS per FMA; C = 4 keeps twice as many
// threads busy on a block of fewer than 8 NT outputs.  The FMA order per output is n = 0, 1, 2,
// ... as in the plain sum.
template <typename T, int C>
__device__ __forceinline__ void td_step(const T* hi, const T* lo, const T* kt, int n0, T* acc) {
    // hi[e] = x[m0 - n0 + e], lo[e] = x[m0 - n0 - C + e]; output i, tap n0 + t reads x[m0 + i - n0 - t]
#pragma unroll
    for (int t = 0; t < C; ++t) {
        const T kv = ld_uniform(kt, n0 + t);
#pragma unroll
        for (int i = 0; i < C; ++i) {
            const int e = i - t;
            acc[i] = fma(e >= 0 ? hi[e] : lo[C + e], kv, acc[i]);
        }
    }
}

template <typename T, int C>
__device__ __forceinline__ void td_core(const T* x, const T* kt, int npad, int mlo, int mhi, T* r) {
    static_assert((C == 4 || C == 8) && C <= RB && KUN % C == 0, "tiles of 4 or 8 outputs");
    for (int m0 = mlo + C * threadIdx.x; m0 < mhi; m0 += C * NT) {
        T acc[C];
#pragma unroll
        for (int i = 0; i < C; ++i) acc[i] = (T)0;
        const T* xp = x + m0;
        T c0[C], c1[C];
#pragma unroll
        for (int e = 0; e < C; ++e) c0[e] = xp[e];
        int n0 = 0;
        for (; n0 + 2 * C <= npad; n0 += 2 * C) {
#pragma unroll
            for (int e = 0; e < C; ++e) c1[e] = xp[e - n0 - C];
            td_step<T, C>(c0, c1, kt, n0, acc);
#pragma unroll
            for (int e = 0; e < C; ++e) c0[e] = xp[e - n0 - 2 * C];
            td_step<T, C>(c1, c0, kt, n0 + C, acc);
        }
        if (n0 < npad) {  // npad is a multiple of 8, so of C: one step left
#pragma unroll
            for (int e = 0; e < C; ++e) c1[e] = xp[e - n0 - C];
            td_step<T, C>(c0, c1, kt, n0, acc);
        }
#pragma unroll
        for (int i = 0; i < C; ++i)
            if (m0 + i < mhi) r[m0 + i - mlo] = acc[i];
    }
}

size_t td_lds_bytes(int mode, int N, int W_block, int T2, int T3) {
    // input words with zero margins + results
    auto words = [&](int lw, int npad, int nres, size_t esz) {
        return (size_t)(npad + 8 + lw + RB + 8) * esz + (size_t)(nres + RB) * esz;
    };
    auto pad8 = [](int n) { return (n + 7) / 8 * 8; };
    size_t b = 0;
    const int nsym = (N + 1) / 2;
    if (mode == MD_SYM || mode == MD_AUTO) b = std::max(b, words(W_block / 2, pad8(nsym), W_block / 2 + 1, 8));
    if (mode == MD_ASYM2 || mode == MD_AUTO) b = std::max(b, words(T2 + N - 1, pad8(N), T2 + N, 8));
    if (mode == MD_ASYM3) b = std::max(b, words(T3 + N - 1, pad8(N), T3 + N, 8));
    if (mode == MD_FULL32 || mode == MD_AUTO) b = std::max(b, words(W_block, pad8(N), W_block, 4));
    if (mode == MD_FULL64) b = std::max(b, words(W_block, pad8(N), W_block, 8));
    return b;
}

template <int MODE, int C>
__device__ void td_item(const RunArgs& a, const Item& it, const Choice& c, char* lds) {
    const int N = a.N;
    if constexpr (MODE == MD_FULL32 || MODE == MD_FULL64) {
        using T = typename std::conditional<MODE == MD_FULL32, float, double>::type;
        const int npad = a.kf_pad;
        const int lw = it.nvalid;
        T* buf = (T*)lds;
        const int pre = npad + 8;
        T* x = buf + pre;
        const int total = pre + a.W_block + RB + 8;
        T* res = buf + total;
        for (int i = threadIdx.x; i < total; i += NT) {
            const int li = i - pre;
            buf[i] = (li >= 0 && li < lw) ? (T)a.s[it.start + li] : (T)0;
        }
        __syncthreads();
        const T* kt = (MODE == MD_FULL32) ? (const T*)a.kf : (const T*)a.kd;
        td_core<T, C>(x, kt, npad, it.j_lo, it.j_hi, res);
        __syncthreads();
        for (int j = it.j_lo + threadIdx.x; j < it.j_hi; j += NT) {
            const int64_t o = it.o0 + (j - it.j_lo);
            a.out[o] = (float)res[j - it.j_lo];
            if (a.fields) a.fields[o] = 0.0;
        }
    } else if constexpr (MODE == MD_SYM) {
        // eq. (4): s-[m] = s~[2m] + eps s~[2m+1] over the whole window
        const double eps = 1.0 / (2.0 * (double)c.R);
        const int nk = a.kq_len[MD_SYM], npad = a.kq_pad[MD_SYM];
        const int lw = a.W_block / 2;
        double* buf = (double*)lds;
        const int pre = npad + 8;
        double* x = buf + pre;
        const int total = pre + lw + RB + 8;
        double* res = buf + total;
        for (int i = threadIdx.x; i < total; i += NT) {
            const int m = i - pre;
            double v = 0.0;
            if (m >= 0 && m < lw) v = sq_at(a, it, c.cs, 2 * m) + eps * sq_at(a, it, c.cs, 2 * m + 1);
            buf[i] = v;
        }
        __syncthreads();
        // words needed: m in [j_lo/2 - 1, (j_hi+1)/2)
        int mlo = (it.j_lo >> 1) - 1;
        if (mlo < 0) mlo = 0;
        const int mhi = (it.j_hi + 1) >> 1;
        (void)nk;
        td_core<double, C>(x, a.kq[MD_SYM], npad, mlo, mhi, res);
        __syncthreads();
        sym_unpack_store(a, it, c, [&](int m) -> double { return m < mlo ? 0.0 : res[m - mlo]; });
    } else {
        constexpr int MM = (MODE == MD_ASYM2) ? 2 : 3;
        // eq. (7) with part stride T; block 0 parts at q T (part 0 valid from word 0), other
        // blocks at 2 + q T (valid from word N-1)
        const double eps = 1.0 / (2.0 * (double)c.R);
        const int npad = a.kq_pad[MODE];
        const int T = a.T[MODE];
        const int lw = T + N - 1;
        const int base_off = (it.w == 0) ? 0 : 2;
        double* buf = (double*)lds;
        const int pre = npad + 8;
        double* x = buf + pre;
        const int total = pre + lw + RB + 8;
        double* res = buf + total;
        for (int i = threadIdx.x; i < total; i += NT) {
            const int m = i - pre;
            double v = 0.0;
            if (m >= 0 && m < lw) {
                double e = 1.0;
#pragma unroll
                for (int q = 0; q < MM; ++q) {
                    v += e * sq_at(a, it, c.cs, base_off + q * T + m);
                    e *= eps;
                }
            }
            buf[i] = v;
        }
        __syncthreads();
        const int m_first0 = (it.w == 0) ? 0 : N - 1;
        td_core<double, C>(x, a.kq[MODE], npad, m_first0, lw, res);
        __syncthreads();
        asym_unpack_store<MM>(a, it, c, T, base_off, m_first0, N - 1, lw,
                              [&](int m) -> double { return res[m - m_first0]; });
    }
}

// C: outputs per thread (the tile of td_core)
template <bool MANY, int C>
__global__ void __launch_bounds__(NT) k_td(RunArgs a0) {
    extern __shared__ char lds_td[];
    int64_t item = blockIdx.x;
    const RunArgs& a = item_args<MANY>(a0, item);
    const Item it = make_item(a, item, false);
    const BlockStats st = block_stats(a.s, it.start, it.nwin);
    const Choice c = choose(a, st);
    write_info(a, it, c, st, true);
    if (c.flags & APX_FLAG_NONFINITE) {
        fill_block(a, it, NAN);
        return;
    }
    if ((c.flags & APX_FLAG_ZERO) && c.mode != MD_FULL32 && c.mode != MD_FULL64) {
        fill_block(a, it, 0.0f);
        return;
    }
    switch (c.mode) {
        case MD_SYM: td_item<MD_SYM, C>(a, it, c, lds_td); break;
        case MD_ASYM2: td_item<MD_ASYM2, C>(a, it, c, lds_td); break;
        case MD_ASYM3: td_item<MD_ASYM3, C>(a, it, c, lds_td); break;
        case MD_FULL64: td_item<MD_FULL64, C>(a, it, c, lds_td); break;
        default: td_item<MD_FULL32, C>(a, it, c, lds_td); break;
    }
}

// tile: outputs per thread, 4 or 8
hipError_t launch_td(const RunArgs& a, size_t lds_bytes, int tile, hipStream_t st) {
    if (lds_bytes > 65536) {
        for (const void* f : {(const void*)k_td<false, 4>, (const void*)k_td<true, 4>, (const void*)k_td<false, 8>,
                              (const void*)k_td<true, 8>}) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
            if (e != hipSuccess) return e;
        }
    }
    const dim3 g((unsigned)a.nitems), b(NT);
    if (tile == 4) {
        if (a.many) hipLaunchKernelGGL((k_td<true, 4>), g, b, lds_bytes, st, a);
        else hipLaunchKernelGGL((k_td<false, 4>), g, b, lds_bytes, st, a);
    } else {
        if (a.many) hipLaunchKernelGGL((k_td<true, 8>), g, b, lds_bytes, st, a);
        else hipLaunchKernelGGL((k_td<false, 8>), g, b, lds_bytes, st, a);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// FFT core
// ------------------------------------------------------------------------------------------
// Complex points of the packed FFT for word length F: MW = F / 2.
// PACKED: the caller has already written the packed words into re / im (pack_regs).
template <int MODE, int MW, typename Sink>
__device__ void fft_item_tail(const RunArgs& a, const Item& it, const Choice& c, char* lds, Sink& sk);

// REGPACK: the register route of the 16 NT and 32 NT point FP64 transforms (below) is allowed.
template <int MODE, int MW, bool PACKED = false, typename Sink = StoreSink, bool REGPACK = true>
__device__ void fft_item(const RunArgs& a, const Item& it, const Choice& c, char* lds, Sink&& sk = Sink{}) {
    using T = typename std::conditional<MODE == MD_FULL32, float, double>::type;
    using T2 = typename tw_of<T>::type;
    constexpr int F = 2 * MW;
    T* re = (T*)lds;
    T* im = re + MW;
    const int N = a.N;
    const T2* tw;
    if constexpr (MODE == MD_FULL32)
        tw = a.twf + F;
    else
        tw = a.twd + F;
    // The FP64 transforms of 16 NT and 32 NT points run in registers: thread t packs its points
    // t + NT k straight into them, with no pass of the words through LDS (not the symmetric words
    // at 32 NT, whose 64 sample-pair loads per thread spill).
    constexpr bool REGF = REGPACK && !PACKED && std::is_same<T, double>::value &&
                          (MW == 16 * NT || (MW == 32 * NT && MODE != MD_SYM));
    if constexpr (REGF) {
        constexpr int E = MW / NT;
        cx<double> v[E];
        const double eps = 1.0 / (2.0 * (double)c.R), cs = c.cs;
        if constexpr (MODE == MD_SYM) {
            const float* sp = a.s + it.start;
            if (4 * MW <= it.nvalid && (reinterpret_cast<uintptr_t>(sp) & 7) == 0) {
                const float2* s2 = reinterpret_cast<const float2*>(sp);
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int n = threadIdx.x + NT * k;
                    const float2 p0 = s2[2 * n], p1 = s2[2 * n + 1];
                    v[k] = {rint(cs * (double)p0.x) + eps * rint(cs * (double)p0.y),
                            rint(cs * (double)p1.x) + eps * rint(cs * (double)p1.y)};
                }
            } else {
#pragma unroll
                for (int k = 0; k < E; ++k) {
                    const int i0 = 4 * (threadIdx.x + NT * k);
                    v[k] = {sq_at(a, it, cs, i0) + eps * sq_at(a, it, cs, i0 + 1),
                            sq_at(a, it, cs, i0 + 2) + eps * sq_at(a, it, cs, i0 + 3)};
                }
            }
        } else {
            constexpr int MM = (MODE == MD_ASYM2) ? 2 : 3;
            const bool prefix = it.j_lo == 0;
            const int Tit = prefix ? (N + 1 + MM - 1) / MM : a.T[MODE];
            const int base_off = it.j_lo - (N - 1);
            const int lw = Tit + N - 1;
#pragma unroll
            for (int k = 0; k < E; ++k) {
                const int n = threadIdx.x + NT * k;
                double w2[2];
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int m = 2 * n + h;
                    double acc = 0.0;
                    if (m < lw) {
                        double e = 1.0;
#pragma unroll
                        for (int q = 0; q < MM; ++q) {
                            acc += e * sq_at(a, it, cs, base_off + q * Tit + m);
                            e *= eps;
                        }
                    }
                    w2[h] = acc;
                }
                v[k] = {w2[0], w2[1]};
            }
        }
        group_fft_regs<E, false>(v, (double*)re, (double*)im, (const double2*)tw);
    }
    if constexpr (!PACKED && !REGF) {
        // ---- pack: z[n] = x[2n] + i x[2n+1]
        if constexpr (MODE == MD_FULL32) {
            const float* sp = a.s + it.start;
            if (2 * MW <= it.nvalid && (reinterpret_cast<uintptr_t>(sp) & 7) == 0) {
                const float2* s2 = reinterpret_cast<const float2*>(sp);
                for (int n = threadIdx.x; n < MW; n += NT) {
                    const float2 p = s2[n];
                    re[n] = p.x;
                    im[n] = p.y;
                }
            } else {
                for (int n = threadIdx.x; n < MW; n += NT) {
                    const int i0 = 2 * n;
                    re[n] = (i0 < it.nvalid) ? a.s[it.start + i0] : 0.0f;
                    im[n] = (i0 + 1 < it.nvalid) ? a.s[it.start + i0 + 1] : 0.0f;
                }
            }
        } else if constexpr (MODE == MD_SYM) {
            const double eps = 1.0 / (2.0 * (double)c.R);
            const float* sp = a.s + it.start;
            if (4 * MW <= it.nvalid && (reinterpret_cast<uintptr_t>(sp) & 7) == 0) {
                // every sample of the packed words is valid: sample pairs, no per-sample bounds
                const float2* s2 = reinterpret_cast<const float2*>(sp);
                const double cs = c.cs;
                for (int n = threadIdx.x; n < MW; n += NT) {
                    const float2 p0 = s2[2 * n], p1 = s2[2 * n + 1];
                    re[n] = rint(cs * (double)p0.x) + eps * rint(cs * (double)p0.y);
                    im[n] = rint(cs * (double)p1.x) + eps * rint(cs * (double)p1.y);
                }
            } else {
                for (int n = threadIdx.x; n < MW; n += NT) {
                    const int i0 = 4 * n;
                    re[n] = sq_at(a, it, c.cs, i0) + eps * sq_at(a, it, c.cs, i0 + 1);
                    im[n] = sq_at(a, it, c.cs, i0 + 2) + eps * sq_at(a, it, c.cs, i0 + 3);
                }
            }
        } else {
            constexpr int MM = (MODE == MD_ASYM2) ? 2 : 3;
            const double eps = 1.0 / (2.0 * (double)c.R);
            const bool prefix = it.j_lo == 0;
            const int Tit = prefix ? (N + 1 + MM - 1) / MM : a.T[MODE];
            const int base_off = it.j_lo - (N - 1);
            const int lw = Tit + N - 1;
            for (int n = threadIdx.x; n < MW; n += NT) {
                double v[2];
    #pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int m = 2 * n + h;
                    double acc = 0.0;
                    if (m < lw) {
                        double e = 1.0;
    #pragma unroll
                        for (int q = 0; q < MM; ++q) {
                            acc += e * sq_at(a, it, c.cs, base_off + q * Tit + m);
                            e *= eps;
                        }
                    }
                    v[h] = acc;
                }
                re[n] = v[0];
                im[n] = v[1];
            }
        }
    }
    if constexpr (!REGF) {
        __syncthreads();
        fft_lds<T, MW, false>(re, im, tw);
    }
    fft_item_tail<MODE, MW>(a, it, c, lds, sk);
}

// The steps of fft_item after the forward transform (its spectrum in natural order in the LDS):
// the spectral step, the inverse transform, then unpacking, dequantization and placement.
template <int MODE, int MW, typename Sink>
__device__ void fft_item_tail(const RunArgs& a, const Item& it, const Choice& c, char* lds, Sink& sk) {
    using T = typename std::conditional<MODE == MD_FULL32, float, double>::type;
    using T2 = typename tw_of<T>::type;
    constexpr int F = 2 * MW;
    T* re = (T*)lds;
    T* im = re + MW;
    const int N = a.N;
    const T2* tw;
    const T2* H;
    if constexpr (MODE == MD_FULL32) {
        tw = a.twf + F;
        H = a.spec32;
    } else {
        tw = a.twd + F;
        H = a.spec[MODE];
    }
    spectral_step<T, MW>(re, im, tw, H);
    fft_lds<T, MW, true>(re, im, tw);
    // ---- unpack + dequantize + place
    auto word = [&](int m) -> double {
        if (m < 0) return 0.0;
        return (m & 1) ? (double)im[m >> 1] : (double)re[m >> 1];
    };
    if constexpr (MODE == MD_FULL32) {
        // outputs 2u, 2u + 1 are re[u], im[u]
        const int u_lo = it.j_lo >> 1, u_hi = (it.j_hi + 1) >> 1;
        for (int u = u_lo + threadIdx.x; u < u_hi; u += NT) {
            const float v0 = (float)re[u], v1 = (float)im[u];
            if (2 * u >= it.j_lo) sk.put32(a, it, 2 * u, v0);
            if (2 * u + 1 < it.j_hi) sk.put32(a, it, 2 * u + 1, v1);
        }
    } else if constexpr (MODE == MD_SYM) {
        // words 2u, 2u + 1 are re[u], im[u] and give outputs 4u .. 4u + 3 (eq. 9 digits; the side
        // digit of word 2u - 1 is taken from im[u - 1], word -1 being zero)
        const double two_r = (double)(2 * c.R), R = (double)c.R, inv_two_r = 1.0 / two_r;
        const int u_lo = it.j_lo >> 2, u_hi = (it.j_hi + 3) >> 2;
        for (int u = u_lo + threadIdx.x; u < u_hi; u += NT) {
            const SymDigits d0 = sym_split((double)re[u], two_r, inv_two_r, R);
            const SymDigits d1 = sym_split((double)im[u], two_r, inv_two_r, R);
            const double dprev = u >= 1 ? sym_split((double)im[u - 1], two_r, inv_two_r, R).De : 0.0;
            const double v[4] = {d0.Dm + dprev, d0.B, d1.Dm + d0.De, d1.B};
#pragma unroll
            for (int h = 0; h < 4; ++h) {
                const int j = 4 * u + h;
                if (j >= it.j_lo && j < it.j_hi) sk.put(a, it, j, v[h], c.inv);
            }
        }
    } else {
        constexpr int MM = (MODE == MD_ASYM2) ? 2 : 3;
        const bool prefix = it.j_lo == 0;
        const int Tit = prefix ? (N + 1 + MM - 1) / MM : a.T[MODE];
        const int base_off = it.j_lo - (N - 1);
        const int lw = Tit + N - 1;
        asym_unpack_store<MM>(a, it, c, Tit, base_off, N - 1, N - 1, lw, word, sk);
    }
}

template <int LOGF, bool MANY>
__global__ void __launch_bounds__(NT) k_fft(RunArgs a0) {
    constexpr int F = 1 << LOGF;        // words for FP32 / asymmetric modes
    constexpr int MA = F / 2;           // complex points, FP32 / asymmetric
    constexpr int MS = F / 4;           // complex points, symmetric (F/2 words)
    extern __shared__ __attribute__((aligned(16))) char lds[];  // MA complex FP64 points
    int64_t item = blockIdx.x;
    const RunArgs& a = item_args<MANY>(a0, item);
    const Item it = make_item(a, item, true);
    const BlockStats st = block_stats(a.s, it.start, it.nwin);
    const Choice c = choose(a, st);
    write_info(a, it, c, st, item < a.P);
    if (c.flags & APX_FLAG_NONFINITE) {
        fill_block(a, it, NAN);
        return;
    }
    if ((c.flags & APX_FLAG_ZERO) && c.mode != MD_FULL32) {
        fill_block(a, it, 0.0f);
        return;
    }
    if (it.j_hi <= it.j_lo) return;
    // at 2^14 words the register packing of every mode in one kernel spills: the words go through LDS
    constexpr bool RP = LOGF < 14;
    switch (c.mode) {
        case MD_SYM: fft_item<MD_SYM, MS, false, StoreSink, RP>(a, it, c, lds); break;
        case MD_ASYM2: fft_item<MD_ASYM2, MA, false, AsymSink<MD_ASYM2>, RP>(a, it, c, lds); break;
        case MD_ASYM3: fft_item<MD_ASYM3, MA, false, AsymSink<MD_ASYM3>, RP>(a, it, c, lds); break;
        default: fft_item<MD_FULL32, MA>(a, it, c, lds); break;
    }
}

// One fixed packed mode at a transform of its own length, 2 MW words (MW = 2^LOGMW complex
// points): the asymmetric modes pack T + N - 1 words and the symmetric mode W_block / 2, so
// they need shorter transforms than the W_block words of the FP32 slot that k_fft is sized by.
template <int MODE, int LOGMW, bool MANY>
__global__ void __launch_bounds__(NT) k_fft1(RunArgs a0) {
    extern __shared__ __attribute__((aligned(16))) char lds[];  // MW complex FP64 points
    int64_t item = blockIdx.x;
    const RunArgs& a = item_args<MANY>(a0, item);
    const Item it = make_item(a, item, true);
    const BlockStats st = block_stats(a.s, it.start, it.nwin);
    const Choice c = choose(a, st);  // a fixed mode: c.mode == MODE
    write_info(a, it, c, st, item < a.P);
    if (c.flags & APX_FLAG_NONFINITE) {
        fill_block(a, it, NAN);
        return;
    }
    if (c.flags & APX_FLAG_ZERO) {
        fill_block(a, it, 0.0f);
        return;
    }
    if (it.j_hi <= it.j_lo) return;
    fft_item<MODE, 1 << LOGMW, false, AsymSink<MODE>>(a, it, c, lds);
}

int fft_min_logF() { return 9; }
int fft_max_logF() { return 14; }

#define APX_FFT1_SIZES(X, MODE) X(MODE, 7) X(MODE, 8) X(MODE, 9) X(MODE, 10) X(MODE, 11) X(MODE, 12) X(MODE, 13)

template <bool MANY>
static const void* fft1_fn(int mode, int logmw) {
#define APX_FN(M_, L_) \
    if (mode == M_ && logmw == L_) return (const void*)k_fft1<M_, L_, MANY>;
    APX_FFT1_SIZES(APX_FN, MD_SYM)
    APX_FFT1_SIZES(APX_FN, MD_ASYM2)
    APX_FFT1_SIZES(APX_FN, MD_ASYM3)
#undef APX_FN
    return nullptr;
}

bool fft1_supported(int mode, int logmw) { return fft1_fn<false>(mode, logmw) != nullptr; }

hipError_t fft1_set_lds(int mode, int logmw) {
    for (const void* f : {fft1_fn<false>(mode, logmw), fft1_fn<true>(mode, logmw)}) {
        if (!f) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                          (int)fft_lds_bytes(true, 1 << logmw));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fft1(const RunArgs& a, int mode, int logmw, hipStream_t st) {
    dim3 g((unsigned)a.nitems);
    const size_t lds = fft_lds_bytes(true, 1 << logmw);
#define APX_GO(M_, L_)                                                                  \
    if (mode == M_ && logmw == L_) {                                                    \
        if (a.many) hipLaunchKernelGGL((k_fft1<M_, L_, true>), g, dim3(NT), lds, st, a);  \
        else hipLaunchKernelGGL((k_fft1<M_, L_, false>), g, dim3(NT), lds, st, a);        \
        return hipGetLastError();                                                       \
    }
    APX_FFT1_SIZES(APX_GO, MD_SYM)
    APX_FFT1_SIZES(APX_GO, MD_ASYM2)
    APX_FFT1_SIZES(APX_GO, MD_ASYM3)
#undef APX_GO
    return hipErrorInvalidValue;
}

// the FP64 rows of the asymmetric / FP32 slot (F/2 points) or the symmetric slot (F/4 points)
static size_t fft_lds(int logF) {
    const size_t a = fft_lds_bytes(true, 1 << (logF - 1)), b = fft_lds_bytes(true, 1 << (logF - 2));
    return a > b ? a : b;
}

// Raises the LDS limit of the kernel for logF (once, at kernel preparation: launches may be
// captured into a graph).
template <bool MANY>
static const void* fft_fn(int logF) {
    switch (logF) {
        case 9: return (const void*)k_fft<9, MANY>;
        case 10: return (const void*)k_fft<10, MANY>;
        case 11: return (const void*)k_fft<11, MANY>;
        case 12: return (const void*)k_fft<12, MANY>;
        case 13: return (const void*)k_fft<13, MANY>;
        case 14: return (const void*)k_fft<14, MANY>;
        default: return nullptr;
    }
}

hipError_t fft_set_lds(int logF) {
    for (const void* f : {fft_fn<false>(logF), fft_fn<true>(logF)}) {
        if (!f) return hipErrorInvalidValue;
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)fft_lds(logF));
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fft(const RunArgs& a, int logF, hipStream_t st) {
    dim3 g((unsigned)a.nitems);
    const size_t lds = fft_lds(logF);
#define APX_GO(L_)                                                           \
    case L_:                                                                 \
        if (a.many) hipLaunchKernelGGL((k_fft<L_, true>), g, dim3(NT), lds, st, a);  \
        else hipLaunchKernelGGL((k_fft<L_, false>), g, dim3(NT), lds, st, a);        \
        break;
    switch (logF) {
        APX_GO(9)
        APX_GO(10)
        APX_GO(11)
        APX_GO(12)
        APX_GO(13)
        APX_GO(14)
#undef APX_GO
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}


// ------------------------------------------------------------------------------------------
// Multi-pass FFT core: blocks whose transform exceeds one workgroup's LDS (fixed packed modes
// and FP32).  The MW = F1 F2 complex points of an item are transformed in four steps through a
// device scratch of MW points per item, with index n = n1 F2 + n2 and k = k1 + F1 k2:
//   columns: pack z[n], DFT over n1 (length F1), twiddle W_MW^(n2 k1)      -> scratch (k1, n2)
//   rows:    DFT over n2 (length F2): X[k1 + F1 k2]; the spectral step pairs row k1 with row
//            (F1 - k1) mod F1 (reversed), so one workgroup takes both; inverse DFT over k2,
//            twiddle W_MW^-(n2 k1)                                          -> scratch (k1, n2)
//   columns: inverse DFT over k1: the words of the cyclic convolution at n; unpack (the
//            symmetric mode writes the words and a last pass unpacks them).
// The transforms are radix-2 passes in LDS over several independent sequences at a time.
// ------------------------------------------------------------------------------------------
constexpr int BIG_TC = 16;  // columns per workgroup of the column passes

// buf[i C + c], c < C: C sequences of Fn points.  DIT takes bit-reversed input and leaves natural
// order; DIF takes natural order and leaves bit-reversed order.  tw: W_Fn^t, t < Fn.
template <typename T, int Fn, int C, bool INV>
__device__ __forceinline__ void big_fft_dit(cx<T>* buf, const typename tw_of<T>::type* tw) {
    for (int h = 1; h < Fn; h *= 2) {
        for (int e = threadIdx.x; e < (Fn / 2) * C; e += NT) {
            const int c = e % C, b = e / C;
            const int j = b & (h - 1), base = 2 * (b - j);
            const auto w = tw[j * (Fn / (2 * h))];
            const cx<T> wc = {w.x, INV ? -w.y : w.y};
            const cx<T> u = buf[(base + j) * C + c], v = cmul(buf[(base + j + h) * C + c], wc);
            buf[(base + j) * C + c] = u + v;
            buf[(base + j + h) * C + c] = u - v;
        }
        __syncthreads();
    }
}
template <typename T, int Fn, int C, bool INV>
__device__ __forceinline__ void big_fft_dif(cx<T>* buf, const typename tw_of<T>::type* tw) {
    for (int h = Fn / 2; h >= 1; h /= 2) {
        for (int e = threadIdx.x; e < (Fn / 2) * C; e += NT) {
            const int c = e % C, b = e / C;
            const int j = b & (h - 1), base = 2 * (b - j);
            const auto w = tw[j * (Fn / (2 * h))];
            const cx<T> wc = {w.x, INV ? -w.y : w.y};
            const cx<T> u = buf[(base + j) * C + c], v = buf[(base + j + h) * C + c];
            buf[(base + j) * C + c] = u + v;
            buf[(base + j + h) * C + c] = cmul(u - v, wc);
        }
        __syncthreads();
    }
}
template <int BITS>
__device__ __forceinline__ int big_brev(int i) {
    return (int)(__builtin_bitreverse32((uint32_t)i) >> (32 - BITS));
}

struct BigItem {
    Choice c;
    int32_t run;  // 1: the item needs the transforms; 0: its outputs are written already
    int32_t pad;
};

struct BigArgs {
    RunArgs a;
    BigItem* bi;       // one per item
    void* scr;         // MW complex points per item (double2, or float2 for FP32)
    const void* twF1;  // W_F1^t, W_F2^t, W_MW^t, W_2MW^t tables (double2, or float2 for FP32)
    const void* twF2;
    const void* twMW;
    const void* twF;
    const void* H;     // kernel spectrum H'[k] = H[k] / (4 MW), k <= MW
};

// Statistics, choice and the outputs of the items that need no arithmetic.
__global__ void __launch_bounds__(NT) k_big_stats(RunArgs a, BigItem* bi) {
    const int64_t item = blockIdx.x;
    const Item it = make_item(a, item, true);
    const BlockStats st = block_stats(a.s, it.start, it.nwin);
    const Choice c = choose(a, st);
    write_info(a, it, c, st, item < a.P);
    int run = 1;
    if (c.flags & APX_FLAG_NONFINITE) {
        fill_block(a, it, NAN);
        run = 0;
    } else if ((c.flags & APX_FLAG_ZERO) && c.mode != MD_FULL32) {
        fill_block(a, it, 0.0f);
        run = 0;
    } else if (it.j_hi <= it.j_lo) {
        run = 0;
    }
    if (threadIdx.x == 0) {
        bi[item].c = c;
        bi[item].run = run;
    }
}

// Complex point n of the item's packed sequence (as fft_item packs it).
template <int MODE>
__device__ __forceinline__ cx<typename std::conditional<MODE == MD_FULL32, float, double>::type> big_point(
    const RunArgs& a, const Item& it, const Choice& c, int n) {
    if constexpr (MODE == MD_FULL32) {
        const int i0 = 2 * n;
        return {(i0 < it.nvalid) ? a.s[it.start + i0] : 0.0f, (i0 + 1 < it.nvalid) ? a.s[it.start + i0 + 1] : 0.0f};
    } else if constexpr (MODE == MD_SYM) {
        const double eps = 1.0 / (2.0 * (double)c.R);
        const int i0 = 4 * n;
        return {sq_at(a, it, c.cs, i0) + eps * sq_at(a, it, c.cs, i0 + 1),
                sq_at(a, it, c.cs, i0 + 2) + eps * sq_at(a, it, c.cs, i0 + 3)};
    } else {
        constexpr int MM = (MODE == MD_ASYM2) ? 2 : 3;
        const double eps = 1.0 / (2.0 * (double)c.R);
        const bool prefix = it.j_lo == 0;
        const int N = a.N;
        const int Tit = prefix ? (N + 1 + MM - 1) / MM : a.T[MODE];
        const int base_off = it.j_lo - (N - 1);
        const int lw = Tit + N - 1;
        double v[2];
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int m = 2 * n + h;
            double acc = 0.0;
            if (m < lw) {
                double e = 1.0;
#pragma unroll
                for (int q = 0; q < MM; ++q) {
                    acc += e * sq_at(a, it, c.cs, base_off + q * Tit + m);
                    e *= eps;
                }
            }
            v[h] = acc;
        }
        return {v[0], v[1]};
    }
}

// Column passes.  INV = false: pack, DFT over n1, twiddle, store (k1, n2).  INV = true: inverse
// DFT over k1 of (k1, n2), then the words at n = n1 F2 + n2: unpacked (FP32, asymmetric modes)
// or stored back at n (symmetric mode).
template <int MODE, int LOGMW, bool INV>
__global__ void __launch_bounds__(NT) k_big_cols(BigArgs g) {
    using T = typename std::conditional<MODE == MD_FULL32, float, double>::type;
    using T2 = typename tw_of<T>::type;
    constexpr int MW = 1 << LOGMW, L1 = LOGMW / 2, F1 = 1 << L1, F2 = MW / F1, C = BIG_TC;
    static_assert(F2 % C == 0, "whole column tiles");
    const RunArgs& a = g.a;
    const int64_t item = blockIdx.y;
    const BigItem* b = g.bi + item;
    if (!b->run) return;
    const Choice c = b->c;
    const Item it = make_item(a, item, true);
    __shared__ cx<T> buf[F1 * C];
    cx<T>* scr = reinterpret_cast<cx<T>*>(g.scr) + (size_t)item * MW;
    const T2* tw1 = reinterpret_cast<const T2*>(g.twF1);
    const T2* twm = reinterpret_cast<const T2*>(g.twMW);
    const int n2_0 = blockIdx.x * C;
    if constexpr (!INV) {
        for (int e = threadIdx.x; e < F1 * C; e += NT) {
            const int n1 = e / C, cc = e % C;
            buf[big_brev<L1>(n1) * C + cc] = big_point<MODE>(a, it, c, n1 * F2 + n2_0 + cc);
        }
        __syncthreads();
        big_fft_dit<T, F1, C, false>(buf, tw1);
        for (int e = threadIdx.x; e < F1 * C; e += NT) {
            const int k1 = e / C, cc = e % C, n2 = n2_0 + cc;
            const T2 w = twm[k1 * n2];  // W_MW^(k1 n2), k1 n2 < MW
            scr[k1 * F2 + n2] = cmul(buf[k1 * C + cc], cx<T>{w.x, w.y});
        }
    } else {
        for (int e = threadIdx.x; e < F1 * C; e += NT) {
            const int k1 = e / C, cc = e % C;
            buf[k1 * C + cc] = scr[k1 * F2 + n2_0 + cc];
        }
        __syncthreads();
        big_fft_dif<T, F1, C, true>(buf, tw1);
        // position p holds n1 = brev(p)
        if constexpr (MODE == MD_SYM) {
            for (int e = threadIdx.x; e < F1 * C; e += NT) {
                const int p = e / C, cc = e % C;
                scr[big_brev<L1>(p) * F2 + n2_0 + cc] = buf[p * C + cc];
            }
        } else if constexpr (MODE == MD_FULL32) {
            StoreSink sk;
            for (int e = threadIdx.x; e < F1 * C; e += NT) {
                const int p = e / C, cc = e % C;
                const int n = big_brev<L1>(p) * F2 + n2_0 + cc;
                const cx<T> v = buf[p * C + cc];
                if (2 * n >= it.j_lo && 2 * n < it.j_hi) sk.put32(a, it, 2 * n, (float)v.x);
                if (2 * n + 1 >= it.j_lo && 2 * n + 1 < it.j_hi) sk.put32(a, it, 2 * n + 1, (float)v.y);
            }
        } else {
            constexpr int MM = (MODE == MD_ASYM2) ? 2 : 3;
            const int N = a.N;
            const bool prefix = it.j_lo == 0;
            const int Tit = prefix ? (N + 1 + MM - 1) / MM : a.T[MODE];
            const int base_off = it.j_lo - (N - 1);
            const int lw = Tit + N - 1;
            const double two_r = (double)(2 * c.R);
            for (int e = threadIdx.x; e < 2 * F1 * C; e += NT) {
                const int p = e / (2 * C), r = e % (2 * C), cc = r >> 1, h = r & 1;
                const int m = 2 * (big_brev<L1>(p) * F2 + n2_0 + cc) + h;  // word
                if (m < N - 1 || m >= lw) continue;
                const cx<T> v = buf[p * C + cc];
                double x = h ? (double)v.y : (double)v.x;
#pragma unroll
                for (int q = 0; q < MM; ++q) {
                    const double d = rint(x);
                    x = (x - d) * two_r;
                    const int j = base_off + q * Tit + m;
                    if (j >= it.j_lo && j < it.j_hi) put(a, it, j, d, c.inv);
                }
            }
        }
    }
}

// Row pairs: workgroup p takes rows p and F1 - p (p = 1 .. F1/2 - 1), workgroup 0 the rows 0 and
// F1/2, each of which pairs with itself.
template <int MODE, int LOGMW>
__global__ void __launch_bounds__(NT) k_big_rows(BigArgs g) {
    using T = typename std::conditional<MODE == MD_FULL32, float, double>::type;
    using T2 = typename tw_of<T>::type;
    constexpr int MW = 1 << LOGMW, L1 = LOGMW / 2, F1 = 1 << L1, L2 = LOGMW - L1, F2 = 1 << L2;
    const int64_t item = blockIdx.y;
    if (!g.bi[item].run) return;
    const int pr = blockIdx.x;
    const int row[2] = {pr, pr == 0 ? F1 / 2 : F1 - pr};
    __shared__ cx<T> buf[2 * F2];
    cx<T>* scr = reinterpret_cast<cx<T>*>(g.scr) + (size_t)item * MW;
    const T2* tw2 = reinterpret_cast<const T2*>(g.twF2);
    const T2* twm = reinterpret_cast<const T2*>(g.twMW);
    const T2* twF = reinterpret_cast<const T2*>(g.twF);
    const T2* H = reinterpret_cast<const T2*>(g.H);
    for (int e = threadIdx.x; e < 2 * F2; e += NT) {
        const int cc = e / F2, n2 = e % F2;
        buf[big_brev<L2>(n2) * 2 + cc] = scr[row[cc] * F2 + n2];
    }
    __syncthreads();
    big_fft_dit<T, F2, 2, false>(buf, tw2);
    // spectral step (as spectral_step) on the pair (k, MW - k), k the smaller index; element
    // (k2, cc) holds X[row[cc] + F1 k2]
    auto step = [&](int ka, int pa, int kb, int pb) {  // X[ka] at buf[pa], X[kb] at buf[pb], kb = (MW - ka) mod MW
        if (ka > kb) {
            const int t0 = ka, t1 = pa;
            ka = kb;
            pa = pb;
            kb = t0;
            pb = t1;
        }
        const cx<T> za = buf[pa], zb = buf[pb];
        const T2 wt = twF[ka];
        const cx<T> w = {wt.x, wt.y};
        const cx<T> A = za + conj(zb);
        const cx<T> Bd = za - conj(zb);
        const cx<T> wB = cmul(w, Bd);
        const cx<T> x_k = A - mul_i(wB);
        const cx<T> x_mk = conj(A + mul_i(wB));
        const T2 h0 = H[ka], h1 = H[MW - ka];
        const cx<T> yk = cmul(x_k, cx<T>{h0.x, h0.y});
        const cx<T> ymk = cmul(x_mk, cx<T>{h1.x, h1.y});
        const cx<T> P = yk + conj(ymk);
        const cx<T> Q = yk - conj(ymk);
        const cx<T> cQ = mul_i(cmul(conj(w), Q));
        buf[pa] = P + cQ;
        if (ka != 0 && kb != ka) buf[pb] = conj(P - cQ);
    };
    if (pr != 0) {
        // (row A, k2) pairs with (row B, F2 - 1 - k2)
        for (int k2 = threadIdx.x; k2 < F2; k2 += NT)
            step(row[0] + F1 * k2, k2 * 2 + 0, row[1] + F1 * (F2 - 1 - k2), (F2 - 1 - k2) * 2 + 1);
    } else {
        // row 0: (0, k2) with (0, (F2 - k2) mod F2); row F1/2: (F1/2, k2) with (F1/2, F2 - 1 - k2)
        for (int k2 = threadIdx.x; k2 <= F2 / 2; k2 += NT) {
            const int kb2 = (F2 - k2) & (F2 - 1);
            step(F1 * k2, k2 * 2, F1 * kb2, kb2 * 2);
        }
        for (int k2 = threadIdx.x; k2 < F2 / 2; k2 += NT)
            step(F1 / 2 + F1 * k2, k2 * 2 + 1, F1 / 2 + F1 * (F2 - 1 - k2), (F2 - 1 - k2) * 2 + 1);
    }
    __syncthreads();
    big_fft_dif<T, F2, 2, true>(buf, tw2);
    for (int e = threadIdx.x; e < 2 * F2; e += NT) {
        const int cc = e / F2, pp = e % F2;
        const int n2 = big_brev<L2>(pp);
        const int k1 = row[cc];
        const T2 w = twm[k1 * n2];
        scr[k1 * F2 + n2] = cmul(buf[pp * 2 + cc], cx<T>{w.x, -w.y});
    }
}

// Symmetric words at n (re: word 2n, im: word 2n + 1) -> outputs (as sym_unpack_store).
template <int LOGMW>
__global__ void __launch_bounds__(NT) k_big_sym_unpack(BigArgs g) {
    constexpr int MW = 1 << LOGMW;
    const RunArgs& a = g.a;
    const int64_t item = blockIdx.y;
    const BigItem* b = g.bi + item;
    if (!b->run) return;
    const Choice c = b->c;
    const Item it = make_item(a, item, true);
    const cx<double>* scr = reinterpret_cast<const cx<double>*>(g.scr) + (size_t)item * MW;
    auto rbar = [&](int m) -> double {
        if (m < 0) return 0.0;
        const cx<double> v = scr[m >> 1];
        return (m & 1) ? v.y : v.x;
    };
    const double two_r = (double)(2 * c.R), R = (double)c.R, inv_two_r = 1.0 / two_r;
    const int m_lo = it.j_lo >> 1, m_hi = (it.j_hi + 1) >> 1;
    for (int m = m_lo + (int)(blockIdx.x * NT + threadIdx.x); m < m_hi; m += (int)(NT * gridDim.x)) {
        const SymDigits cur = sym_split(rbar(m), two_r, inv_two_r, R);
        const int j0 = 2 * m, j1 = 2 * m + 1;
        if (j0 >= it.j_lo && j0 < it.j_hi) {
            const double de_prev = (m >= 1) ? sym_split(rbar(m - 1), two_r, inv_two_r, R).De : 0.0;
            put(a, it, j0, cur.Dm + de_prev, c.inv);
        }
        if (j1 >= it.j_lo && j1 < it.j_hi) put(a, it, j1, cur.B, c.inv);
    }
}

// H'[k] = (1 / (2F)) sum_n h[n] W_F^(n k), k <= F/2 (direct DFT in FP64, the table W_F^t).
template <typename OUT2>
__global__ void __launch_bounds__(NT) k_big_spectrum(const double* __restrict__ h, int32_t nh, int32_t F,
                                                     const double2* __restrict__ twF, OUT2* spec) {
    const int k = blockIdx.x * NT + threadIdx.x;
    if (k > F / 2) return;
    double re = 0.0, im = 0.0;
    int idx = 0;
    for (int n = 0; n < nh; ++n) {
        const double2 w = twF[idx];
        re = fma(h[n], w.x, re);
        im = fma(h[n], w.y, im);
        idx += k;
        if (idx >= F) idx -= F;
    }
    const double sc = 1.0 / (2.0 * (double)F);
    if constexpr (std::is_same<OUT2, double2>::value) spec[k] = make_double2(re * sc, im * sc);
    else spec[k] = make_float2((float)(re * sc), (float)(im * sc));
}

hipError_t launch_big_spectrum(const double* h, int32_t nh, int32_t F, const double2* twF, void* spec, bool fp32,
                               hipStream_t st) {
    const unsigned grid = (unsigned)((F / 2 + 1 + NT - 1) / NT);
    if (fp32) hipLaunchKernelGGL(k_big_spectrum<float2>, dim3(grid), dim3(NT), 0, st, h, nh, F, twF, (float2*)spec);
    else hipLaunchKernelGGL(k_big_spectrum<double2>, dim3(grid), dim3(NT), 0, st, h, nh, F, twF, (double2*)spec);
    return hipGetLastError();
}

bool big_supported(int logmw, bool fp32) {
    return logmw >= BIG_LOGMW_MIN && logmw <= (fp32 ? BIG_LOGMW_MAX_FP32 : BIG_LOGMW_MAX);
}

template <int MODE, int LOGMW>
static hipError_t big_run(const BigArgs& g, hipStream_t st) {
    constexpr int L1 = LOGMW / 2, F1 = 1 << L1, F2 = (1 << LOGMW) / F1;
    const unsigned items = (unsigned)g.a.nitems;
    hipLaunchKernelGGL(k_big_stats, dim3(items), dim3(NT), 0, st, g.a, g.bi);
    hipLaunchKernelGGL((k_big_cols<MODE, LOGMW, false>), dim3(F2 / BIG_TC, items), dim3(NT), 0, st, g);
    hipLaunchKernelGGL((k_big_rows<MODE, LOGMW>), dim3(F1 / 2, items), dim3(NT), 0, st, g);
    hipLaunchKernelGGL((k_big_cols<MODE, LOGMW, true>), dim3(F2 / BIG_TC, items), dim3(NT), 0, st, g);
    if constexpr (MODE == MD_SYM)
        hipLaunchKernelGGL((k_big_sym_unpack<LOGMW>), dim3(16, items), dim3(NT), 0, st, g);
    return hipGetLastError();
}

hipError_t launch_big(const RunArgs& a, int mode, int logmw, void* bi, void* scr, const void* twF1,
                      const void* twF2, const void* twMW, const void* twF, const void* H, hipStream_t st) {
    if (a.nitems > 65535) return hipErrorInvalidValue;  // items run along grid y
    BigArgs g;
    g.a = a;
    g.bi = reinterpret_cast<BigItem*>(bi);
    g.scr = scr;
    g.twF1 = twF1;
    g.twF2 = twF2;
    g.twMW = twMW;
    g.twF = twF;
    g.H = H;
#define APX_BIG(L_)                                                  \
    case L_:                                                         \
        switch (mode) {                                              \
            case MD_FULL32: return big_run<MD_FULL32, L_>(g, st);    \
            case MD_SYM: return big_run<MD_SYM, L_>(g, st);          \
            case MD_ASYM2: return big_run<MD_ASYM2, L_>(g, st);      \
            case MD_ASYM3: return big_run<MD_ASYM3, L_>(g, st);      \
            default: return hipErrorInvalidValue;                    \
        }
    switch (logmw) {
        APX_BIG(10)
        APX_BIG(11)
        APX_BIG(12)
        APX_BIG(13)
        APX_BIG(14)
        APX_BIG(15)
        case 16:  // FP32 only: 256 x 256 points, 32 KB of LDS per column tile
            if (mode == MD_FULL32) return big_run<MD_FULL32, 16>(g, st);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
#undef APX_BIG
}

size_t big_item_bytes() { return sizeof(BigItem); }

// Fixed symmetric or FP32 items of the batched kernel read their window once: point n =
// threadIdx.x + NT k holds samples SPP n .. SPP n + SPP - 1 of the window in registers (zero at
// or past nwin); the block statistics are taken from them and the packed words are written from
// them (block_stats + the packing of fft_item, with one read of the window instead of two).
template <int MODE, int MW>
struct WinRegs {
    static constexpr int SPP = MODE == MD_SYM ? 4 : 2;  // samples per complex point
    static constexpr int PPT = MW / NT;                 // points per thread (at most 64 samples)
    static_assert(MW % NT == 0, "points must fill the threads");
    float x[PPT][SPP];
};

template <int MODE, int MW>
__device__ BlockStats window_regs(const RunArgs& a, const Item& it, WinRegs<MODE, MW>& wr) {
    using R = WinRegs<MODE, MW>;
    __shared__ double red_m[NT / 64], red_s[NT / 64];
    __shared__ int red_f[NT / 64];
    const float* sp = a.s + it.start;
    if (R::SPP * MW <= it.nwin && (reinterpret_cast<uintptr_t>(sp) & 7) == 0) {
        const float2* s2 = reinterpret_cast<const float2*>(sp);
#pragma unroll
        for (int k = 0; k < R::PPT; ++k) {
            const int n = threadIdx.x + NT * k;
#pragma unroll
            for (int h = 0; h < R::SPP / 2; ++h) {
                const float2 v = s2[(R::SPP / 2) * n + h];
                wr.x[k][2 * h] = v.x;
                wr.x[k][2 * h + 1] = v.y;
            }
        }
    } else {
#pragma unroll
        for (int k = 0; k < R::PPT; ++k) {
            const int n = threadIdx.x + NT * k;
#pragma unroll
            for (int h = 0; h < R::SPP; ++h) {
                const int i = R::SPP * n + h;
                wr.x[k][h] = (i < it.nwin) ? sp[i] : 0.0f;
            }
        }
    }
    double m = 0.0, q = 0.0;
    int nf = 0;
#pragma unroll
    for (int k = 0; k < R::PPT; ++k) {
#pragma unroll
        for (int h = 0; h < R::SPP; ++h) {
            const float v = wr.x[k][h];
            if (!isfinite(v)) {
                nf = 1;
            } else {
                const double d = (double)v;
                m = fmax(m, fabs(d));
                q += d * d;
            }
        }
    }
    m = wave_max(m);
    q = wave_sum(q);
    nf = wave_or(nf);
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red_m[wv] = m;
        red_s[wv] = q;
        red_f[wv] = nf;
    }
    __syncthreads();
    BlockStats r;
    r.smax = red_m[0];
    r.sumsq = red_s[0];
    r.nonfinite = red_f[0];
#pragma unroll
    for (int i = 1; i < NT / 64; ++i) {
        r.smax = fmax(r.smax, red_m[i]);
        r.sumsq += red_s[i];
        r.nonfinite |= red_f[i];
    }
    __syncthreads();
    return r;
}

// The packed words of fft_item from the registers: samples at or past nvalid are zero.
template <int MODE, int MW>
__device__ void pack_regs(const Item& it, const Choice& c, const WinRegs<MODE, MW>& wr, char* lds) {
    using R = WinRegs<MODE, MW>;
    using T = typename std::conditional<MODE == MD_FULL32, float, double>::type;
    T* re = (T*)lds;
    T* im = re + MW;
    const bool full = R::SPP * MW <= it.nvalid;
#pragma unroll
    for (int k = 0; k < R::PPT; ++k) {
        const int n = threadIdx.x + NT * k;
        float v[R::SPP];
#pragma unroll
        for (int h = 0; h < R::SPP; ++h) v[h] = (full || R::SPP * n + h < it.nvalid) ? wr.x[k][h] : 0.0f;
        if constexpr (MODE == MD_FULL32) {
            re[n] = v[0];
            im[n] = v[1];
        } else {
            const double eps = 1.0 / (2.0 * (double)c.R), cs = c.cs;
            re[n] = rint(cs * (double)v[0]) + eps * rint(cs * (double)v[1]);
            im[n] = rint(cs * (double)v[2]) + eps * rint(cs * (double)v[3]);
        }
    }
}

// The symmetric packed points of pack_regs kept in registers: point threadIdx.x + NT k in v[k].
template <int MW>
__device__ void pack_regs_points(const Item& it, const Choice& c, const WinRegs<MD_SYM, MW>& wr, cx<double>* v) {
    using R = WinRegs<MD_SYM, MW>;
    const bool full = R::SPP * MW <= it.nvalid;
    const double eps = 1.0 / (2.0 * (double)c.R), cs = c.cs;
#pragma unroll
    for (int k = 0; k < R::PPT; ++k) {
        const int n = threadIdx.x + NT * k;
        float x[R::SPP];
#pragma unroll
        for (int h = 0; h < R::SPP; ++h) x[h] = (full || R::SPP * n + h < it.nvalid) ? wr.x[k][h] : 0.0f;
        v[k] = {rint(cs * (double)x[0]) + eps * rint(cs * (double)x[1]),
                rint(cs * (double)x[2]) + eps * rint(cs * (double)x[3])};
    }
}

// ------------------------------------------------------------------------------------------
// Batched cross-correlation matching: one persistent launch over a work list of (pair, block)
// items.  Each workgroup takes `chunk` consecutive items at a time from a global counter, runs
// the FFT core on each (same steps as k_fft, per pair arguments from `targs`) and folds the
// block's outputs into the pair's argmax key with one atomic max per wave.
// ------------------------------------------------------------------------------------------
__device__ __forceinline__ unsigned long long wave_umax64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned int lo = __shfl_xor((unsigned int)v, o);
        const unsigned int hi = __shfl_xor((unsigned int)(v >> 32), o);
        const unsigned long long w = ((unsigned long long)hi << 32) | lo;
        v = w > v ? w : v;
    }
    return v;
}

// two waves per SIMD wherever the LDS of one item lets two workgroups share a CU (measured 1.65x
// on the symmetric 2^13 length: the latency of one item's passes is hidden by the other's)
template <int MODE, int LOGW>
__global__ void __launch_bounds__(NT, (MODE == MD_FULL32 ? LOGW <= 14 : LOGW <= 13) ? 2 : 1)
    k_batch(const RunArgs* __restrict__ targs, const int2* __restrict__ items,
                                              int32_t nitems, int32_t chunk, unsigned int* counter,
                                              unsigned long long* keys) {
    constexpr int MW = 1 << (LOGW - 1);  // complex points: 2^LOGW packed words
    extern __shared__ __attribute__((aligned(16))) char lds[];
    __shared__ int grab;
    for (;;) {
        __syncthreads();  // everyone has read `grab` and is done with the LDS
        if (threadIdx.x == 0) grab = (int)atomicAdd(counter, (unsigned int)chunk);
        __syncthreads();
        const int base = __builtin_amdgcn_readfirstlane(grab);
        if (base >= nitems) break;
        const int end = min(base + chunk, nitems);
        for (int idx = base; idx < end; ++idx) {
            const int2 ti = items[idx];
            const int t = __builtin_amdgcn_readfirstlane(ti.x);
            const int w = __builtin_amdgcn_readfirstlane(ti.y);
            // symmetric: the pair table through the constant address space, its fields read once
            // and its data pointers taken as device memory (global loads; measured 13.2 -> 12.8
            // ms).  The other modes keep generic reads: there the scalar copies cost registers
            // that the transforms need (FP32 17.4 -> 21.8 ms with spills)
            const RunArgs& a = MODE == MD_SYM
                                   ? *(const RunArgs*)((__attribute__((address_space(4))) const RunArgs*)targs + t)
                                   : targs[t];
            ArgmaxSink sk;
            const Item it = make_item(a, w, true);
            if constexpr ((MODE == MD_SYM || MODE == MD_FULL32) && WinRegs<MODE, MW>::PPT * WinRegs<MODE, MW>::SPP <= 64) {
                WinRegs<MODE, MW> wr;
                const BlockStats st = window_regs<MODE, MW>(a, it, wr);
                const Choice c = choose(a, st);
                if (!(c.flags & APX_FLAG_NONFINITE) && it.j_hi > it.j_lo) {
                    if ((c.flags & APX_FLAG_ZERO) && MODE != MD_FULL32) {
                        sk.consider(it.o0, 0.0f);  // all outputs of the block are zero
                    } else {
                        if constexpr (MODE == MD_SYM && MW == 16 * NT) {
                            // the FP64 transform runs in registers: the packed points go straight in
                            cx<double> v[16];
                            pack_regs_points<MW>(it, c, wr, v);
                            group_fft_regs<16, false>(v, (double*)lds, (double*)lds + MW, a.twd + 2 * MW);
                            fft_item_tail<MODE, MW>(a, it, c, lds, sk);
                        } else {
                            pack_regs<MODE, MW>(it, c, wr, lds);
                            fft_item<MODE, MW, true>(a, it, c, lds, sk);
                        }
                    }
                }
            } else {
                const BlockStats st = block_stats(a.s, it.start, it.nwin);
                const Choice c = choose(a, st);
                if (!(c.flags & APX_FLAG_NONFINITE) && it.j_hi > it.j_lo) {
                    if ((c.flags & APX_FLAG_ZERO) && MODE != MD_FULL32)
                        sk.consider(it.o0, 0.0f);  // all outputs of the block are zero
                    else
                        fft_item<MODE, MW>(a, it, c, lds, sk);
                }
            }
            const unsigned long long k = wave_umax64(sk.key());
            if ((threadIdx.x & 63) == 0 && k != 0) atomicMax(&keys[t], k);
            __syncthreads();
        }
    }
}

__global__ void __launch_bounds__(NT) k_batch_init(unsigned int* counter, unsigned long long* keys, int32_t n) {
    const int i = blockIdx.x * NT + threadIdx.x;
    if (i == 0) *counter = 0u;
    if (i < n) keys[i] = 0ull;
}

// keys -> (lag, value); lag = r_out index - (N - 1).  No finite output: lag INT64_MIN, value NaN.
__global__ void __launch_bounds__(NT) k_batch_final(const unsigned long long* __restrict__ keys,
                                                    const int32_t* __restrict__ Ngiven, int32_t n, int64_t* lag,
                                                    float* val) {
    const int i = blockIdx.x * NT + threadIdx.x;
    if (i >= n) return;
    const unsigned long long k = keys[i];
    if (k == 0ull) {
        lag[i] = INT64_MIN;
        val[i] = NAN;
        return;
    }
    const unsigned int u = (unsigned int)(k >> 32);
    const unsigned int o = 0xFFFFFFFFu - (unsigned int)(k & 0xFFFFFFFFull);
    const unsigned int b = (u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u;
    lag[i] = (int64_t)o - (int64_t)(Ngiven[i] - 1);
    val[i] = __uint_as_float(b);
}

size_t batch_lds_bytes(int mode, int logW) {
    return fft_lds_bytes(mode != MD_FULL32, 1 << (logW - 1));  // 2^(LOGW-1) complex points
}

namespace {
template <int MODE, int LOGW>
hipError_t batch_one(const BatchLaunch& b, bool query, int* per_cu) {
    auto kern = k_batch<MODE, LOGW>;
    const size_t lds = batch_lds_bytes(MODE, LOGW);
    if (query) {
        // sets the LDS limit once, before any launch (launches may be captured into a graph)
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kern, NT, lds);
    }
    hipLaunchKernelGGL(kern, dim3(b.grid), dim3(NT), lds, b.st, b.targs, b.items, b.nitems, b.chunk, b.counter,
                       b.keys);
    return hipGetLastError();
}

template <int MODE>
hipError_t batch_mode(const BatchLaunch& b, bool query, int* per_cu) {
    switch (b.logW) {
        case 11: return batch_one<MODE, 11>(b, query, per_cu);
        case 12: return batch_one<MODE, 12>(b, query, per_cu);
        case 13: return batch_one<MODE, 13>(b, query, per_cu);
        case 14: return batch_one<MODE, 14>(b, query, per_cu);
        default: return hipErrorInvalidValue;
    }
}

hipError_t batch_dispatch(const BatchLaunch& b, bool query, int* per_cu) {
    switch (b.mode) {
        case MD_FULL32: return batch_mode<MD_FULL32>(b, query, per_cu);
        case MD_SYM: return batch_mode<MD_SYM>(b, query, per_cu);
        case MD_ASYM2: return batch_mode<MD_ASYM2>(b, query, per_cu);
        case MD_ASYM3: return batch_mode<MD_ASYM3>(b, query, per_cu);
        default: return hipErrorInvalidValue;
    }
}
}  // namespace

hipError_t batch_occupancy(int mode, int logW, int* per_cu) {
    BatchLaunch b{};
    b.mode = mode;
    b.logW = logW;
    return batch_dispatch(b, true, per_cu);
}

hipError_t launch_batch(const BatchLaunch& b) {
    const int nb = (b.npairs + NT - 1) / NT;
    hipLaunchKernelGGL(k_batch_init, dim3(nb > 0 ? nb : 1), dim3(NT), 0, b.st, b.counter, b.keys, b.npairs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (b.nitems > 0) {
        e = batch_dispatch(b, false, nullptr);
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_batch_final, dim3(nb > 0 ? nb : 1), dim3(NT), 0, b.st, b.keys, b.Ngiven, b.npairs, b.lag,
                       b.val);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Kernel preparation (Section IV "Initialization": ||k||_inf, eq. 2 on k, eq. 5)
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) k_prepare(const float* __restrict__ k_in, int32_t Ng, int32_t N, int32_t reverse,
                                                KState* ks, float* kf, double* kd, int32_t kf_pad, double* kq1,
                                                double* kq2, double* kq3, int32_t K1, int32_t K2, int32_t K3,
                                                int64_t R1, int32_t kq1_pad, int32_t kq23_pad) {
    __shared__ double s_kmax, s_ss;
    __shared__ int s_nf;
    // the taps as used: reversed for correlation, one zero appended for an even count
    auto tap = [&](int n) -> float {
        if (n >= Ng) return 0.0f;
        return reverse ? k_in[Ng - 1 - n] : k_in[n];
    };
    BlockStats st = block_stats(k_in, 0, Ng);
    if (threadIdx.x == 0) {
        s_kmax = st.smax;
        s_ss = st.sumsq;
        s_nf = st.nonfinite;
    }
    __syncthreads();
    const double kmax = s_kmax;
    const int Kq[4] = {0, K1, K2, K3};
    double ck[4] = {0.0, 0.0, 0.0, 0.0};
    for (int m = 1; m < 4; ++m) ck[m] = (kmax == 0.0 || Kq[m] == 0) ? 0.0 : (double)Kq[m] / kmax;
    if (threadIdx.x == 0) {
        ks->kmax = kmax;
        ks->krms = sqrt(s_ss / (double)Ng);
        for (int m = 0; m < 4; ++m) ks->ck[m] = ck[m];
        ks->nonfinite = s_nf;
        ks->pad = 0;
    }
    for (int n = threadIdx.x; n < kf_pad; n += NT) {
        float v = (n < N) ? tap(n) : 0.0f;
        kf[n] = v;
        kd[n] = (double)v;
    }
    // companded taps (eq. 2) for the asymmetric modes, FP64 holding exact integers
    for (int n = threadIdx.x; n < kq23_pad; n += NT) {
        double v = (n < N) ? (double)tap(n) : 0.0;
        if (kq2) kq2[n] = (n < N) ? rint(ck[2] * v) : 0.0;
        if (kq3) kq3[n] = (n < N) ? rint(ck[3] * v) : 0.0;
    }
    // symmetric packed taps (eq. 5 for convolution): k-[n] = k~[2n+1] + 2R k~[2n]
    if (kq1) {
        const double two_r = (double)(2 * R1);
        const int nk = (N + 1) / 2;
        for (int n = threadIdx.x; n < kq1_pad; n += NT) {
            double v = 0.0;
            if (n < nk) {
                double e = rint(ck[1] * (double)tap(2 * n));
                double o = (2 * n + 1 < N) ? rint(ck[1] * (double)tap(2 * n + 1)) : 0.0;
                v = o + two_r * e;
            }
            kq1[n] = v;
        }
    }
}

hipError_t launch_prepare_kernel(const float* k_in, int32_t Ng, int32_t N, int32_t reverse, KState* ks, float* kf,
                                 double* kd, int32_t kf_pad, double* kq1, double* kq2, double* kq3, const int32_t* K,
                                 const int64_t* R, int32_t kq1_pad, int32_t kq23_pad, hipStream_t st) {
    hipLaunchKernelGGL(k_prepare, dim3(1), dim3(NT), 0, st, k_in, Ng, N, reverse, ks, kf, kd, kf_pad, kq1, kq2, kq3,
                       K[1], K[2], K[3], R[1], kq1_pad, kq23_pad);
    return hipGetLastError();
}

// Spectrum of a real tap sequence (zero padded to F words), prescaled for spectral_step.
template <typename T, int MW>
__global__ void __launch_bounds__(NT) k_spectrum(const T* __restrict__ taps, int32_t ntaps,
                                                 const typename tw_of<T>::type* tw,
                                                 typename tw_of<T>::type* spec) {
    extern __shared__ __attribute__((aligned(16))) char sp_lds[];
    T* re = (T*)sp_lds;
    T* im = re + MW;
    for (int n = threadIdx.x; n < MW; n += NT) {
        re[n] = (2 * n < ntaps) ? taps[2 * n] : (T)0;
        im[n] = (2 * n + 1 < ntaps) ? taps[2 * n + 1] : (T)0;
    }
    __syncthreads();
    fft_lds<T, MW, false>(re, im, tw);
    real_spectrum_out<T, MW>(re, im, tw, spec);
}

template <typename T, int MW>
hipError_t spectrum_one(const T* taps, int32_t ntaps, const typename tw_of<T>::type* tw,
                        typename tw_of<T>::type* spec, hipStream_t st) {
    auto kern = k_spectrum<T, MW>;
    const size_t lds = fft_lds_bytes(std::is_same<T, double>::value, MW);
    hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kern, dim3(1), dim3(NT), lds, st, taps, ntaps, tw, spec);
    return hipGetLastError();
}

template <typename T>
hipError_t spectrum_any(const T* taps, int32_t ntaps, int32_t Fw, const typename tw_of<T>::type* tw,
                        typename tw_of<T>::type* spec, hipStream_t st) {
    switch (Fw) {
        case 256: return spectrum_one<T, 128>(taps, ntaps, tw, spec, st);
        case 512: return spectrum_one<T, 256>(taps, ntaps, tw, spec, st);
        case 1024: return spectrum_one<T, 512>(taps, ntaps, tw, spec, st);
        case 2048: return spectrum_one<T, 1024>(taps, ntaps, tw, spec, st);
        case 4096: return spectrum_one<T, 2048>(taps, ntaps, tw, spec, st);
        case 8192: return spectrum_one<T, 4096>(taps, ntaps, tw, spec, st);
        case 16384: return spectrum_one<T, 8192>(taps, ntaps, tw, spec, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_spectrum(const double* taps, int32_t ntaps, int32_t Fw, const double2* twd, double2* spec,
                           hipStream_t st) {
    return spectrum_any<double>(taps, ntaps, Fw, twd + Fw, spec, st);
}

hipError_t launch_spectrum32(const float* taps, int32_t ntaps, int32_t Fw, const float2* twf, float2* spec,
                             hipStream_t st) {
    return spectrum_any<float>(taps, ntaps, Fw, twf + Fw, spec, st);
}

// ------------------------------------------------------------------------------------------
// Calibration (Section IV.D): on one block, sum r_ref^2 and sum (r_q - r_ref)^2 over its kept
// outputs, r_ref the FP64 block convolution, r_q the companded one at S_q = K_q = Q.
// Workgroup g handles outputs g, g + G, ... and writes its two partial sums to partial[2g..].
// ------------------------------------------------------------------------------------------
__global__ void __launch_bounds__(NT) k_calib(RunArgs a, int64_t block, int32_t Q, double* partial) {
    const Item it = make_item(a, block, false);
    const BlockStats st = block_stats(a.s, it.start, it.nwin);
    const KState ks = *a.ks;
    const double cs = st.smax == 0.0 ? 0.0 : (double)Q / st.smax;
    const double ck = ks.kmax == 0.0 ? 0.0 : (double)Q / ks.kmax;
    double pr = 0.0, pe = 0.0;
    const int G = gridDim.x;
    for (int j = it.j_lo + blockIdx.x * NT + threadIdx.x; j < it.j_hi; j += G * NT) {
        double rr = 0.0, rq = 0.0;
        for (int n = 0; n < a.N; ++n) {
            const int i = j - n;
            if (i < 0 || i >= it.nvalid) continue;
            const double x = (double)a.s[it.start + i];
            const double k = a.kd[n];
            rr = fma(x, k, rr);
            rq = fma(rint(cs * x), rint(ck * k), rq);
        }
        const double r = (cs == 0.0 || ck == 0.0) ? 0.0 : rq / (cs * ck);
        pr += rr * rr;
        pe += (r - rr) * (r - rr);
    }
    __shared__ double sp[NT / 64], se[NT / 64];
    pr = wave_sum(pr);
    pe = wave_sum(pe);
    if ((threadIdx.x & 63) == 0) {
        sp[threadIdx.x >> 6] = pr;
        se[threadIdx.x >> 6] = pe;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a0 = 0.0, a1 = 0.0;
        for (int i = 0; i < NT / 64; ++i) {
            a0 += sp[i];
            a1 += se[i];
        }
        partial[2 * blockIdx.x] = a0;
        partial[2 * blockIdx.x + 1] = a1;
        if (blockIdx.x == 0) {
            partial[2 * G] = st.smax;
            partial[2 * G + 1] = a.sigma_s > 0.0 ? a.sigma_s : sqrt(st.sumsq / (double)a.W_block);
        }
    }
}

// Calibration workspace of apx_run_auto_noalloc, in the library's own device memory for callers
// that cannot allocate.  Each device holds one copy for the life of the process, shared by every
// call on that device.  Host code must not pass `scratch` itself to a kernel (in host code the
// name stands for a host-side placeholder): noalloc_scratch gives its device address.
constexpr size_t NOALLOC_SCRATCH_BYTES = 2048;
static __device__ __align__(256) char scratch[NOALLOC_SCRATCH_BYTES];

// Device address of this device's scratch (call with the device current).
hipError_t noalloc_scratch(void** ptr, size_t* bytes) {
    *bytes = NOALLOC_SCRATCH_BYTES;
    return hipGetSymbolAddress(ptr, HIP_SYMBOL(scratch));
}

hipError_t launch_calib(const RunArgs& a, int64_t block, int32_t Q, double* partial, int32_t nparts, hipStream_t st) {
    hipLaunchKernelGGL(k_calib, dim3(nparts), dim3(NT), 0, st, a, block, Q, partial);
    return hipGetLastError();
}

// Same arithmetic as the host side of apx_calibrate, in the same order.  A block without
// quantization error or without signal gives offset 0 (the model alone).
__global__ void k_calib_finish(const double* __restrict__ partial, int32_t nparts, const KState* __restrict__ ks,
                               int32_t Q, double* out, double krms_override, double snr_min_db) {
    if (threadIdx.x != 0) return;
    double pr = 0.0, pe = 0.0;
    for (int i = 0; i < nparts; ++i) {
        pr += partial[2 * i];
        pe += partial[2 * i + 1];
    }
    const double smax = partial[2 * nparts], rms = partial[2 * nparts + 1];
    const double kmax = ks->kmax, krms = ks->krms > 0.0 && krms_override > 0.0 ? krms_override : ks->krms;
    double off = 0.0;
    if (pe > 0.0 && pr > 0.0 && rms > 0.0 && krms > 0.0) {
        const double measured = 10.0 * log10(pr / pe);
        const double r12 = sqrt(12.0);
        const double svs = smax / (Q * r12), svk = kmax / (Q * r12);
        const double D = (rms * svk) * (rms * svk) + (krms * svs) * (krms * svs) + (svk * svs) * (svk * svs);
        const double model = 10.0 * log10((rms * krms) * (rms * krms) / D);
        off = measured - model;
    }
    out[0] = off;
    out[1] = pow(10.0, (snr_min_db - off) / 10.0);  // the ratio a candidate's model must reach
}

hipError_t launch_calib_finish(const double* partial, int32_t nparts, const KState* ks, int32_t Q, double* out,
                               double krms_override, double snr_min_db, hipStream_t st) {
    hipLaunchKernelGGL(k_calib_finish, dim3(1), dim3(64), 0, st, partial, nparts, ks, Q, out, krms_override, snr_min_db);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Marginal-CDF fit of a source's samples (Section IV.D, Fig. 4): one workgroup of 1024 threads
// runs the whole fit.  Laplacian (zero mean): b = mean |x|.  Weibull (positive samples): the
// shape kappa solves sum(y^k ln y) / sum(y^k) - 1/k - mean(ln y) = 0 (lambda profiled out), by
// Newton's method from the moment start pi / (sqrt 6 sd(ln y)), with y = x / max(x); then
// lambda = max(x) (mean y^kappa)^(1/kappa).  sigma: square root of the fitted second moment.
// ------------------------------------------------------------------------------------------
constexpr int FIT_NT = 1024;

// sums of three values over the workgroup; every thread gets the totals
__device__ __forceinline__ void fit_sum3(double& a, double& b, double& c, double* red) {
    a = wave_sum(a);
    b = wave_sum(b);
    c = wave_sum(c);
    const int w = threadIdx.x >> 6;
    __syncthreads();  // red is reused by consecutive calls
    if ((threadIdx.x & 63) == 0) {
        red[3 * w] = a;
        red[3 * w + 1] = b;
        red[3 * w + 2] = c;
    }
    __syncthreads();
    a = b = c = 0.0;
    for (int i = 0; i < FIT_NT / 64; ++i) {
        a += red[3 * i];
        b += red[3 * i + 1];
        c += red[3 * i + 2];
    }
}

__global__ void __launch_bounds__(FIT_NT) k_fit_marginal(const float* __restrict__ x, int64_t n, int32_t model,
                                                         double* out) {
    __shared__ double red[3 * (FIT_NT / 64)];
    if (model == 0) {
        double s = 0.0, z0 = 0.0, z1 = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += FIT_NT) s += fabs((double)x[i]);
        fit_sum3(s, z0, z1, red);
        if (threadIdx.x == 0) {
            const double b = s / (double)n;
            out[0] = b;
            out[1] = 1.0;
            out[2] = sqrt(2.0) * b;
            out[3] = (double)n;
        }
        return;
    }
    // positive samples: count and maximum
    double cnt = 0.0, mx = 0.0, z1 = 0.0, z2 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += FIT_NT) {
        const double v = (double)x[i];
        if (v > 0.0) {
            cnt += 1.0;
            mx = fmax(mx, v);
        }
    }
    {
        // the maximum: a reduction of its own
        double m = mx;
        for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o));
        const int w = threadIdx.x >> 6;
        if ((threadIdx.x & 63) == 0) red[w] = m;
        __syncthreads();
        mx = 0.0;
        for (int i = 0; i < FIT_NT / 64; ++i) mx = fmax(mx, red[i]);
        __syncthreads();
    }
    fit_sum3(cnt, z1, z2, red);
    if (cnt < 2.0) {
        if (threadIdx.x == 0) {
            out[0] = 0.0;
            out[1] = 1.0;
            out[2] = 0.0;
            out[3] = cnt;
        }
        return;
    }
    // mean and spread of ln y
    double s1 = 0.0, s2 = 0.0, s3 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += FIT_NT) {
        const double v = (double)x[i];
        if (v > 0.0) {
            const double ly = log(v / mx);
            s1 += ly;
            s2 += ly * ly;
        }
    }
    fit_sum3(s1, s2, s3, red);
    const double mly = s1 / cnt;
    const double var = fmax(s2 / cnt - mly * mly, 0.0);
    double k = var > 0.0 ? 3.14159265358979323846 / (sqrt(6.0) * sqrt(var)) : 1.0;
    for (int it = 0; it < 200; ++it) {
        double a0 = 0.0, a1 = 0.0, a2 = 0.0;
        for (int64_t i = threadIdx.x; i < n; i += FIT_NT) {
            const double v = (double)x[i];
            if (v > 0.0) {
                const double ly = log(v / mx);
                const double yk = exp(k * ly);
                a0 += yk;
                a1 += yk * ly;
                a2 += yk * ly * ly;
            }
        }
        fit_sum3(a0, a1, a2, red);
        const double g = a1 / a0 - 1.0 / k - mly;
        const double dg = (a2 * a0 - a1 * a1) / (a0 * a0) + 1.0 / (k * k);
        double kn = k - g / dg;
        if (kn <= 0.0) kn = 0.5 * k;
        const bool done = fabs(kn - k) <= 1e-13 * k;  // same value in every thread
        k = kn;
        if (done) break;
    }
    double a0 = 0.0, d1 = 0.0, d2 = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += FIT_NT) {
        const double v = (double)x[i];
        if (v > 0.0) a0 += exp(k * log(v / mx));
    }
    fit_sum3(a0, d1, d2, red);
    if (threadIdx.x == 0) {
        const double lam = mx * pow(a0 / cnt, 1.0 / k);
        out[0] = lam;
        out[1] = k;
        out[2] = lam * sqrt(tgamma(1.0 + 2.0 / k));
        out[3] = cnt;
    }
}

hipError_t launch_fit_marginal(const float* x, int64_t n, int32_t model, double* out, hipStream_t st) {
    hipLaunchKernelGGL(k_fit_marginal, dim3(1), dim3(FIT_NT), 0, st, x, n, model, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------------------------------
// Integer matrix-core core.  The companded block convolution r~ = s~ * k~ (eq. 2 applied to
// both operands: the integers every packing of Section III carries) is computed exactly with
// int8 MFMA and int32 accumulation, then dequantized by eq. (16).  There is no FP64 packing:
// this is another Tier-2 convolution under the same companding, and its outputs equal those of
// the packed cores wherever their unpacking is exact.
// One block is a Toeplitz product.  Output m = m0 + 32 i + j (tile row i, column j < 32):
//   r~[m] = sum_kappa A[i][kappa] B[kappa][j],  A[i][kappa] = s~[m0 + 32 i + kappa - (N - 1)],
//   B[kappa][j] = k~[j - kappa + N - 1] (zero outside the taps), kappa < 32 ksteps, ksteps =
//   ceil((N + 31) / 32).
// An operand wider than int8 (S_q or K_q above 127) is split into balanced base-128 digits,
// v = 128 hi + lo with lo in [-64, 63]; the digit products are summed in int32 (exact for any
// N below 2^17) and joined in int64.
// ------------------------------------------------------------------------------------------
typedef int i8x16 __attribute__((ext_vector_type(4)));   // 16 int8 per lane
typedef int i32x16 __attribute__((ext_vector_type(16)));
// device-memory views of the signal, output and debug pointers: global (not flat) loads and
// stores, and copies taken once, since a store through a generic pointer could in the
// compiler's view rewrite a signal's arguments in the multi-signal table
typedef __attribute__((address_space(1))) const float gcfloat;
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(1))) const f32x2 gcf32x2;
typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) double gdouble;

constexpr int I8_TILE = 1024;  // outputs per 32 x 32 tile

__device__ __forceinline__ void i8_digits(int v, bool split, int& lo, int& hi) {
    if (split) {
        hi = (v + 64) >> 7;  // floor((v + 64) / 128): arithmetic shift
        lo = v - hi * 128;
    } else {
        hi = 0;
        lo = v;
    }
}

// B fragments, [plane][k-step][lane] x 16 bytes: plane 0 the low digits (or the value), plane 1
// the high digits.  Lane l holds column l % 32 and kappa = 32 s + 16 (l / 32) + byte; A uses the
// same kappa for the same (lane half, byte), so the k order the hardware assigns is immaterial.
__global__ void __launch_bounds__(NT) k_i8_frag(const float* __restrict__ kf, const KState* __restrict__ ks,
                                                int mode, int N, int ksteps, int split, i8x16* __restrict__ frag) {
    const double ck = ks->ck[mode];
    const int n = 2 * ksteps * 64;
    for (int f = blockIdx.x * NT + threadIdx.x; f < n; f += gridDim.x * NT) {
        const int plane = f / (ksteps * 64);
        const int s = (f / 64) % ksteps;
        const int l = f % 64;
        int w[4] = {0, 0, 0, 0};
        for (int b = 0; b < 16; ++b) {
            const int kappa = 32 * s + 16 * (l >> 5) + b;
            const int t = (l & 31) - kappa + N - 1;
            const int v = (t >= 0 && t < N) ? (int)rint(ck * (double)kf[t]) : 0;  // eq. (2), as k_prepare
            int lo, hi;
            i8_digits(v, split != 0, lo, hi);
            w[b >> 2] |= ((plane ? hi : lo) & 255) << (8 * (b & 3));
        }
        i8x16 r;
        r.x = w[0];
        r.y = w[1];
        r.z = w[2];
        r.w = w[3];
        frag[f] = r;
    }
}

// One wavefront per block (time-domain items: block 0 yields its outputs from 0), up to I8_WPB
// blocks per workgroup (fewer workgroups to launch); the waves share nothing and never wait for each
// other.  A wave's LDS region holds the block's companded samples as two digit planes of plane_len bytes (byte i + N - 1 of a plane is
// digit p of s~[i], zero outside [0, nvalid)), so every A fragment is one aligned 16-byte read,
// and behind them, for a window longer than I8_REG_WIN samples, the window that the planes are
// built from.  The taps' B fragments stream from L2 in chunks of I8_KC k-steps, the next
// chunk in flight while the current one runs.
constexpr int I8_KC = 4;
constexpr int I8_REG_WIN = 1024;  // longest window held in registers (a multiple of 128)
constexpr int I8_WPB = 1;  // most waves (blocks) per workgroup (2 measured no faster)

// LDS order point between the lanes of one wave (the LDS unit runs a wave's instructions in
// order; the fence keeps the compiler from moving LDS accesses across it)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// SS, SK: the samples' / the taps' companding range exceeds 127 (two digit planes); TM: output
// tiles per pass over the taps (more tiles reuse each fragment load, fewer keep fewer accumulators
// and do no work for a block that has fewer tiles)
template <bool SS, bool SK, bool MANY, int TM>
__global__ void __launch_bounds__(64 * I8_WPB, (SS || SK || TM > 1) ? 2 : 7) k_i8(RunArgs a0, const i8x16* __restrict__ frag, int ksteps,
                                                       int plane_len, int region) {
    extern __shared__ __attribute__((aligned(16))) char lds_all[];
    const int lane = threadIdx.x & 63;
    // the wave's block index is uniform: its lookups (the signal's arguments) are scalar loads
    const int wv = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    int64_t blk = (int64_t)blockIdx.x * (blockDim.x >> 6) + wv;
    if (blk >= a0.nitems) return;
    const RunArgs& a = item_args<MANY>(a0, blk);
    char* lds_i8 = lds_all + (size_t)wv * region;
    const Item it = make_item(a, blk, false);
    const int off = a.N - 1;
    const KState ksv = *a0.ks;  // one taps' state for every signal of the launch
    // A window of at most I8_REG_WIN samples stays in registers (one load step) and its digits go
    // straight to the planes; a longer one passes through LDS behind the planes, shifted by
    // (N - 1) mod 4 samples so that the four samples of one plane word are one aligned 16-byte
    // read.
    const bool inreg = a.W_block <= I8_REG_WIN;
    float* win = reinterpret_cast<float*>(lds_i8 + (SS ? 2 : 1) * plane_len) + (off & 3);
    int* p0 = reinterpret_cast<int*>(lds_i8);
    int* p1 = reinterpret_cast<int*>(lds_i8 + plane_len);
    if (inreg) {  // zero planes: the digits of the window overwrite their part
        for (int w = lane; w < plane_len / 16; w += 64) {
            reinterpret_cast<int4*>(p0)[w] = make_int4(0, 0, 0, 0);
            if (SS) reinterpret_cast<int4*>(p1)[w] = make_int4(0, 0, 0, 0);
        }
    }
    // window with its statistics; start is even and s_in 8-byte aligned (float2 loads).  The
    // maximum is taken in FP32 (exact), and x * 0 accumulated in z stays zero while every
    // sample is finite; a lane that meets a non-finite sample takes its partials again with the
    // exact per-sample rule (non-finite samples count as zero and set the flag).
    // samples per load step: 128 CH = I8_REG_WIN (twice as many measured slower on long blocks)
    constexpr int CR = I8_REG_WIN / 128;
    constexpr int CH = CR;
    float2 f[CH];  // the last load step's samples: the whole window when inreg
    BlockStats st;
    {
        float m = 0.0f;
        double q = 0.0;
        int nf = 0;
        gcfloat* p = (gcfloat*)(a.s + it.start);
        for (int base = 0; base < a.W_block; base += 128 * CH) {
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int i = base + 2 * lane + 128 * c;
                f[c] = make_float2(0.0f, 0.0f);
                if (base + 128 * c < it.nwin) {  // uniform: the chunk holds samples
                    if (i + 1 < it.nwin) {
                        const f32x2 v = *(gcf32x2*)(p + i);
                        f[c] = make_float2(v.x, v.y);
                    } else if (i < it.nwin) {
                        f[c].x = p[i];
                    }
                }
            }
            float z = 0.0f;
            float mc = 0.0f;
            double qc = 0.0;
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int i = base + 2 * lane + 128 * c;
                if (base + 128 * c < a.W_block && i < a.W_block) {
                    const float x0 = f[c].x, x1 = f[c].y;
                    mc = fmaxf(mc, fmaxf(fabsf(x0), fabsf(x1)));
                    z = fmaf(x0, 0.0f, z);
                    z = fmaf(x1, 0.0f, z);
                    qc = fma((double)x0, (double)x0, qc);
                    qc = fma((double)x1, (double)x1, qc);
                    if (!inreg) *reinterpret_cast<float2*>(win + i) = f[c];
                }
            }
            if (z != 0.0f) {  // a non-finite sample in this lane's part
                mc = 0.0f;
                qc = 0.0;
#pragma unroll
                for (int c = 0; c < CH; ++c) {
                    const int i = base + 2 * lane + 128 * c;
                    if (i < a.W_block) {
                        const float x0 = f[c].x, x1 = f[c].y;
                        if (!isfinite(x0) || !isfinite(x1)) nf = 1;
                        const float y0 = isfinite(x0) ? x0 : 0.0f, y1 = isfinite(x1) ? x1 : 0.0f;
                        mc = fmaxf(mc, fmaxf(fabsf(y0), fabsf(y1)));
                        qc = fma((double)y0, (double)y0, qc);
                        qc = fma((double)y1, (double)y1, qc);
                    }
                }
            }
            m = fmaxf(m, mc);
            q += qc;
        }
        st.smax = (double)wave_max_dpp(m);
        st.sumsq = wave_sum_dpp(q);
        st.nonfinite = __ballot(nf) != 0;
    }
    const Choice c = choose(a, st, ksv);
    gfloat* const outp = (gfloat*)a.out;
    gdouble* const fldp = (gdouble*)a.fields;
    const int64_t ob = it.o0 - it.j_lo;  // r_out index of local output m: ob + m
    write_info(a, it, c, st, true, lane == 0);
    if ((c.flags & APX_FLAG_NONFINITE) || (c.flags & APX_FLAG_ZERO)) {
        const float v = (c.flags & APX_FLAG_NONFINITE) ? NAN : 0.0f;
        for (int j = it.j_lo + lane; j < it.j_hi; j += 64) {
            a.out[it.o0 + (j - it.j_lo)] = v;
            if (a.fields) a.fields[it.o0 + (j - it.j_lo)] = 0.0;
        }
        return;
    }
    // Blocks walk the k-steps from different starting chunks (the integer sums do not depend on
    // the order), so the waves of the GPU do not all read the same fragment rows at once.  The
    // fragments load during the companding, not beside the window: registers held through the
    // window's phase would cost a wave per SIMD.
    const int kpad = (ksteps + I8_KC - 1) / I8_KC * I8_KC;
    const int nchunk = kpad / I8_KC;
    const int c_first = (int)(blk % nchunk);
    i8x16 bc[I8_KC][SK ? 2 : 1], bn[I8_KC][SK ? 2 : 1];
#pragma unroll
    for (int kk = 0; kk < I8_KC; ++kk) {
        bc[kk][0] = frag[(c_first * I8_KC + kk) * 64 + lane];
        if constexpr (SK) bc[kk][SK ? 1 : 0] = frag[(kpad + c_first * I8_KC + kk) * 64 + lane];
    }
    // companded samples (eq. 2, as sq_at), as digit planes: byte j of a plane is a digit of
    // s~[j - (N - 1)], zero wherever that sample is outside [0, nvalid) (samples past nwin
    // were loaded as zeros, nvalid = nwin on this core)
    const bool split_s = SS;
    if (inreg) {
#pragma unroll
        for (int c2 = 0; c2 < CR; ++c2) {
            const int i = 2 * lane + 128 * c2;
            if (128 * c2 < a.W_block && i < a.W_block) {
                int lo0, hi0, lo1, hi1;
                i8_digits((int)rint(c.cs * (double)f[c2].x), split_s, lo0, hi0);
                i8_digits((int)rint(c.cs * (double)f[c2].y), split_s, lo1, hi1);
                *reinterpret_cast<unsigned short*>(lds_i8 + off + i) = (unsigned short)((lo0 & 255) | ((lo1 & 255) << 8));
                if (split_s)
                    *reinterpret_cast<unsigned short*>(lds_i8 + plane_len + off + i) =
                        (unsigned short)((hi0 & 255) | ((hi1 & 255) << 8));
            }
        }
    } else {
        // word w4 holds samples i0 .. i0 + 3, i0 = 4 w4 - (N - 1): inside the window one
        // 16-byte read, outside it zero digits, across an edge sample by sample
        for (int w4 = lane; w4 < plane_len / 4; w4 += 64) {
            const int i0 = 4 * w4 - off;
            float x[4] = {0.0f, 0.0f, 0.0f, 0.0f};
            if (i0 >= 0 && i0 + 3 < a.W_block) {
                const float4 x4 = *reinterpret_cast<const float4*>(win + i0);
                x[0] = x4.x;
                x[1] = x4.y;
                x[2] = x4.z;
                x[3] = x4.w;
            } else if (i0 + 3 >= 0 && i0 < a.W_block) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    if (i0 + e >= 0 && i0 + e < a.W_block) x[e] = win[i0 + e];
            }
            int lo4 = 0, hi4 = 0;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int v = (int)rint(c.cs * (double)x[e]);
                int lo, hi;
                i8_digits(v, split_s, lo, hi);
                lo4 |= (lo & 255) << (8 * e);
                hi4 |= (hi & 255) << (8 * e);
            }
            p0[w4] = lo4;
            if (split_s) p1[w4] = hi4;
        }
    }
    wave_lds_sync();
    const int j0 = it.j_lo & ~15;
    const int ntiles = (it.j_hi - j0 + I8_TILE - 1) / I8_TILE;
    const int row = lane & 31, half = lane >> 5;
    const char* a0p = lds_i8 + 32 * row + 16 * half;
    const char* a1p = a0p + plane_len;
    // every pass computes TM tiles over kpad k-steps (the planes and the zero-padded fragment
    // rows cover them); a last pass with fewer tiles repeats the last tile, and outputs past j_hi
    // are not stored.  A pass ends with the next pass's first chunk in bc.
    constexpr int NACC = SS && SK ? 3 : (SS || SK ? 2 : 1);
    // one accumulator set per digit product: a second set for independent MFMA chains measured
    // slower, the registers it takes costing a wave per SIMD
    for (int t0 = 0; t0 < ntiles; t0 += TM) {
        i32x16 acc[NACC][TM];
#pragma unroll
        for (int g = 0; g < NACC; ++g)
#pragma unroll
            for (int u = 0; u < TM; ++u)
#pragma unroll
                for (int r = 0; r < 16; ++r) acc[g][u][r] = 0;
        int tofs[TM];  // tile origin in the planes
#pragma unroll
        for (int u = 0; u < TM; ++u) tofs[u] = j0 + min(t0 + u, ntiles - 1) * I8_TILE;
        for (int ci = 0; ci < nchunk; ++ci) {
            int c = c_first + ci;
            if (c >= nchunk) c -= nchunk;
            const int k0 = c * I8_KC;
            int cn = c + 1;
            if (cn >= nchunk) cn -= nchunk;
            const int kn = cn * I8_KC;
            // the next chunk's fragments, or the next pass's first.  One-tile passes (short blocks,
            // where a block has one chunk and one pass) skip the load that nothing would use; the
            // others load unconditionally, which lets the compiler keep the two register sets
            // without copies (measured 4-7% faster there, and 2% slower for one-tile blocks)
            const bool pre = TM > 1 || ci + 1 < nchunk || t0 + TM < ntiles;
            if (pre) {
#pragma unroll
                for (int kk = 0; kk < I8_KC; ++kk) {
                    bn[kk][0] = frag[(kn + kk) * 64 + lane];
                    if constexpr (SK) bn[kk][SK ? 1 : 0] = frag[(kpad + kn + kk) * 64 + lane];
                }
            }
#pragma unroll
            for (int kk = 0; kk < I8_KC; ++kk) {
#pragma unroll
                for (int u = 0; u < TM; ++u) {
                    const int ofs = tofs[u] + 32 * (k0 + kk);
                    const i8x16 x0 = *reinterpret_cast<const i8x16*>(a0p + ofs);
                    acc[0][u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(x0, bc[kk][0], acc[0][u], 0, 0, 0);
                    if constexpr (SK)
                        acc[1][u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(x0, bc[kk][SK ? 1 : 0], acc[SK ? 1 : 0][u],
                                                                          0, 0, 0);
                    if constexpr (SS) {
                        const i8x16 x1 = *reinterpret_cast<const i8x16*>(a1p + ofs);
                        acc[1][u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(x1, bc[kk][0], acc[NACC > 1 ? 1 : 0][u],
                                                                          0, 0, 0);
                        if constexpr (SK)
                            acc[NACC - 1][u] = __builtin_amdgcn_mfma_i32_32x32x32_i8(x1, bc[kk][SK ? 1 : 0],
                                                                                     acc[NACC - 1][u], 0, 0, 0);
                    }
                }
            }
            if (pre) {
#pragma unroll
                for (int kk = 0; kk < I8_KC; ++kk) {
                    bc[kk][0] = bn[kk][0];
                    if constexpr (SK) bc[kk][SK ? 1 : 0] = bn[kk][SK ? 1 : 0];
                }
            }
        }
        // D[r] of lane l is row 8 (r / 4) + 4 (l / 32) + r % 4, column l % 32
#pragma unroll
        for (int u = 0; u < TM; ++u) {
            if (t0 + u >= ntiles) continue;
            const int m0 = j0 + (t0 + u) * I8_TILE;
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int m = m0 + 32 * (8 * (r >> 2) + 4 * half + (r & 3)) + row;
                if (m >= it.j_lo && m < it.j_hi) {
                    // exact in FP64: every partial sum stays below 2^53 in magnitude
                    double v = (double)acc[0][u][r];
                    if constexpr (NACC > 1) v = fma(128.0, (double)acc[NACC > 1 ? 1 : 0][u][r], v);
                    if constexpr (NACC > 2) v = fma(16384.0, (double)acc[NACC - 1][u][r], v);
                    v += 0.0;  // a zero digit is +0, as the integer it stands for
                    if (fldp) fldp[ob + m] = v;
                    outp[ob + m] = (float)(c.inv * v);  // eq. (16)
                }
            }
        }
    }
}

// Host side of the integer core.  frag: 2 planes of i8_kpad(N) rows of 64 entries of 16 bytes
// (rows from ksteps on are zero).
int i8_ksteps(int N_odd) { return (N_odd + 31 + 31) / 32; }
int i8_kpad(int N_odd) { return (i8_ksteps(N_odd) + I8_KC - 1) / I8_KC * I8_KC; }

// output tiles of the block with the most (block 0 from output 0, later blocks from N + 1)
int i8_tiles(int N_odd, int W) {
    const int nt0 = (W + N_odd - 1 + I8_TILE - 1) / I8_TILE;
    const int j0 = (N_odd + 1) & ~15;
    const int nt1 = (N_odd + 1 + W - j0 + I8_TILE - 1) / I8_TILE;
    return std::max(nt0, nt1);
}

int i8_plane_len(int N_odd, int W) {
    const int nt0 = (W + N_odd - 1 + I8_TILE - 1) / I8_TILE;     // block 0: outputs from 0
    const int j0 = (N_odd + 1) & ~15;                             // later blocks
    const int nt1 = (N_odd + 1 + W - j0 + I8_TILE - 1) / I8_TILE;
    const int need = std::max(nt0 * I8_TILE, j0 + nt1 * I8_TILE) + 32 * i8_kpad(N_odd);
    return (need + 15) & ~15;
}

hipError_t launch_i8_frag(const float* kf, const KState* ks, int mode, int N_odd, int split, void* frag,
                          hipStream_t st) {
    const int n = 2 * i8_kpad(N_odd) * 64;
    hipLaunchKernelGGL(k_i8_frag, dim3((n + NT - 1) / NT), dim3(NT), 0, st, kf, ks, mode, N_odd, i8_kpad(N_odd),
                       split, reinterpret_cast<i8x16*>(frag));
    return hipGetLastError();
}

template <int TM>
static void i8_fns(const void** fs) {
    fs[0] = (const void*)k_i8<false, false, false, TM>;
    fs[1] = (const void*)k_i8<false, true, false, TM>;
    fs[2] = (const void*)k_i8<true, false, false, TM>;
    fs[3] = (const void*)k_i8<true, true, false, TM>;
    fs[4] = (const void*)k_i8<false, false, true, TM>;
    fs[5] = (const void*)k_i8<false, true, true, TM>;
    fs[6] = (const void*)k_i8<true, false, true, TM>;
    fs[7] = (const void*)k_i8<true, true, true, TM>;
}

hipError_t i8_set_lds(int bytes) {
    const void* fs[24];
    i8_fns<1>(fs);
    i8_fns<2>(fs + 8);
    i8_fns<3>(fs + 16);
    for (const void* f : fs) {
        hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// LDS region of one block: the digit planes (two when the samples' range exceeds 127) and, for
// a window longer than I8_REG_WIN, the window.  i8_lds_bytes is the largest (two planes).  A workgroup holds I8_WPB
// regions while that leaves room for two workgroups per CU, else one.
static size_t i8_region(int plane_len, int W_block, int planes = 2) {
    // a longer window passes through LDS (shifted by up to 3 samples)
    const size_t win = W_block <= I8_REG_WIN ? 0 : (size_t)4 * W_block + 16;
    return ((size_t)planes * plane_len + win + 15) & ~(size_t)15;
}
static int i8_wpb(size_t region) { return I8_WPB * region <= 81920 ? I8_WPB : 1; }
size_t i8_lds_bytes(int plane_len, int W_block) {
    const size_t rg = i8_region(plane_len, W_block);
    return (size_t)i8_wpb(rg) * rg;
}

// split_s: the fixed mode's S_q > 127 (every block of the call uses it)
hipError_t launch_i8(const RunArgs& a, const void* frag, int split_s, int split_k, int plane_len, int tm, hipStream_t st) {
    const int rg = (int)i8_region(plane_len, a.W_block, split_s ? 2 : 1);
    const int wpb = i8_wpb((size_t)rg);
    const dim3 g((unsigned)((a.nitems + wpb - 1) / wpb)), b(64 * wpb);
    const size_t lds = (size_t)wpb * rg;
    const i8x16* fr = reinterpret_cast<const i8x16*>(frag);
    const int ks = i8_ksteps(a.N);
#define APX_GOT(SS_, SK_, TM_)                                                                          \
    if (a.many) hipLaunchKernelGGL((k_i8<SS_, SK_, true, TM_>), g, b, lds, st, a, fr, ks, plane_len, rg);  \
    else hipLaunchKernelGGL((k_i8<SS_, SK_, false, TM_>), g, b, lds, st, a, fr, ks, plane_len, rg);
#define APX_GO(SS_, SK_)                  \
    if (tm == 1) {                        \
        APX_GOT(SS_, SK_, 1)              \
    } else if (tm == 2) {                 \
        APX_GOT(SS_, SK_, 2)              \
    } else {                              \
        APX_GOT(SS_, SK_, 3)              \
    }
    if (split_s && split_k) {
        APX_GO(true, true)
    } else if (split_s) {
        APX_GO(true, false)
    } else if (split_k) {
        APX_GO(false, true)
    } else {
        APX_GO(false, false)
    }
#undef APX_GO
#undef APX_GOT
    return hipGetLastError();
}

}  // namespace apx
