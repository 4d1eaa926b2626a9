// FFT convolution core, one wavefront per overlap-save block.
//
// Each 64-lane wave owns one block: it reads the window, takes the block statistics with
// cross-lane reductions, chooses the packing, builds the packed words in registers, runs a
// complex FFT of M = F/2 points (F = real FFT length in words) as three Stockham passes
// (radix E = M/64 in registers, then radix 8, radix 8; the wave's own LDS slice carries the two
// exchanges), applies the kernel spectrum through a precomputed real-split coefficient table,
// runs the inverse the same way and unpacks + dequantizes straight from registers to r_out.
// Workgroups are a single wave, so no barrier ever waits on another wave.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "fft.h"
#include "internal.h"
#include "items.h"

namespace apx {

// exp(-2 pi i m / 32) and exp(-2 pi i m / 24), filled by the host (extended precision).
__constant__ double2 c_w32d[32];
__constant__ double2 c_w24d[24];
__constant__ float2 c_w32f[32];
__constant__ float2 c_w24f[24];

hipError_t upload_dft_constants(const double2* w32, const double2* w24) {
    float2 f32[32], f24[24];
    for (int i = 0; i < 32; ++i) f32[i] = make_float2((float)w32[i].x, (float)w32[i].y);
    for (int i = 0; i < 24; ++i) f24[i] = make_float2((float)w24[i].x, (float)w24[i].y);
    hipError_t e = hipMemcpyToSymbol(HIP_SYMBOL(c_w32d), w32, sizeof(double2) * 32);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_w24d), w24, sizeof(double2) * 24);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_w32f), f32, sizeof(float2) * 32);
    if (e == hipSuccess) e = hipMemcpyToSymbol(HIP_SYMBOL(c_w24f), f24, sizeof(float2) * 24);
    return e;
}

template <typename T>
__device__ __forceinline__ cx<T> cw_table(int R, int m) {
    if constexpr (std::is_same<T, double>::value) {
        double2 w = (32 % R == 0) ? c_w32d[m * (32 / R)] : c_w24d[m * (24 / R)];
        return {w.x, w.y};
    } else {
        float2 w = (32 % R == 0) ? c_w32f[m * (32 / R)] : c_w24f[m * (24 / R)];
        return {w.x, w.y};
    }
}

// a * W_R^m, W_R = exp(-2 pi i / R) (forward) or its conjugate (inverse).  m, R are constants
// after unrolling; the trivial factors cost no multiplication.
template <typename T, bool INV>
__device__ __forceinline__ cx<T> mulw(cx<T> a, int R, int m) {
    m %= R;
    if (m == 0) return a;
    if (2 * m == R) return {-a.x, -a.y};
    if (4 * m == R) return rot<T, INV>(a);
    if (4 * m == 3 * R) return rot<T, !INV>(a);
    const T h = (T)0.70710678118654752440084436210484903928;
    if (8 * m == R) return INV ? cx<T>{(a.x - a.y) * h, (a.x + a.y) * h} : cx<T>{(a.x + a.y) * h, (a.y - a.x) * h};
    if (8 * m == 3 * R)
        return INV ? cx<T>{(-a.x - a.y) * h, (a.x - a.y) * h} : cx<T>{(a.y - a.x) * h, (-a.x - a.y) * h};
    if (8 * m == 5 * R)
        return INV ? cx<T>{(a.y - a.x) * h, (-a.x - a.y) * h} : cx<T>{(-a.x - a.y) * h, (a.x - a.y) * h};
    if (8 * m == 7 * R)
        return INV ? cx<T>{(a.x + a.y) * h, (a.y - a.x) * h} : cx<T>{(a.x - a.y) * h, (a.x + a.y) * h};
    cx<T> w = cw_table<T>(R, m);
    if (INV) w.y = -w.y;
    return cmul(a, w);
}

template <typename T, bool INV>
__device__ __forceinline__ void dft3(cx<T>& a, cx<T>& b, cx<T>& c) {
    const T s3 = (T)0.86602540378443864676372317075293618347;  // sqrt(3)/2
    cx<T> t = b + c, d = b - c;
    cx<T> m = {a.x - (T)0.5 * t.x, a.y - (T)0.5 * t.y};
    cx<T> r = rot<T, INV>(d);
    cx<T> s = {r.x * s3, r.y * s3};
    a = a + t;
    b = m + s;
    c = m - s;
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftn(cx<T>* v);

// Cooley-Tukey R = R1 R2 in registers: inner DFTs of size R1 over stride R2, twiddles W_R^(n2 k1),
// outer DFTs of size R2; output in natural order.
template <typename T, int R1, int R2, bool INV>
__device__ __forceinline__ void dft_ct(cx<T>* v) {
    constexpr int R = R1 * R2;
#pragma unroll
    for (int n2 = 0; n2 < R2; ++n2) {
        cx<T> a[R1];
#pragma unroll
        for (int n1 = 0; n1 < R1; ++n1) a[n1] = v[R2 * n1 + n2];
        dftn<T, R1, INV>(a);
#pragma unroll
        for (int k1 = 0; k1 < R1; ++k1) v[R2 * k1 + n2] = mulw<T, INV>(a[k1], R, n2 * k1);
    }
    cx<T> out[R];
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
        cx<T> b[R2];
#pragma unroll
        for (int n2 = 0; n2 < R2; ++n2) b[n2] = v[R2 * k1 + n2];
        dftn<T, R2, INV>(b);
#pragma unroll
        for (int k2 = 0; k2 < R2; ++k2) out[k1 + R1 * k2] = b[k2];
    }
#pragma unroll
    for (int i = 0; i < R; ++i) v[i] = out[i];
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftn(cx<T>* v) {
    if constexpr (R == 2) dft2<T, INV>(v);
    else if constexpr (R == 3) dft3<T, INV>(v[0], v[1], v[2]);
    else if constexpr (R == 4) dft4<T, INV>(v[0], v[1], v[2], v[3]);
    else if constexpr (R == 8) dft8<T, INV>(v);
    else if constexpr (R == 16) dft_ct<T, 4, 4, INV>(v);
    else if constexpr (R == 24) dft_ct<T, 8, 3, INV>(v);
    else if constexpr (R == 32) dft_ct<T, 8, 4, INV>(v);
    else static_assert(R == 2, "unsupported in-register DFT size");
}

// row[off / sizeof(V)] for a wave-uniform row pointer and a per-lane byte offset below 4 GiB
template <typename V>
__device__ __forceinline__ V ld_row(const V* row, uint32_t off) {
    return *reinterpret_cast<const V*>(reinterpret_cast<const char*>(row) + off);
}

// An opaque copy of a wave-uniform table pointer: loads through it cannot be merged with loads
// through the original, so table entries read in one phase are not kept in registers for a
// later phase that reads them again (the inverse transform reuses the forward one's twiddles).
template <typename V>
__device__ __forceinline__ const V* table_fresh(const V* p) {
    const uint64_t b = (uint64_t)(uintptr_t)p;
    uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b), hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    // device memory: global loads (a generic pointer's flat loads would also count against the
    // LDS wait counter, so every wait for an LDS exchange would wait for table reads too)
    return (const V*)(const __attribute__((address_space(1))) V*)(uintptr_t)(((uint64_t)hi << 32) | lo);
}

// An opaque copy of the lane id (0..63 in every wave of the workgroup): address arithmetic derived from it cannot be shared between
// phases, so nothing computed for one phase stays live (in registers) through the next.
__device__ __forceinline__ int lane_id_fresh() {
    int l = (int)threadIdx.x & 63;
    asm volatile("" : "+v"(l));
    return l;
}

// Complex FFT of M points by one wave: lane l holds v[r] = z[l + 64 r] on entry and
// v[t] = Z[l + 64 t] on exit (one-wave workgroups: its barriers wait on no other wave).  Passes: radix E (= M/64, registers only), radix 8, radix 8.
// The two exchanges use the wave's LDS slice in a padded layout, point i at i + floor(i/E)
// (rows of E points padded by one: the strided writes of the first pass spread over the
// banks); every address below is that mapping in closed form.
// Twiddles: TS > 1 reads W_M^t at tw[t TS] (a sub-transform of a longer table).  TS = 1 reads
// the per-pass copies that follow the M-entry table: W_M^{8 r k} at tw[M + (r-1) E + k] and
// W_M^{r j} at tw[M + 7 E + (r-1) M/8 + j], so that the 64 lanes of one load read adjacent
// entries (a few cache lines) instead of entries r or 8 r apart.
template <typename T, int M, bool INV, int TS = 1>
__device__ __forceinline__ void wave_fft(cx<T>* v, cx<T>* lds, const typename tw_of<T>::type* tw) {
    constexpr int E = M / 64;
    static_assert(E % 8 == 0, "points per lane must be a multiple of 8");
    constexpr int NB = E / 8;  // radix-8 butterflies per lane in passes B and C
    constexpr int S = E + 1;   // padded row
    using TW = typename tw_of<T>::type;
    // per-pass entries: a uniform row base plus the lane's unsigned 32-bit byte offset, so each
    // load is one instruction on a scalar base (no 64-bit address arithmetic per load)
    auto twB = [&](int r, int k) {
        if constexpr (TS == 1) return ld_row(tw + M + (r - 1) * E, (uint32_t)k * (uint32_t)sizeof(TW));
        else return tw[r * k * 8 * TS];
    };
    auto twC = [&](int r, int j) {
        if constexpr (TS == 1) return ld_row(tw + M + 7 * E + (r - 1) * (M / 8), (uint32_t)j * (uint32_t)sizeof(TW));
        else return tw[r * j * TS];
    };
    // pass A: radix E, no twiddles (sub-transform size 1); output i = l E + r
    dftn<T, E, INV>(v);
    {
        cx<T>* p = lds + lane_id_fresh() * S;
#pragma unroll
        for (int r = 0; r < E; ++r) p[r] = v[r];
    }
    __syncthreads();
    // pass B: radix 8 over sub-transforms of size E; input i = j + 8E r, output 8E q + k + E r
    {
        const int l = lane_id_fresh();
        cx<T> u[NB][8];
        int wofs[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = l + 64 * b;
            const int q = j / E;
            const int k = j - q * E;
            const cx<T>* rp = lds + j + q;
#pragma unroll
            for (int r = 0; r < 8; ++r) u[b][r] = rp[8 * r * S];
#pragma unroll
            for (int r = 1; r < 8; ++r) {
                auto w = twB(r, k);  // W_{8E}^{rk} = W_M^{8rk}
                u[b][r] = cmul(u[b][r], cx<T>{w.x, INV ? -w.y : w.y});
            }
            dft8<T, INV>(u[b]);
            wofs[b] = q * 8 * S + k;
        }
        __syncthreads();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            cx<T>* wp = lds + wofs[b];
#pragma unroll
            for (int r = 0; r < 8; ++r) wp[r * S] = u[b][r];
        }
        __syncthreads();
    }
    // pass C: radix 8 over sub-transforms of size M/8; results stay in registers
    {
        const int l = lane_id_fresh();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = l + 64 * b;
            const cx<T>* rp = lds + j + j / E;
            cx<T> x[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) x[r] = rp[8 * r * S];
#pragma unroll
            for (int r = 1; r < 8; ++r) {
                auto w = twC(r, j);
                x[r] = cmul(x[r], cx<T>{w.x, INV ? -w.y : w.y});
            }
            dft8<T, INV>(x);
#pragma unroll
            for (int r = 0; r < 8; ++r) v[b + NB * r] = x[r];
        }
    }
    __syncthreads();
}

// Real-signal spectral step: V[k] = alpha_k Z[k] + beta_k conj(Z[M-k]) with alpha, beta built
// from the kernel spectrum (see k_coef); the unnormalized inverse of V is the cyclic convolution
// (even words + i odd words).  Plain layout here: point i at i, plus Z[M] := Z[0].
template <typename T, int M>
__device__ __forceinline__ void wave_spectral(cx<T>* v, cx<T>* lds, const typename tw_of<T>::type* coef) {
    constexpr int E = M / 64;
    {
        const int l = lane_id_fresh();
        cx<T>* p = lds + l;
#pragma unroll
        for (int t = 0; t < E; ++t) p[64 * t] = v[t];
        if (l == 0) lds[M] = v[0];
    }
    __syncthreads();
    {
        const int l = lane_id_fresh();
        const cx<T>* rb = lds + (M - l) - 64 * (E - 1);  // rb[64 (E-1-t)] = Z[M - l - 64 t]
        const uint32_t co = (uint32_t)l * (uint32_t)(2 * sizeof(*coef));  // lane's (alpha, beta) pair
#pragma unroll
        for (int t = 0; t < E; ++t) {
            const cx<T> zb = rb[64 * (E - 1 - t)];
            const auto al = ld_row(coef + 128 * t, co);
            const auto be = ld_row(coef + 128 * t + 1, co);
            const cx<T> z = v[t];
            v[t] = cmul(z, cx<T>{al.x, al.y}) + cmul(conj(zb), cx<T>{be.x, be.y});
            if ((t & 3) == 3) __builtin_amdgcn_sched_barrier(0);  // bound the loads in flight
        }
    }
    __syncthreads();
}

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}
__device__ __forceinline__ double wmax(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    return v;
}
__device__ __forceinline__ int wor(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v |= __shfl_xor(v, o);
    return v;
}

struct WStats {
    double smax, sumsq;
    int nonfinite;
};

// Items, choice, placement and digit splitting are shared with the block kernels.
struct WItem {
    int64_t start;
    int nwin, nvalid, j_lo, j_hi;
    int64_t o0, w;
};

__device__ __forceinline__ WItem wave_make_item(const RunArgs& a, int64_t item) {
    WItem it;
    const int N = a.N;
    const bool prefix = item >= a.P;
    it.w = prefix ? 0 : item;
    it.start = it.w == 0 ? 0 : (int64_t)a.W * it.w - 2;
    const int64_t rem = a.L - it.start;
    it.nwin = (int)(rem < a.W_block ? rem : a.W_block);
    it.nvalid = it.nwin;
    if (prefix) {
        it.j_lo = 0;
        it.j_hi = N + 1;
        it.o0 = 0;
        if (it.nvalid > N + 1) it.nvalid = N + 1;
    } else if (it.w == 0) {
        it.j_lo = N + 1;
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

struct WChoice {
    int mode, S, K, flags;
    int64_t R;
    double cs, inv, snr_db;  // inv = (c_s c_k)^-1 of eq. (16)
};

__device__ __forceinline__ double wsnr_ratio(double rms, double smax, double krms, double kmax, int S, int K) {
    const double r12 = 3.4641016151377545870548926830117447;
    double svs = smax / ((double)S * r12);
    double svk = kmax / ((double)K * r12);
    double a = rms * svk, b = krms * svs, c = svk * svs;
    double D = a * a + b * b + c * c;
    double p = rms * krms;
    return (p * p) / D;
}

// Inputs of the choice that live in device memory (the taps' statistics, this call's
// calibration), requested at the start of a block so that their latency overlaps the window load.
struct WChoiceIn {
    KState ks;
    double calib, thr;
};
__device__ __forceinline__ WChoiceIn wave_choice_inputs(const RunArgs& a) {
    WChoiceIn in;
    in.ks = *a.ks;
    in.calib = a.calib_db;
    in.thr = a.thr_lin;
    if (a.mode == MD_AUTO && a.calib_dev) {  // this call's calibration: offset and threshold ratio
        in.calib = a.calib_dev[0];
        in.thr = a.calib_dev[1];
    }
    return in;
}

__device__ __forceinline__ WChoice wave_choose(const RunArgs& a, const WStats& st, const WChoiceIn& in) {
    WChoice c;
    KState ks = in.ks;
    // eq. (18)'s sigmas: the block's and the taps' root second moments, or source-level values
    const double rms = a.sigma_s > 0.0 ? a.sigma_s : sqrt(st.sumsq / (double)a.W_block);
    // the block's mean square (rms^2) for the division-free comparison below
    const double ms = a.sigma_s > 0.0 ? a.sigma_s * a.sigma_s : st.sumsq * a.inv_wb;
    const bool kzero = ks.krms == 0.0;
    if (a.sigma_k > 0.0) ks.krms = a.sigma_k;
    c.flags = 0;
    c.snr_db = INFINITY;
    c.mode = a.mode;
    if (a.mode == MD_AUTO) {
        const double thr = in.thr, calib = in.calib;
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
        const bool s1 = c.mode == MD_SYM, s2 = c.mode == MD_ASYM2;
        c.S = s1 ? a.S[1] : (s2 ? a.S[2] : a.S[3]);
        c.K = s1 ? a.K[1] : (s2 ? a.K[2] : a.K[3]);
        c.R = s1 ? a.R[1] : (s2 ? a.R[2] : a.R[3]);
        const double ck = s1 ? ks.ck[1] : (s2 ? ks.ck[2] : ks.ck[3]);
        c.cs = st.smax == 0.0 ? 0.0 : (double)c.S / st.smax;
        c.inv = 1.0 / (c.cs * ck);
        if (a.info && a.mode != MD_AUTO && st.smax != 0.0 && !kzero)
            c.snr_db = 10.0 * log10(wsnr_ratio(rms, st.smax, ks.krms, ks.kmax, c.S, c.K));
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



// digits of a symmetric-packed word: rb = 2R Dm + B + eps De, |B| <= R.  The quotient estimate
// uses the rounded reciprocal of 2R; it can be off by one only, which the range corrections
// below undo.  A base digit at |B| = R is ambiguous ((Dm, R) and (Dm + 1, -R) make the same
// word) and is split toward the smaller |Dm|, as in the block kernels.
__device__ __forceinline__ void wsym_split(double rb, double two_r, double inv_two_r, double R, double& Dm, double& B,
                                           double& De) {
    const double I = rint(rb);
    De = rint((rb - I) * two_r);
    double q = rint(I * inv_two_r);
    double b = I - q * two_r;
    if (b > R) {
        q += 1.0;
        b -= two_r;
    }
    if (b < -R) {
        q -= 1.0;
        b += two_r;
    }
    if (b == R && q < 0.0) {
        q += 1.0;
        b -= two_r;
    }
    if (b == -R && q > 0.0) {
        q -= 1.0;
        b += two_r;
    }
    Dm = q;
    B = b;
}

// Window of the item in the wave's LDS slice as FP32 (zero past nvalid), with its statistics
// taken from the same loads: every input sample is read from memory once.
__device__ __forceinline__ WStats wave_load_window(const RunArgs& a, const WItem& it, float* win) {
    double m = 0.0, q = 0.0;
    int nf = 0;
    const float* p = a.s + it.start;  // start is even and s_in 8-byte aligned (checked on the host)
    constexpr int CH = 16;             // float2 loads in flight per lane
    // statistics of one sample pair (non-finite samples count as zero and flag the block)
    auto take = [&](float x0, float x1) {
        const bool f0 = isfinite(x0), f1 = isfinite(x1);
        if (!(f0 && f1)) nf = 1;
        const double d0 = (double)(f0 ? x0 : 0.0f), d1 = (double)(f1 ? x1 : 0.0f);
        m = fmax(m, fmax(fabs(d0), fabs(d1)));
        q += d0 * d0 + d1 * d1;
    };
    for (int base = 0; base < a.W_block; base += 128 * CH) {
        float2 f[CH];
        // wave-uniform: the whole chunk lies inside the signal, the valid part and the window, so
        // it needs no per-sample bounds (every block but the last)
        const int end = base + 128 * CH;
        if (end <= it.nwin && end <= it.nvalid && end <= a.W_block) {
#pragma unroll
            for (int c = 0; c < CH; ++c) f[c] = *reinterpret_cast<const float2*>(p + base + 2 * threadIdx.x + 128 * c);
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int i = base + 2 * threadIdx.x + 128 * c;
                take(f[c].x, f[c].y);
                win[i] = f[c].x;
                win[i + 1] = f[c].y;
            }
            continue;
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int i = base + 2 * threadIdx.x + 128 * c;
            f[c] = make_float2(0.0f, 0.0f);
            if (i + 1 < it.nwin) f[c] = *reinterpret_cast<const float2*>(p + i);
            else if (i < it.nwin) f[c].x = p[i];
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int i = base + 2 * threadIdx.x + 128 * c;
            if (i < a.W_block) {
                take(f[c].x, f[c].y);
                win[i] = (i < it.nvalid) ? f[c].x : 0.0f;
                win[i + 1] = (i + 1 < it.nvalid) ? f[c].y : 0.0f;
            }
        }
    }
    if (threadIdx.x == 0) {
        win[-1] = 0.0f;
        win[a.W_block] = 0.0f;
    }
    WStats r;
    r.smax = wmax(m);
    r.sumsq = wsum(q);
    r.nonfinite = wor(nf);
    __syncthreads();
    return r;
}

// Exact digits of a symmetric-packed word are split by wsym_split; asymmetric words are
// balanced base-2R digits taken one after the other (see the block kernels).
template <int MODE, int M, bool FIELDS>
__device__ __forceinline__ void wave_item(const RunArgs& a, const WItem& it, const WChoice& c, char* lds_raw) {
    using T = typename std::conditional<MODE == MD_FULL32, float, double>::type;
    constexpr int E = M / 64;
    const int N = a.N;
    cx<T>* lds = reinterpret_cast<cx<T>*>(lds_raw);
    const float* win = reinterpret_cast<const float*>(lds_raw) + 1;  // win[-1], win[W_block] are zero
    const typename tw_of<T>::type* tw;
    const typename tw_of<T>::type* coef;
    if constexpr (MODE == MD_FULL32) {
        tw = a.wtwf;
        coef = a.coef32;
    } else {
        tw = (MODE == MD_SYM) ? a.wtw[1] : (MODE == MD_ASYM2 ? a.wtw[2] : a.wtw[3]);
        coef = (MODE == MD_SYM) ? a.coef[1] : (MODE == MD_ASYM2 ? a.coef[2] : a.coef[3]);
    }
    constexpr int MM = (MODE == MD_ASYM3) ? 3 : 2;
    const bool prefix = it.j_lo == 0;
    int Tit = 0, base_off = 0, lw = 0;
    if constexpr (MODE == MD_ASYM2 || MODE == MD_ASYM3) {
        Tit = prefix ? (N + 1 + MM - 1) / MM : a.T[MODE];
        base_off = it.j_lo - (N - 1);
        lw = Tit + N - 1;
    }
    const int wb = a.W_block;
    // window sample, clamped onto the zero sentinels outside [0, W_block)
    auto rd = [&](int i) -> float { return win[min(max(i, -1), wb)]; };
    // companded sample s~[i] (eq. 2)
    auto sqd = [&](int i) -> double { return rint(c.cs * (double)rd(i)); };
    // ---- pack: v[r] = x[2n] + i x[2n+1], n = l + 64 r (eq. 4 / eq. 7)
    cx<T> v[E];
    {
        const int l = lane_id_fresh();
        const double eps = (MODE == MD_FULL32) ? 0.0 : a.eps[MODE];  // eq. (6), formed on the host
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int n = l + 64 * r;
            if constexpr (MODE == MD_FULL32) {
                v[r].x = rd(2 * n);
                v[r].y = rd(2 * n + 1);
            } else if constexpr (MODE == MD_SYM) {
                v[r].x = sqd(4 * n) + eps * sqd(4 * n + 1);
                v[r].y = sqd(4 * n + 2) + eps * sqd(4 * n + 3);
            } else {
                double w2[2] = {0.0, 0.0};
                // words 128 r .. 128 r + 127 of this step: none is packed past lw (wave-uniform)
                if (128 * r < lw) {
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int m = 2 * n + h;
                        double acc = 0.0, e = 1.0;
#pragma unroll
                        for (int q = 0; q < MM; ++q) {
                            acc += e * sqd(base_off + q * Tit + m);
                            e *= eps;
                        }
                        w2[h] = (m < lw) ? acc : 0.0;
                    }
                }
                v[r].x = w2[0];
                v[r].y = w2[1];
            }
            if (r & 1) __builtin_amdgcn_sched_barrier(0);  // bound the window reads in flight
        }
    }
    __syncthreads();  // the window is dead from here on: the FFT reuses the slice
    wave_fft<T, M, false>(v, lds, tw);
    wave_spectral<T, M>(v, lds, coef);
    wave_fft<T, M, true>(v, lds, tw);
    // ---- unpack + dequantize (eq. 16) into a staging row in LDS, then a contiguous copy-out
    float* st = reinterpret_cast<float*>(lds_raw);
    const int l = lane_id_fresh();
    int sbase;  // staging index of the first kept output
    if constexpr (MODE == MD_FULL32) {
#pragma unroll
        for (int t = 0; t < E; ++t) {
            const int n = l + 64 * t;
            if (FIELDS) {
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int j = 2 * n + h;
                    if (j >= it.j_lo && j < it.j_hi) a.fields[it.o0 + (j - it.j_lo)] = 0.0;
                }
            }
            *reinterpret_cast<float2*>(st + 2 * n) = make_float2(v[t].x, v[t].y);
        }
        sbase = it.j_lo;
    } else if constexpr (MODE == MD_SYM) {
        const double two_r = (double)(2 * c.R), R = (double)c.R, inv_two_r = 1.0 / two_r;
        double de_last = 0.0;  // side digit of word 2n - 1 for lane 0: lane 63's odd word at t - 1
#pragma unroll
        for (int t = 0; t < E; ++t) {
            const int n = l + 64 * t;
            double Dm0, B0, De0, Dm1, B1, De1;
            wsym_split(v[t].x, two_r, inv_two_r, R, Dm0, B0, De0);  // word 2n
            wsym_split(v[t].y, two_r, inv_two_r, R, Dm1, B1, De1);  // word 2n+1
            // side digit of word 2n-1 (the odd word of point n-1): neighbour lane, or the wrap
            const double up = __shfl_up(De1, 1);
            const double Dep = (n == 0) ? 0.0 : ((l == 0) ? de_last : up);
            de_last = __shfl(De1, 63);
            // r~[4n .. 4n+3]; a zero digit is +0, as the integer it stands for
            const double f0 = Dm0 + Dep + 0.0, f1 = B0 + 0.0, f2 = Dm1 + De0 + 0.0, f3 = B1 + 0.0;
            if (FIELDS) {
                const double fv[4] = {f0, f1, f2, f3};
#pragma unroll
                for (int h = 0; h < 4; ++h) {
                    const int j = 4 * n + h;
                    if (j >= it.j_lo && j < it.j_hi) a.fields[it.o0 + (j - it.j_lo)] = fv[h];
                }
            }
            *reinterpret_cast<float4*>(st + 4 * n) =
                make_float4((float)(c.inv * f0), (float)(c.inv * f1), (float)(c.inv * f2), (float)(c.inv * f3));
            if (t & 1) __builtin_amdgcn_sched_barrier(0);
        }
        sbase = it.j_lo;
    } else {
        const double two_r = (double)(2 * c.R);
        // word m, digit q -> staging index q Tit + m (= local output - j_lo + N - 1)
#pragma unroll
        for (int t = 0; t < E; ++t) {
            // words 128 t .. 128 t + 127 of this step: none is kept before N - 1 or from lw on
            if (128 * t + 127 < N - 1 || 128 * t >= lw) continue;
            const int n = l + 64 * t;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int m = 2 * n + h;
                double x = h ? (double)v[t].y : (double)v[t].x;
                const bool ok = (m >= N - 1) && (m < lw);
#pragma unroll
                for (int q = 0; q < MM; ++q) {
                    const double d = rint(x) + 0.0;  // a zero digit is +0
                    x = (x - d) * two_r;
                    if (ok) {
                        st[q * Tit + m] = (float)(c.inv * d);
                        if (FIELDS) {
                            const int j = base_off + q * Tit + m;
                            if (j >= it.j_lo && j < it.j_hi) a.fields[it.o0 + (j - it.j_lo)] = d;
                        }
                    }
                }
            }
            if (t & 1) __builtin_amdgcn_sched_barrier(0);
        }
        sbase = N - 1;
    }
    __syncthreads();
    const int nout = it.j_hi - it.j_lo;
    const float* src = st + sbase;
    float* dst = a.out + it.o0;
#pragma unroll 4
    for (int s = l; s < nout; s += 64) out_store(&dst[s], src[s]);
}

// LDS slice of one wave: the padded FFT layout (M + M/E points) and Z[M] of the spectral step.
// The same bytes hold the window (W_block + 2 floats) before and the output staging row after.
template <int M>
constexpr size_t wave_lds_bytes(size_t esz) {
    return (size_t)(M + M / (M / 64) + 1) * 2 * esz;
}

// MASK: bit m set = the packing mode m (MD_*) is compiled in; a block whose chosen mode is not
// compiled in cannot occur (the host launches the instance that holds every mode it can choose).
template <int MS, int MA2, int MA3, int MF, int MASK, bool FIELDS, bool MANY>
__global__ void __launch_bounds__(64) k_fftw(RunArgs a0) {
    constexpr size_t B1 = ((MASK >> MD_SYM) & 1) ? wave_lds_bytes<MS>(8) : 0;
    constexpr size_t B2 = ((MASK >> MD_ASYM2) & 1) ? wave_lds_bytes<MA2>(8) : 0;
    constexpr size_t B3 = ((MASK >> MD_ASYM3) & 1) ? wave_lds_bytes<MA3>(8) : 0;
    constexpr size_t B4 = ((MASK >> MD_FULL32) & 1) ? wave_lds_bytes<MF>(4) : 0;
    constexpr size_t BW = 4 * (2 * (size_t)MF + 2);  // window with sentinels (W_block <= 2 MF)
    constexpr size_t B12 = B1 > B2 ? B1 : B2, B34 = B3 > B4 ? B3 : B4;
    constexpr size_t BF = B12 > B34 ? B12 : B34;
    constexpr size_t BYTES = BF > BW ? BF : BW;
    __shared__ __attribute__((aligned(16))) char lds[BYTES];
    // one item per workgroup (a loop here makes the compiler keep every per-lane address of the
    // body live across iterations, which spills)
    // consecutive blocks share N + 1 samples: give consecutive blocks to workgroups of one XCD
    // (workgroups go to the 8 XCDs in turn), so that the shared samples meet in one L2
    const int64_t nblk = a0.nitems, q8 = nblk / 8, r8 = nblk % 8, x8 = blockIdx.x % 8;
    int64_t item = x8 * q8 + (x8 < r8 ? x8 : r8) + blockIdx.x / 8;
    if (blockIdx.x >= nblk) return;
    const RunArgs& a = item_args<MANY>(a0, item);
    {
        const WChoiceIn cin = wave_choice_inputs(a);
        const WItem it = wave_make_item(a, item);
        const WStats st = wave_load_window(a, it, reinterpret_cast<float*>(lds) + 1);
        const WChoice c = wave_choose(a, st, cin);
        if (a.info && item < a.P && threadIdx.x == 0) {
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
        const bool zero = (c.flags & APX_FLAG_ZERO) && c.mode != MD_FULL32;
        if ((c.flags & APX_FLAG_NONFINITE) || zero || it.j_hi <= it.j_lo) {
            const float v = (c.flags & APX_FLAG_NONFINITE) ? NAN : 0.0f;
            for (int j = it.j_lo + threadIdx.x; j < it.j_hi; j += 64) {
                a.out[it.o0 + (j - it.j_lo)] = v;
                if (FIELDS) a.fields[it.o0 + (j - it.j_lo)] = 0.0;
            }
            return;
        }
        if constexpr ((MASK >> MD_SYM) & 1)
            if (c.mode == MD_SYM) wave_item<MD_SYM, MS, FIELDS>(a, it, c, lds);
        if constexpr ((MASK >> MD_ASYM2) & 1)
            if (c.mode == MD_ASYM2) wave_item<MD_ASYM2, MA2, FIELDS>(a, it, c, lds);
        if constexpr ((MASK >> MD_ASYM3) & 1)
            if (c.mode == MD_ASYM3) wave_item<MD_ASYM3, MA3, FIELDS>(a, it, c, lds);
        if constexpr ((MASK >> MD_FULL32) & 1)
            if (c.mode == MD_FULL32) wave_item<MD_FULL32, MF, FIELDS>(a, it, c, lds);
    }
}

// The wave-FFT size sets that are compiled (complex points per mode: sym, asym2, asym3, fp32).
#define APX_WAVE_SETS(X)          \
    X(1024, 1536, 1024, 2048)     \
    X(1024, 1536, 1536, 2048)     \
    X(512, 1024, 512, 1024)       \
    X(512, 1024, 1024, 1024)      \
    X(512, 512, 512, 1024)        \
    X(512, 512, 512, 512)

bool wave_supported(int ms, int ma2, int ma3, int mf) {
#define APX_CHECK(a_, b_, c_, d_) \
    if (ms == a_ && ma2 == b_ && ma3 == c_ && mf == d_) return true;
    APX_WAVE_SETS(APX_CHECK)
#undef APX_CHECK
    return false;
}

// One instance per size set and mode set: the four fixed modes alone, the per-block choice
// (symmetric, asymmetric M=2, FP32), and every mode with the integer-field output.
template <int A, int B, int C, int D>
static hipError_t launch_set(const RunArgs& a, unsigned grid, hipStream_t st) {
    constexpr int ALL = (1 << MD_SYM) | (1 << MD_ASYM2) | (1 << MD_ASYM3) | (1 << MD_FULL32);
    constexpr int AUTO = (1 << MD_SYM) | (1 << MD_ASYM2) | (1 << MD_FULL32);
#define APX_W(MASK_)                                                                                           \
    if (a.many) hipLaunchKernelGGL((k_fftw<A, B, C, D, MASK_, false, true>), dim3(grid), dim3(64), 0, st, a);  \
    else hipLaunchKernelGGL((k_fftw<A, B, C, D, MASK_, false, false>), dim3(grid), dim3(64), 0, st, a);
    if (a.fields) {
        hipLaunchKernelGGL((k_fftw<A, B, C, D, ALL, true, false>), dim3(grid), dim3(64), 0, st, a);
    } else {
        switch (a.mode) {
            case MD_SYM: APX_W(1 << MD_SYM) break;
            case MD_ASYM2: APX_W(1 << MD_ASYM2) break;
            case MD_ASYM3: APX_W(1 << MD_ASYM3) break;
            case MD_FULL32: APX_W(1 << MD_FULL32) break;
            default: APX_W(AUTO) break;
        }
    }
#undef APX_W
    return hipGetLastError();
}

hipError_t launch_fftw(const RunArgs& a, int ms, int ma2, int ma3, int mf, hipStream_t st) {
    const unsigned grid = (unsigned)a.nitems;
#define APX_LAUNCH(a_, b_, c_, d_) \
    if (ms == a_ && ma2 == b_ && ma3 == c_ && mf == d_) return launch_set<a_, b_, c_, d_>(a, grid, st);
    APX_WAVE_SETS(APX_LAUNCH)
#undef APX_LAUNCH
    return hipErrorInvalidValue;
}


// ------------------------------------------------------------------------------------------
// Multi-wave FFT core: one workgroup of NW waves per block.  A mode's transform of M points is
// split by decimation in time into R transforms of MS = M / R points, one per wave, each run in
// the wave's own LDS region with exchanges ordered inside the wave only (no workgroup barrier),
// and the R results are joined by a radix-R step:
//   Z[k + MS j] = sum_w W_R^(w j) W_M^(w k) Z_w[k],   Z_w = DFT_MS(z[R n + w]).
// The spectral step pairs Z[k'] with Z[M - k'].  Both lie in the columns k and MS - k of the
// join, so the join, the spectral step and the split of the inverse (decimation in frequency)
//   y_w[k] = W_M^(-w k) sum_j W_R^(-w j) V[k + MS j],   x[R n + w] = IDFT_MS(y_w)[n]
// run as one pass over column pairs.  The window goes to LDS with its statistics, every wave
// packs its own decimated points, and the words of the inverse go to LDS, from which
// consecutive threads unpack consecutive outputs.  Blocks are spread over more waves than one
// wave per block gives, which hides memory and LDS latency behind other waves' arithmetic; the
// first wave makes the block's mode choice and hands it to the others through LDS.
// ------------------------------------------------------------------------------------------

// A value every lane of the wave holds equally, moved to scalar registers (frees vector registers
// for the transforms).
__device__ __forceinline__ double uni_d(double v) {
    const uint64_t b = (uint64_t)__double_as_longlong(v);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)b);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(b >> 32));
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}
__device__ __forceinline__ int uni_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ int64_t uni_l(int64_t v) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Ordering point for an LDS exchange among the lanes of one wave: the wave's own LDS
// operations have completed, and the fences keep the compiler from moving LDS accesses across
// it.  No s_barrier: the other waves of the workgroup are not waited for.
__device__ __forceinline__ void region_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Position of point i in a wave region of rows of E points.  E a power of two: the column is
// XORed with the row (mod E), so the row writes of the first pass and the strided reads of the
// next ones spread over the banks with no padding; otherwise each row is padded by one point.
template <int E>
__device__ __forceinline__ int gpos(int i) {
    if constexpr ((E & (E - 1)) == 0) return i ^ ((i / E) & (E - 1));
    else return i + i / E;
}
template <int MS>
constexpr int greg_points() {
    constexpr int E = MS / 64;
    return ((E & (E - 1)) == 0) ? MS : MS + MS / E;
}

// Complex FFT of MS points by one wave in its region `reg`: lane l holds v[r] = z[l + 64 r] on
// entry and v[t] = Z[l + 64 t] on exit.  Passes: radix E = MS/64 in registers, then two radix-8
// passes through the region.  tw: the W_MS^t table followed by its per-pass copies (W^{8 r k} at
// MS + (r-1) E + k, W^{r j} at MS + 7 E + (r-1) MS/8 + j), read at adjacent entries per load.
template <typename T, int MS, bool INV>
__device__ __forceinline__ void gsub_fft(cx<T>* v, cx<T>* reg, const typename tw_of<T>::type* tw) {
    constexpr int E = MS / 64;
    static_assert(E % 8 == 0 && (E & (E - 1)) == 0, "points per lane: a power of two, multiple of 8");
    constexpr int NB = E / 8;
    constexpr int S8 = E / 8;  // distinct row offsets (mod E) among the rows q + 8 r
    using TW = typename tw_of<T>::type;
    auto twB = [&](int r, int k) { return ld_row(tw + MS + (r - 1) * E, (uint32_t)k * (uint32_t)sizeof(TW)); };
    auto twC = [&](int r, int j) {
        return ld_row(tw + MS + 7 * E + (r - 1) * (MS / 8), (uint32_t)j * (uint32_t)sizeof(TW));
    };
    // Positions follow gpos<E>, written out so that each access is a per-lane base plus a
    // constant: point j + 8 E r (row q + 8 r, column k, q = j / E, k = j % E) sits at
    // (q + 8 r) E + (k ^ ((q + 8 r) mod E)), and (q + 8 r) mod E takes E / 8 values as r runs.
    dftn<T, E, INV>(v);  // pass A: output i = l E + r, at l E + (r ^ (l mod E))
    {
        const int l = lane_id_fresh();
        cx<T>* row = reg + l * E;
        const int c = l & (E - 1);
#pragma unroll
        for (int r = 0; r < E; ++r) row[r ^ c] = v[r];
    }
    region_sync();
    // pass B: radix 8 over sub-transforms of size E; input i = j + 8E r, output 8E q + k + E r
    {
        const int l = lane_id_fresh();
        cx<T> u[NB][8];
        int q_[NB], k_[NB];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = l + 64 * b;
            const int q = j / E;
            const int k = j - q * E;
            q_[b] = q;
            k_[b] = k;
            const cx<T>* base[S8];
#pragma unroll
            for (int s = 0; s < S8; ++s) base[s] = reg + q * E + (k ^ ((q + 8 * s) & (E - 1)));
#pragma unroll
            for (int r = 0; r < 8; ++r) u[b][r] = base[r % S8][8 * E * r];
#pragma unroll
            for (int r = 1; r < 8; ++r) {
                const auto w = twB(r, k);  // W_{8E}^{rk} = W_MS^{8rk}
                u[b][r] = cmul(u[b][r], cx<T>{w.x, INV ? -w.y : w.y});
            }
            dft8<T, INV>(u[b]);
        }
        region_sync();
        // point 8 E q + k + E r: row 8 q + r, whose value mod E is 8 (q mod (E / 8)) + r
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            cx<T>* row0 = reg + 8 * E * q_[b];
            const int kx = k_[b] ^ (8 * (q_[b] & (S8 - 1)));
#pragma unroll
            for (int r = 0; r < 8; ++r) row0[E * r + (kx ^ r)] = u[b][r];
        }
    }
    region_sync();
    // pass C: radix 8 over sub-transforms of size MS/8; results stay in registers
    {
        const int l = lane_id_fresh();
#pragma unroll
        for (int b = 0; b < NB; ++b) {
            const int j = l + 64 * b;
            const int q = j / E;
            const int k = j - q * E;
            const cx<T>* base[S8];
#pragma unroll
            for (int s = 0; s < S8; ++s) base[s] = reg + q * E + (k ^ ((q + 8 * s) & (E - 1)));
            cx<T> x[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) x[r] = base[r % S8][8 * E * r];
#pragma unroll
            for (int r = 1; r < 8; ++r) {
                const auto w = twC(r, j);
                x[r] = cmul(x[r], cx<T>{w.x, INV ? -w.y : w.y});
            }
            dft8<T, INV>(x);
#pragma unroll
            for (int r = 0; r < 8; ++r) v[b + NB * r] = x[r];
        }
    }
    region_sync();  // the region is free for the caller
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftr(cx<T>* v) {
    if constexpr (R == 2) dft2<T, INV>(v);
    else if constexpr (R == 3) dft3<T, INV>(v[0], v[1], v[2]);
    else if constexpr (R == 4) dft4<T, INV>(v[0], v[1], v[2], v[3]);
    else static_assert(R == 1, "join radix 1..4");
}

// One pass over column pairs of the R wave regions (plain layout, region w at reg + w RP):
// join (forward radix R), spectral step V[k'] = alpha_k' Z[k'] + beta_k' conj(Z[(M - k') mod M])
// with (alpha, beta) from the kernel's real-split table, split (inverse radix R); in place.
// Thread u takes columns (u, MS - u); thread 0 takes the two self-paired columns 0 and MS / 2.
template <typename T, int M, int R, int RP, int NTH>
__device__ __forceinline__ void gjoin_spectral_split(cx<T>* reg, const typename tw_of<T>::type* twM,
                                                     const typename tw_of<T>::type* coef) {
    constexpr int MS = M / R;
    using TW = typename tw_of<T>::type;
    constexpr uint32_t ES = sizeof(TW);
    for (int u = threadIdx.x; u < MS / 2; u += NTH) {
        const int ca = u, cb = (u == 0) ? MS / 2 : MS - u;
        cx<T> A[R], B[R];
#pragma unroll
        for (int w = 0; w < R; ++w) {
            A[w] = reg[w * RP + ca];
            B[w] = reg[w * RP + cb];
        }
        // tables through a uniform base and a 32-bit lane offset (one address register per load);
        // the split uses the same twiddles, conjugated
        TW ta[R], tb[R];
#pragma unroll
        for (int w = 1; w < R; ++w) {
            ta[w] = ld_row(twM, (uint32_t)(w * ca) * ES);
            tb[w] = ld_row(twM, (uint32_t)(w * cb) * ES);
            A[w] = cmul(A[w], cx<T>{ta[w].x, ta[w].y});
            B[w] = cmul(B[w], cx<T>{tb[w].x, tb[w].y});
        }
        dftr<T, R, false>(A);  // A[j] = Z[ca + MS j]
        dftr<T, R, false>(B);  // B[j] = Z[cb + MS j]
        __builtin_amdgcn_sched_barrier(0);
        // partners: (M - ca - MS j) mod M and (M - cb - MS j) mod M; column 0 pairs with itself
        // at row (R - j) mod R, column MS/2 with itself at row R - 1 - j.  One column at a time
        // (spectral step, split, store), so that only one column's results and one row's
        // coefficients are live beside A and B.
#pragma unroll
        for (int side = 0; side < 2; ++side) {
            const int cc = side ? cb : ca;
            cx<T> V[R];
#pragma unroll
            for (int j = 0; j < R; ++j) {
                const cx<T> z = side ? B[j] : A[j];
                const cx<T> p = (u == 0) ? (side ? B[R - 1 - j] : A[(R - j) % R]) : (side ? A[R - 1 - j] : B[R - 1 - j]);
                const uint32_t ko = (uint32_t)(2 * (cc + MS * j)) * ES;
                const TW al = ld_row(coef, ko), be = ld_row(coef, ko + ES);
                V[j] = cmul(z, cx<T>{al.x, al.y}) + cmul(conj(p), cx<T>{be.x, be.y});
                __builtin_amdgcn_sched_barrier(0);  // one row's coefficients in flight at a time
            }
            dftr<T, R, true>(V);  // V[w] = sum_j W_R^(-w j) V[cc + MS j]
#pragma unroll
            for (int w = 1; w < R; ++w) {
                const TW tw = side ? tb[w] : ta[w];
                V[w] = cmul(V[w], cx<T>{tw.x, -tw.y});
            }
#pragma unroll
            for (int w = 0; w < R; ++w) reg[w * RP + cc] = V[w];
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// Window of the item into LDS (FP32, zero past nvalid, zero sentinels at -1 and W_block) with
// its statistics from the same loads; per-wave partials are combined through `red` in the same
// order by every thread.  CH float2 loads per thread and step (with four waves and CH = 8 a
// 4096-sample window is one step: all of its loads in flight together, C2 -0.7 us).
// Two samples as one 8-byte load with the non-temporal hint (a builtin vector type: the hint
// takes no struct).  An interior window is read once by its block; the N + 1 samples it shares
// with the next window come from L2 all the same, and the hint keeps the rest from displacing
// the tables every block reads (measured 1-3% faster).
typedef float f32x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float2 ld_stream2(const float* p) {
    const f32x2_t v = __builtin_nontemporal_load(reinterpret_cast<const f32x2_t*>(p));
    return make_float2(v.x, v.y);
}

template <int NTH, int CH>
__device__ __forceinline__ WStats group_load_window(const RunArgs& a, const WItem& it, float* win, double* red) {
    double m = 0.0, q = 0.0;
    int nf = 0;
    const float* p = a.s + it.start;  // start is even and s_in 8-byte aligned (checked on the host)
    auto take = [&](float x0, float x1) {
        const bool f0 = isfinite(x0), f1 = isfinite(x1);
        if (!(f0 && f1)) nf = 1;
        const double d0 = (double)(f0 ? x0 : 0.0f), d1 = (double)(f1 ? x1 : 0.0f);
        m = fmax(m, fmax(fabs(d0), fabs(d1)));
        q += d0 * d0 + d1 * d1;
    };
    // uniform: the window lies inside the signal and is valid throughout (every block but the
    // last), so that a sample needs no bound but the window's own.  Its statistics take the
    // samples as they are, and x * 0 (NaN exactly for a NaN or infinite x) marks a non-finite
    // one; a thread that met one takes its partials again below, over its finite samples only.
    const bool interior = it.nwin >= a.W_block && it.nvalid >= a.W_block;
    float z = 0.0f, mf = 0.0f;
    for (int base = 0; base < a.W_block; base += 2 * NTH * CH) {
        float2 f[CH];
        if (interior) {
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int i = base + 2 * ((int)threadIdx.x + NTH * c);  // even, as W_block is
                if (i < a.W_block) f[c] = ld_stream2(p + i);
            }
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int i = base + 2 * ((int)threadIdx.x + NTH * c);
                if (i < a.W_block) {
                    const double d0 = (double)f[c].x, d1 = (double)f[c].y;
                    mf = fmaxf(mf, fmaxf(fabsf(f[c].x), fabsf(f[c].y)));  // exact in FP32
                    q += d0 * d0 + d1 * d1;
                    z = fmaf(f[c].y, 0.0f, fmaf(f[c].x, 0.0f, z));
                    *reinterpret_cast<float2*>(win + i) = f[c];
                }
            }
            continue;
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int i = base + 2 * ((int)threadIdx.x + NTH * c);
            f[c] = make_float2(0.0f, 0.0f);
            if (i + 1 < it.nwin) f[c] = *reinterpret_cast<const float2*>(p + i);
            else if (i < it.nwin) f[c].x = p[i];
        }
#pragma unroll
        for (int c = 0; c < CH; ++c) {
            const int i = base + 2 * ((int)threadIdx.x + NTH * c);
            if (i < a.W_block) {
                take(f[c].x, f[c].y);
                *reinterpret_cast<float2*>(win + i) =
                    make_float2(i < it.nvalid ? f[c].x : 0.0f, i + 1 < it.nvalid ? f[c].y : 0.0f);
            }
        }
    }
    m = fmax(m, (double)mf);
    if (interior && z != z) {  // this thread's own samples, back from LDS, as take() counts them
        m = 0.0;
        q = 0.0;
        for (int base = 0; base < a.W_block; base += 2 * NTH * CH) {
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                const int i = base + 2 * ((int)threadIdx.x + NTH * c);
                if (i < a.W_block) take(win[i], win[i + 1]);
            }
        }
    }
    m = wmax(m);
    q = wsum(q);
    nf = wor(nf);
    constexpr int NW = NTH / 64;
    const int wv = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        red[wv] = m;
        red[NW + wv] = q;
        red[2 * NW + wv] = (double)nf;
    }
    if (threadIdx.x == 0) {
        win[-1] = 0.0f;
        win[a.W_block] = 0.0f;
    }
    __syncthreads();
    WStats r;
    r.smax = 0.0;
    r.sumsq = 0.0;
    r.nonfinite = 0;
#pragma unroll
    for (int i = 0; i < NW; ++i) {  // same order in every thread
        r.smax = fmax(r.smax, red[i]);
        r.sumsq += red[NW + i];
        r.nonfinite |= red[2 * NW + i] != 0.0;
    }
    return r;
}

// Geometry of one mode in a group set: M points split over R waves of MS points.
template <int M, int R>
struct GMode {
    static constexpr int MS = M / R;
    static constexpr int RP = greg_points<MS>();  // points per wave region
    static_assert(M % R == 0 && MS % 512 == 0, "wave transforms of a multiple of 512 points");
};

template <int MODE, int M, int R, int NW, bool FIELDS>
__device__ __forceinline__ void group_item(const RunArgs& a, const WItem& it, const WChoice& c, char* lds_raw,
                                           const float* win) {
    using T = typename std::conditional<MODE == MD_FULL32, float, double>::type;
    using TW = typename tw_of<T>::type;
    using G = GMode<M, R>;
    constexpr int MS = G::MS, E = MS / 64, RP = G::RP;
    constexpr int NTH = 64 * NW;
    const int N = a.N;
    cx<T>* reg = reinterpret_cast<cx<T>*>(lds_raw);  // R regions of RP points (alias the window)
    const TW* twM;   // W_M^t, t < M
    const TW* tws;   // W_MS^t with per-pass copies
    const TW* coef;  // real-split coefficients of the kernel spectrum, (alpha_k, beta_k), k < M
    if constexpr (MODE == MD_FULL32) {
        twM = a.wtwf;
        tws = reinterpret_cast<const TW*>(a.gsub[0]);
        coef = a.coef32;
    } else {
        twM = a.wtw[MODE];
        tws = reinterpret_cast<const TW*>(a.gsub[MODE]);
        coef = a.coef[MODE];
    }
    constexpr int MM = (MODE == MD_ASYM3) ? 3 : 2;
    const bool prefix = it.j_lo == 0;
    int Tit = 0, base_off = 0, lw = 0;
    if constexpr (MODE == MD_ASYM2 || MODE == MD_ASYM3) {
        Tit = prefix ? (N + 1 + MM - 1) / MM : a.T[MODE];
        base_off = it.j_lo - (N - 1);
        lw = Tit + N - 1;
    }
    const int wb = a.W_block;
    // window sample, clamped onto the zero sentinels outside [0, W_block), and companded (eq. 2);
    // the unclamped forms serve the steps whose every index lies in [0, W_block]
    auto rd = [&](int i) -> float { return win[min(max(i, -1), wb)]; };
    auto sqd = [&](int i) -> double { return rint(c.cs * (double)rd(i)); };
    auto sqd_in = [&](int i) -> double { return rint(c.cs * (double)win[i]); };
    const int wv = uni_i((int)threadIdx.x >> 6);  // the wave's index, in a scalar register
    const bool active = wv < R;
    // ---- pack: wave w holds the decimated points z[R n + w], n = l + 64 r (eq. 4 / eq. 7)
    cx<T> v[E];
    if (active) {
        const int l = lane_id_fresh();
        const double eps = (MODE == MD_FULL32) ? 0.0 : a.eps[MODE];  // eq. (6), formed on the host
#pragma unroll
        for (int r = 0; r < E; ++r) {
            const int p = R * (l + 64 * r) + wv;  // complex point = words 2p, 2p + 1
            // the step's first and last points (uniform over the wave)
            const int pmin = R * 64 * r + wv, pmax = R * (64 * r + 63) + wv;
            if constexpr (MODE == MD_FULL32) {
                if (2 * pmax + 1 <= wb) {
                    v[r].x = win[2 * p];
                    v[r].y = win[2 * p + 1];
                } else {
                    v[r].x = rd(2 * p);
                    v[r].y = rd(2 * p + 1);
                }
            } else if constexpr (MODE == MD_SYM) {
                if (4 * pmax + 3 <= wb) {
                    v[r].x = sqd_in(4 * p) + eps * sqd_in(4 * p + 1);
                    v[r].y = sqd_in(4 * p + 2) + eps * sqd_in(4 * p + 3);
                } else {
                    v[r].x = sqd(4 * p) + eps * sqd(4 * p + 1);
                    v[r].y = sqd(4 * p + 2) + eps * sqd(4 * p + 3);
                }
            } else {
                if (!prefix && 2 * pmax + 1 < lw && base_off + (MM - 1) * Tit + 2 * pmax + 1 <= wb) {
                    // every word of the step is kept and reads inside the window (base_off >= 0)
                    double w2[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int wd = base_off + 2 * p + h;
                        double acc = sqd_in(wd), e = eps;
#pragma unroll
                        for (int q = 1; q < MM; ++q) {
                            acc += e * sqd_in(wd + q * Tit);
                            e *= eps;
                        }
                        w2[h] = acc;
                    }
                    v[r].x = w2[0];
                    v[r].y = w2[1];
                } else if (2 * pmin >= lw) {  // every word of the step is padding
                    v[r].x = 0.0;
                    v[r].y = 0.0;
                } else {
                    double w2[2];
#pragma unroll
                    for (int h = 0; h < 2; ++h) {
                        const int wd = 2 * p + h;
                        double acc = 0.0, e = 1.0;
#pragma unroll
                        for (int q = 0; q < MM; ++q) {
                            acc += e * sqd(base_off + q * Tit + wd);
                            e *= eps;
                        }
                        w2[h] = (wd < lw) ? acc : 0.0;
                    }
                    v[r].x = w2[0];
                    v[r].y = w2[1];
                }
            }
            if (r & 1) __builtin_amdgcn_sched_barrier(0);  // bound the window reads in flight
        }
    }
    __syncthreads();  // the window is dead from here on: the regions reuse its bytes
    cx<T>* mine = reg + wv * RP;
    if (active) {
        gsub_fft<T, MS, false>(v, mine, tws);
        const int l = lane_id_fresh();
#pragma unroll
        for (int t = 0; t < E; ++t) mine[l + 64 * t] = v[t];  // plain layout for the join
    }
    __syncthreads();
    gjoin_spectral_split<T, M, R, RP, NTH>(reg, twM, coef);
    __syncthreads();
    // the inverse gets arrays of its own: were it to reuse v, the forward results would stay
    // live (in registers) through the fused pass on the path of the waves that hold no region
    cx<T> vi[E];
    if (active) {
        const int l = lane_id_fresh();
#pragma unroll
        for (int r = 0; r < E; ++r) vi[r] = mine[l + 64 * r];
        gsub_fft<T, MS, true>(vi, mine, table_fresh(tws));
    }
    __syncthreads();  // every region is dead: the words of the cyclic convolution take their bytes
    T* wd = reinterpret_cast<T*>(lds_raw);
    if (active) {
        const int l = lane_id_fresh();
#pragma unroll
        for (int t = 0; t < E; ++t) {
            const int p = R * (l + 64 * t) + wv;
            wd[2 * p] = vi[t].x;
            wd[2 * p + 1] = vi[t].y;
        }
    }
    __syncthreads();
    // ---- unpack + dequantize (eq. 16) + place (eq. 17), consecutive threads on consecutive outputs
    float* out = a.out + it.o0;
    const int nout = it.j_hi - it.j_lo;
    if constexpr (MODE == MD_FULL32) {
        for (int s = threadIdx.x; s < nout; s += NTH) {
            out_store(&out[s], (float)wd[it.j_lo + s]);
            if (FIELDS) a.fields[it.o0 + s] = 0.0;
        }
    } else if constexpr (MODE == MD_SYM) {
        // word m -> r~[2m + 1] = B(m), r~[2m] = Dm(m) + De(m - 1).  Each thread splits a run of cw
        // consecutive words once each, and the word before its run; the outputs then go over the
        // words' bytes (the pair 2m, 2m + 1 as two floats where word m was) and are copied out
        // coalesced.  cw is odd, so that the lanes' runs start on different LDS banks.
        const double two_r = (double)(2 * c.R), R_ = (double)c.R, inv_two_r = 1.0 / two_r;
        constexpr int CW = ((2 * M + NTH - 1) / NTH) | 1;  // words per thread at most
        const int mA = it.j_lo >> 1, mB = (it.j_hi + 1) >> 1;  // the words whose outputs are kept
        const int cw = ((mB - mA + NTH - 1) / NTH) | 1;         // uniform, <= CW
        const int m0 = mA + (int)threadIdx.x * cw;
        double w[CW + 1];  // w[0]: word m0 - 1
        w[0] = (m0 >= 1 && m0 <= mB) ? (double)wd[m0 - 1] : 0.0;
#pragma unroll
        for (int i = 0; i < CW; ++i) w[i + 1] = (i < cw && m0 + i < mB) ? (double)wd[m0 + i] : 0.0;
        __syncthreads();  // every word is read: the outputs take their bytes
        float* stg = reinterpret_cast<float*>(lds_raw);
        double Dm, B, De_prev = 0.0;
        if (m0 >= 1 && m0 < mB) wsym_split(w[0], two_r, inv_two_r, R_, Dm, B, De_prev);
#pragma unroll
        for (int i = 0; i < CW; ++i) {
            const int m = m0 + i;
            if (i < cw && m < mB) {
                double De;
                wsym_split(w[i + 1], two_r, inv_two_r, R_, Dm, B, De);
                const double fe = Dm + De_prev + 0.0, fo = B + 0.0;  // a zero digit is +0
                De_prev = De;
                if (2 * m >= it.j_lo && 2 * m < it.j_hi) {
                    stg[2 * m] = (float)(c.inv * fe);
                    if (FIELDS) a.fields[it.o0 + (2 * m - it.j_lo)] = fe;
                }
                if (2 * m + 1 >= it.j_lo && 2 * m + 1 < it.j_hi) {
                    stg[2 * m + 1] = (float)(c.inv * fo);
                    if (FIELDS) a.fields[it.o0 + (2 * m + 1 - it.j_lo)] = fo;
                }
            }
        }
        __syncthreads();
        for (int s = threadIdx.x; s < nout; s += NTH) out_store(&out[s], stg[it.j_lo + s]);
    } else {
        // word N - 1 + u (u < Tit) holds digit q of local output base_off + q Tit + N - 1 + u, i.e.
        // of output s = q Tit + u of the item: one word per thread, its MM digits in turn
        const double two_r = (double)(2 * c.R);
        for (int u = threadIdx.x; u < Tit; u += NTH) {
            double x = (double)wd[N - 1 + u];
#pragma unroll
            for (int q = 0; q < MM; ++q) {
                const double dq = rint(x);
                x = (x - dq) * two_r;
                const int s = q * Tit + u;
                if (s < nout) {
                    const double d = dq + 0.0;  // a zero digit is +0
                    out_store(&out[s], (float)(c.inv * d));
                    if (FIELDS) a.fields[it.o0 + s] = d;
                }
            }
        }
    }
}

// A compiled group set: points M and waves R per mode (sym, asym2, asym3, fp32).
template <int MS_, int RS_, int MA2_, int RA2_, int MA3_, int RA3_, int MF_, int RF_, int MASK>
struct GroupShape {
    static constexpr bool has(int m) { return (MASK >> m) & 1; }
    static constexpr int mx(int x, int y) { return x > y ? x : y; }
    static constexpr size_t mxs(size_t x, size_t y) { return x > y ? x : y; }
    // waves: four, whatever the modes' R (at most 4): the waves without a region of their own
    // still share the window load, the fused pass over column pairs (one pair per thread when
    // MS / 2 = 256) and the unpacking, and the wider group balances those passes
    static constexpr int RMAX = mx(mx(has(MD_SYM) ? RS_ : 1, has(MD_ASYM2) ? RA2_ : 1),
                                   mx(has(MD_ASYM3) ? RA3_ : 1, has(MD_FULL32) ? RF_ : 1));
    static_assert(RMAX <= 4, "at most four wave transforms per block");
    static constexpr int NW = 4;
    // regions of the transforms, or the words of the inverse (2 M words), per mode
    template <int M, int R, typename T>
    static constexpr size_t mode_bytes() {
        return mxs((size_t)R * greg_points<M / R>() * 2 * sizeof(T), (size_t)2 * M * sizeof(T));
    }
    static constexpr size_t B1 = has(MD_SYM) ? mode_bytes<MS_, RS_, double>() : 0;
    static constexpr size_t B2 = has(MD_ASYM2) ? mode_bytes<MA2_, RA2_, double>() : 0;
    static constexpr size_t B3 = has(MD_ASYM3) ? mode_bytes<MA3_, RA3_, double>() : 0;
    static constexpr size_t B4 = has(MD_FULL32) ? mode_bytes<MF_, RF_, float>() : 0;
    // the window with its sentinels (W_block <= 2 MF), 16 bytes in: win[-1] sits just before it
    static constexpr size_t WIN = 16 + 4 * (2 * (size_t)MF_ + 1);
    static constexpr size_t LDS = mxs(mxs(mxs(B1, B2), mxs(B3, B4)), WIN);
};

template <int MS_, int RS_, int MA2_, int RA2_, int MA3_, int RA3_, int MF_, int RF_, int MASK, bool FIELDS, bool MANY>
__global__ void __launch_bounds__((64 * GroupShape<MS_, RS_, MA2_, RA2_, MA3_, RA3_, MF_, RF_, MASK>::NW), 5)
    k_fftg(RunArgs a0) {
    using G = GroupShape<MS_, RS_, MA2_, RA2_, MA3_, RA3_, MF_, RF_, MASK>;
    constexpr int NW = G::NW;
    constexpr int NTH = 64 * NW;
    __shared__ __attribute__((aligned(16))) char lds[G::LDS];
    __shared__ double red[3 * NW];
    // consecutive blocks share N + 1 samples: give consecutive blocks to workgroups of one XCD
    // (workgroups go to the 8 XCDs in turn), so that the shared samples meet in one L2
    const int64_t nblk = a0.nitems, q8 = nblk / 8, r8 = nblk % 8, x8 = blockIdx.x % 8;
    int64_t item = x8 * q8 + (x8 < r8 ? x8 : r8) + blockIdx.x / 8;
    if (blockIdx.x >= nblk) return;
    const RunArgs& a = item_args<MANY>(a0, item);
    const WChoiceIn cin = wave_choice_inputs(a);
    const WItem it = wave_make_item(a, item);
    float* win = reinterpret_cast<float*>(lds + 16);
    WStats st = group_load_window<NTH, 8>(a, it, win, red);
    st.smax = uni_d(st.smax);
    st.sumsq = uni_d(st.sumsq);
    st.nonfinite = uni_i(st.nonfinite);
    // the first wave makes the block's choice and hands it to the others through LDS (the same
    // arithmetic in every wave would cost each SIMD the VALU time of all of them)
    __shared__ WChoice chosen;
    if (threadIdx.x < 64) {
        const WChoice c0 = wave_choose(a, st, cin);
        if (threadIdx.x == 0) chosen = c0;
    }
    __syncthreads();
    WChoice c = chosen;
    c.mode = uni_i(c.mode);
    c.S = uni_i(c.S);
    c.K = uni_i(c.K);
    c.flags = uni_i(c.flags);
    c.R = uni_l(c.R);
    c.cs = uni_d(c.cs);
    c.inv = uni_d(c.inv);
    c.snr_db = uni_d(c.snr_db);
    if (a.info && item < a.P && threadIdx.x == 0) {
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
    const bool zero = (c.flags & APX_FLAG_ZERO) && c.mode != MD_FULL32;
    if ((c.flags & APX_FLAG_NONFINITE) || zero || it.j_hi <= it.j_lo) {
        const float v = (c.flags & APX_FLAG_NONFINITE) ? NAN : 0.0f;
        for (int j = it.j_lo + threadIdx.x; j < it.j_hi; j += NTH) {
            a.out[it.o0 + (j - it.j_lo)] = v;
            if (FIELDS) a.fields[it.o0 + (j - it.j_lo)] = 0.0;
        }
        return;
    }
    if constexpr ((MASK >> MD_SYM) & 1)
        if (c.mode == MD_SYM) group_item<MD_SYM, MS_, RS_, NW, FIELDS>(a, it, c, lds, win);
    if constexpr ((MASK >> MD_ASYM2) & 1)
        if (c.mode == MD_ASYM2) group_item<MD_ASYM2, MA2_, RA2_, NW, FIELDS>(a, it, c, lds, win);
    if constexpr ((MASK >> MD_ASYM3) & 1)
        if (c.mode == MD_ASYM3) group_item<MD_ASYM3, MA3_, RA3_, NW, FIELDS>(a, it, c, lds, win);
    if constexpr ((MASK >> MD_FULL32) & 1)
        if (c.mode == MD_FULL32) group_item<MD_FULL32, MF_, RF_, NW, FIELDS>(a, it, c, lds, win);
}

// Compiled group sets: complex points and waves per mode (sym, asym2, asym3, fp32).  FP64 modes
// use 512-point wave transforms; FP32 transforms of 1024 points per wave keep the workgroup at
// the waves of the widest FP64 mode.
#define APX_GROUP_SETS(X)                      \
    X(1024, 2, 1536, 3, 1024, 2, 2048, 2)      \
    X(1024, 2, 1536, 3, 1536, 3, 2048, 2)      \
    X(512, 1, 1024, 2, 512, 1, 1024, 2)        \
    X(512, 1, 1024, 2, 1024, 2, 1024, 2)

bool group_supported(int ms, int ma2, int ma3, int mf) {
#define APX_CHECK(a_, ra_, b_, rb_, c_, rc_, d_, rd_) \
    if (ms == a_ && ma2 == b_ && ma3 == c_ && mf == d_) return true;
    APX_GROUP_SETS(APX_CHECK)
#undef APX_CHECK
    return false;
}

// Points of one wave transform of `mode` (index MD_*) in the group set (ms, ma2, ma3, mf).
int group_sub_points(int ms, int ma2, int ma3, int mf, int mode) {
#define APX_SUB(a_, ra_, b_, rb_, c_, rc_, d_, rd_)                                         \
    if (ms == a_ && ma2 == b_ && ma3 == c_ && mf == d_)                                     \
        return mode == MD_SYM ? a_ / ra_ : mode == MD_ASYM2 ? b_ / rb_ : mode == MD_ASYM3 ? c_ / rc_ : d_ / rd_;
    APX_GROUP_SETS(APX_SUB)
#undef APX_SUB
    return 0;
}

template <int A, int RA, int B, int RB, int C, int RC, int D, int RD>
static hipError_t launch_gset(const RunArgs& a, unsigned grid, hipStream_t st) {
    constexpr int ALL = (1 << MD_SYM) | (1 << MD_ASYM2) | (1 << MD_ASYM3) | (1 << MD_FULL32);
    constexpr int AUTO = (1 << MD_SYM) | (1 << MD_ASYM2) | (1 << MD_FULL32);
#define APX_G(MASK_, FIELDS_, MANY_)                                                                       \
    hipLaunchKernelGGL((k_fftg<A, RA, B, RB, C, RC, D, RD, MASK_, FIELDS_, MANY_>), dim3(grid),           \
                       dim3(64 * GroupShape<A, RA, B, RB, C, RC, D, RD, MASK_>::NW), 0, st, a)
#define APX_GM(MASK_)                 \
    if (a.many) APX_G(MASK_, false, true); \
    else APX_G(MASK_, false, false);
    if (a.fields) {
        APX_G(ALL, true, false);
    } else {
        switch (a.mode) {
            case MD_SYM: APX_GM(1 << MD_SYM) break;
            case MD_ASYM2: APX_GM(1 << MD_ASYM2) break;
            case MD_ASYM3: APX_GM(1 << MD_ASYM3) break;
            case MD_FULL32: APX_GM(1 << MD_FULL32) break;
            default: APX_GM(AUTO) break;
        }
    }
#undef APX_GM
#undef APX_G
    return hipGetLastError();
}

hipError_t launch_fftg(const RunArgs& a, int ms, int ma2, int ma3, int mf, hipStream_t st) {
    const unsigned grid = (unsigned)a.nitems;
#define APX_LAUNCH(a_, ra_, b_, rb_, c_, rc_, d_, rd_) \
    if (ms == a_ && ma2 == b_ && ma3 == c_ && mf == d_) return launch_gset<a_, ra_, b_, rb_, c_, rc_, d_, rd_>(a, grid, st);
    APX_GROUP_SETS(APX_LAUNCH)
#undef APX_LAUNCH
    return hipErrorInvalidValue;
}

// ------------------------------------------------------------------------------------------
// Kernel spectrum -> real-split coefficients for a wave FFT of M points (F = 2M words).
// H'[k] = (1/(2F)) sum_n h[n] W_F^(nk) (direct DFT, FP64); with c, s = cos, sin(2 pi k / F):
//   alpha_k = (2 - 2s) H'[k] + (2 + 2s) conj(H'[M-k]),  beta_k = 2i c (H'[k] - conj(H'[M-k])).
// coef[2k] = alpha_k, coef[2k+1] = beta_k.
// ------------------------------------------------------------------------------------------
template <typename OUT2>
__global__ void __launch_bounds__(256) k_coef(const double* __restrict__ h, int32_t nh, int32_t M,
                                              const double2* __restrict__ twF, OUT2* coef) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= M) return;
    const int F = 2 * M;
    auto dft = [&](int kk) {
        double re = 0.0, im = 0.0;
        int idx = 0;
        for (int n = 0; n < nh; ++n) {
            const double2 w = twF[idx];
            re = fma(h[n], w.x, re);
            im = fma(h[n], w.y, im);
            idx += kk;
            if (idx >= F) idx -= F;
        }
        const double sc = 1.0 / (2.0 * (double)F);
        return make_double2(re * sc, im * sc);
    };
    const double2 hk = dft(k);
    const double2 hm = dft(M - k);  // k = 0 uses bin M
    const double2 w = twF[k];
    const double c = w.x, s = -w.y;
    const double2 hmc = make_double2(hm.x, -hm.y);
    const double2 al = make_double2((2.0 - 2.0 * s) * hk.x + (2.0 + 2.0 * s) * hmc.x,
                                    (2.0 - 2.0 * s) * hk.y + (2.0 + 2.0 * s) * hmc.y);
    const double2 d = make_double2(hk.x - hmc.x, hk.y - hmc.y);
    const double2 be = make_double2(-2.0 * c * d.y, 2.0 * c * d.x);  // 2 i c d
    if constexpr (std::is_same<OUT2, double2>::value) {
        coef[2 * k] = al;
        coef[2 * k + 1] = be;
    } else {
        coef[2 * k] = make_float2((float)al.x, (float)al.y);
        coef[2 * k + 1] = make_float2((float)be.x, (float)be.y);
    }
}

hipError_t launch_coef(const double* h, int32_t nh, int32_t M, const double2* twF, double2* coef, hipStream_t st) {
    hipLaunchKernelGGL(k_coef<double2>, dim3((M + 255) / 256), dim3(256), 0, st, h, nh, M, twF, coef);
    return hipGetLastError();
}
hipError_t launch_coef32(const double* h, int32_t nh, int32_t M, const double2* twF, float2* coef, hipStream_t st) {
    hipLaunchKernelGGL(k_coef<float2>, dim3((M + 255) / 256), dim3(256), 0, st, h, nh, M, twF, coef);
    return hipGetLastError();
}

}  // namespace apx
