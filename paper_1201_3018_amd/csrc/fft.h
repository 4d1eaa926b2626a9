// LDS-resident complex FFT for one workgroup (Stockham auto-sort, radix 16/8/4/2).
//
// Used by the FFT convolution core: a real sequence of F words is transformed as a complex
// sequence of F/2 points (even words real, odd words imaginary), split into the real spectrum,
// multiplied by a resident kernel spectrum, merged back and inverted.  Twiddles come from a
// table exp(-2 pi i t / F), t < F, computed on the host in extended precision.
#pragma once

#include <type_traits>

#include <hip/hip_runtime.h>

#include "internal.h"

namespace apx {

template <typename T>
struct cx {
    T x, y;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }  // a * i

// a * (-i) for the forward transform, a * (+i) for the inverse.
template <typename T, bool INV>
__device__ __forceinline__ cx<T> rot(cx<T> a) {
    return INV ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
}

template <typename T>
struct tw_of;
template <>
struct tw_of<double> {
    using type = double2;
};
template <>
struct tw_of<float> {
    using type = float2;
};

template <typename T, bool INV>
__device__ __forceinline__ void dft2(cx<T>* v) {
    cx<T> a = v[0], b = v[1];
    v[0] = a + b;
    v[1] = a - b;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft4(cx<T>& v0, cx<T>& v1, cx<T>& v2, cx<T>& v3) {
    cx<T> t0 = v0 + v2, t1 = v0 - v2, t2 = v1 + v3, t3 = rot<T, INV>(v1 - v3);
    v0 = t0 + t2;
    v2 = t0 - t2;
    v1 = t1 + t3;
    v3 = t1 - t3;
}

template <typename T, bool INV>
__device__ __forceinline__ void dft8(cx<T>* v) {
    const T h = (T)0.70710678118654752440084436210484903928;
    cx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    cx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4<T, INV>(e0, e1, e2, e3);
    dft4<T, INV>(o0, o1, o2, o3);
    // o_k *= w8^k, w8 = exp(-+ i pi / 4)
    if (INV) {
        o1 = {(o1.x - o1.y) * h, (o1.x + o1.y) * h};
        o3 = {(-o3.x - o3.y) * h, (o3.x - o3.y) * h};
    } else {
        o1 = {(o1.x + o1.y) * h, (o1.y - o1.x) * h};
        o3 = {(o3.y - o3.x) * h, (-o3.x - o3.y) * h};
    }
    o2 = rot<T, INV>(o2);
    v[0] = e0 + o0;
    v[4] = e0 - o0;
    v[1] = e1 + o1;
    v[5] = e1 - o1;
    v[2] = e2 + o2;
    v[6] = e2 - o2;
    v[3] = e3 + o3;
    v[7] = e3 - o3;
}

// a * W_16^m, W_16 = exp(-2 pi i / 16) (forward) or its conjugate; m in [0, 9] is a constant
// after unrolling.  cos(pi/8), sin(pi/8) and 1/sqrt(2) are the exactly rounded literals.
template <typename T, bool INV>
__device__ __forceinline__ cx<T> mulw16(cx<T> a, int m) {
    const T c = (T)0.92387953251128675612818318939678828682, s = (T)0.38268343236508977172845998403039886676,
            h = (T)0.70710678118654752440084436210484903928;
    T wr = 1, wi = 0;
    switch (m) {
        case 0: return a;
        case 4: return rot<T, INV>(a);
        case 1: wr = c; wi = -s; break;
        case 2: wr = h; wi = -h; break;
        case 3: wr = s; wi = -c; break;
        case 6: wr = -h; wi = -h; break;
        case 9: wr = -c; wi = s; break;
        default: break;
    }
    return cmul(a, cx<T>{wr, INV ? -wi : wi});
}

// DFT of 16 points as 4 x 4: DFT-4 over stride 4, twiddles W_16^(n2 k1), DFT-4 over the four
// results; natural order in and out.
template <typename T, bool INV>
__device__ __forceinline__ void dft16(cx<T>* v) {
    cx<T> y[16];
#pragma unroll
    for (int n2 = 0; n2 < 4; ++n2) {
        cx<T> a0 = v[n2], a1 = v[4 + n2], a2 = v[8 + n2], a3 = v[12 + n2];
        dft4<T, INV>(a0, a1, a2, a3);
        y[n2] = a0;
        y[4 + n2] = mulw16<T, INV>(a1, n2);
        y[8 + n2] = mulw16<T, INV>(a2, 2 * n2);
        y[12 + n2] = mulw16<T, INV>(a3, 3 * n2);
    }
#pragma unroll
    for (int k1 = 0; k1 < 4; ++k1) {
        cx<T> b0 = y[4 * k1], b1 = y[4 * k1 + 1], b2 = y[4 * k1 + 2], b3 = y[4 * k1 + 3];
        dft4<T, INV>(b0, b1, b2, b3);
        v[k1] = b0;
        v[k1 + 4] = b1;
        v[k1 + 8] = b2;
        v[k1 + 12] = b3;
    }
}

template <typename T, int R, bool INV>
__device__ __forceinline__ void dftR(cx<T>* v) {
    if constexpr (R == 2) dft2<T, INV>(v);
    if constexpr (R == 4) dft4<T, INV>(v[0], v[1], v[2], v[3]);
    if constexpr (R == 8) dft8<T, INV>(v);
    if constexpr (R == 16) dft16<T, INV>(v);
}

// One Stockham pass of radix R over M complex points held in LDS (re[], im[]).
// Ns = size of the sub-transforms already done.  tw = table for F = 2M.
template <typename T, int M, int R, bool INV>
__device__ __forceinline__ void stockham_pass(T* re, T* im, int Ns, const typename tw_of<T>::type* tw) {
    constexpr int NB = M / R;
    constexpr int PER = (NB + NT - 1) / NT;
    constexpr int F = 2 * M;
    cx<T> v[PER][R];
    const int tstride = F / (Ns * R);
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int j = threadIdx.x + b * NT;
        if (NB % NT == 0 || j < NB) {
#pragma unroll
            for (int r = 0; r < R; ++r) v[b][r] = {re[j + r * NB], im[j + r * NB]};
            const int k = j & (Ns - 1);
#pragma unroll
            for (int r = 1; r < R; ++r) {
                auto w = tw[r * k * tstride];
                cx<T> c = {w.x, INV ? -w.y : w.y};
                v[b][r] = cmul(v[b][r], c);
            }
            dftR<T, R, INV>(v[b]);
        }
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < PER; ++b) {
        const int j = threadIdx.x + b * NT;
        if (NB % NT == 0 || j < NB) {
            const int k = j & (Ns - 1);
            const int base = (j - k) * R + k;
#pragma unroll
            for (int r = 0; r < R; ++r) {
                re[base + r * Ns] = v[b][r].x;
                im[base + r * Ns] = v[b][r].y;
            }
        }
    }
    __syncthreads();
}

constexpr int ilog2(int x) { return x <= 1 ? 0 : 1 + ilog2(x / 2); }

// Full complex FFT of M points in LDS.  Caller synchronizes before (data written by others);
// the last pass ends with a barrier.  Forward: exp(-2 pi i ...); inverse: unnormalized.
// LDS bytes that fft_lds<T, M> needs from re on: the two rows of M values, or for FP64 at
// M = 16 NT and 32 NT the padded complex layout of the register-resident transform (group_fft).
__host__ __device__ constexpr size_t fft_lds_bytes(bool fp64, int M) {
    const size_t rows = 2 * (size_t)M * (fp64 ? 8 : 4);
    const size_t padded = (fp64 && (M == 16 * NT || M == 32 * NT)) ? (size_t)(M + NT) * 16 : 0;
    return rows > padded ? rows : padded;
}

// DFT of E = 16 or 32 points in registers; the 32-point one is two 16-point DFTs (even and odd
// points) joined by W_32^k, read from the W_F table (F = 64 NT: W_32^k = tw[2 NT k]).
template <int E, bool INV>
__device__ __forceinline__ void dft_group(cx<double>* v, const double2* tw) {
    if constexpr (E == 16) {
        dft16<double, INV>(v);
    } else {
        static_assert(E == 32, "16 or 32 points per thread");
        cx<double> ev[16], od[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            ev[i] = v[2 * i];
            od[i] = v[2 * i + 1];
        }
        dft16<double, INV>(ev);
        dft16<double, INV>(od);
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const double2 w = tw[2 * NT * k];
            const cx<double> tk = cmul(od[k], cx<double>{w.x, INV ? -w.y : w.y});
            v[k] = ev[k] + tk;
            v[k + 16] = ev[k] - tk;
        }
    }
}

// Complex FFT of M = E NT points in FP64 (E = 16 or 32 per thread): a DFT-E in registers, then
// two radix-16 passes (E / 16 butterflies per thread), with two exchanges through LDS in a padded
// layout (point i at i + floor(i / E), which spreads a pass's strided accesses over the banks),
// where the Stockham form takes five passes through LDS and twice the barriers.  In: point
// t + NT r in v[r] of thread t; no thread may still read or write the fft_lds_bytes(true, M)
// bytes from re on (a barrier since their last use).  Out: natural order in re[], im[].
// tw: W_F^t, F = 2M.
template <int E, bool INV>
__device__ __forceinline__ void group_fft_regs(cx<double>* v, double* re, double* im, const double2* tw) {
    constexpr int M = E * NT, S = E + 1, NB = E / 16, H = M / 16;
    cx<double>* cl = reinterpret_cast<cx<double>*>(re);
    const int t = threadIdx.x;
    // first pass: DFT-E over stride NT; point t E + r goes to t S + r
    dft_group<E, INV>(v, tw);
#pragma unroll
    for (int r = 0; r < E; ++r) cl[t * S + r] = v[r];
    __syncthreads();
    cx<double> u[NB][16];
    // second pass: radix 16 over the sub-transforms of size E, twiddles W_(16E)^(r k) = W_F^(32 r k)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + NT * b, q = j / E, k = j - q * E;
        double2 w[15];  // the pass's twiddles are fetched together, ahead of the LDS reads
#pragma unroll
        for (int r = 1; r < 16; ++r) w[r - 1] = tw[32 * r * k];
#pragma unroll
        for (int r = 0; r < 16; ++r) u[b][r] = cl[j + q + 16 * S * r];
#pragma unroll
        for (int r = 1; r < 16; ++r) u[b][r] = cmul(u[b][r], cx<double>{w[r - 1].x, INV ? -w[r - 1].y : w[r - 1].y});
        dft16<double, INV>(u[b]);
    }
    __syncthreads();
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + NT * b, q = j / E, k = j - q * E;
#pragma unroll
        for (int r = 0; r < 16; ++r) cl[16 * S * q + k + S * r] = u[b][r];
    }
    __syncthreads();
    // third pass: radix 16 over the sub-transforms of size M / 16, twiddles W_M^(r j) = W_F^(2 r j)
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + NT * b;
        double2 w[15];
#pragma unroll
        for (int r = 1; r < 16; ++r) w[r - 1] = tw[2 * r * j];
#pragma unroll
        for (int r = 0; r < 16; ++r) u[b][r] = cl[j + j / E + 16 * S * r];
#pragma unroll
        for (int r = 1; r < 16; ++r) u[b][r] = cmul(u[b][r], cx<double>{w[r - 1].x, INV ? -w[r - 1].y : w[r - 1].y});
        dft16<double, INV>(u[b]);
    }
    __syncthreads();  // every padded read is done before the natural-order writes
#pragma unroll
    for (int b = 0; b < NB; ++b) {
        const int j = t + NT * b;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            re[j + H * r] = u[b][r].x;
            im[j + H * r] = u[b][r].y;
        }
    }
    __syncthreads();
}

// The same transform from natural order in re[], im[].
template <int E, bool INV>
__device__ __forceinline__ void group_fft(double* re, double* im, const double2* tw) {
    cx<double> v[E];
#pragma unroll
    for (int r = 0; r < E; ++r) v[r] = {re[threadIdx.x + NT * r], im[threadIdx.x + NT * r]};
    __syncthreads();  // every natural-order read is done before the padded layout overwrites it
    group_fft_regs<E, INV>(v, re, im, tw);
}

// FP32: radix-16 passes (fewer passes and barriers; measured 12% faster on the batched FP32
// path).  FP64: radix-8 passes (radix-16 Stockham passes hold twice the registers per point and
// measured 5-6% slower), except at M = 16 NT and 32 NT, which run group_fft.
template <typename T, int M, bool INV>
__device__ __forceinline__ void fft_lds(T* re, T* im, const typename tw_of<T>::type* tw) {
    if constexpr (std::is_same<T, double>::value && (M == 16 * NT || M == 32 * NT)) {
        group_fft<M / NT, INV>(re, im, tw);
        return;
    }
    constexpr int L2 = ilog2(M);
    constexpr int RB = std::is_same<T, float>::value ? 4 : 3;  // log2 of the main radix
    constexpr int NP = L2 / RB;
    constexpr int REM = L2 % RB;
    int Ns = 1;
#pragma unroll
    for (int p = 0; p < NP; ++p) {
        stockham_pass<T, M, (1 << RB), INV>(re, im, Ns, tw);
        Ns <<= RB;
    }
    if constexpr (REM == 3) stockham_pass<T, M, 8, INV>(re, im, Ns, tw);
    if constexpr (REM == 2) stockham_pass<T, M, 4, INV>(re, im, Ns, tw);
    if constexpr (REM == 1) stockham_pass<T, M, 2, INV>(re, im, Ns, tw);
}

// Real-signal spectral step between the forward and the inverse transform.
// In: Z = DFT_M(x_even + i x_odd).  For k in [0, M]: X2[k] = 2 X[k] (X = DFT_F(x)),
// Y[k] = X2[k] H'[k] with H' = H / (2F) prescaled, and out V'[k] such that the unnormalized
// inverse DFT_M of V' is y_even + i y_odd, y = x (*) h cyclic of length F = 2M.
template <typename T, int M>
__device__ __forceinline__ void spectral_step(T* re, T* im, const typename tw_of<T>::type* tw,
                                              const typename tw_of<T>::type* H) {
    for (int k = threadIdx.x; k <= M / 2; k += NT) {
        const int kk = (M - k) & (M - 1);
        cx<T> za = {re[k], im[k]};
        cx<T> zb = {re[kk], im[kk]};
        auto wt = tw[k];
        cx<T> w = {wt.x, wt.y};
        cx<T> A = za + conj(zb);
        cx<T> Bd = za - conj(zb);
        cx<T> wB = cmul(w, Bd);
        cx<T> x_k = A - mul_i(wB);            // X2[k]
        cx<T> x_mk = conj(A + mul_i(wB));     // X2[M-k]
        auto h0 = H[k];
        auto h1 = H[M - k];
        cx<T> yk = cmul(x_k, cx<T>{h0.x, h0.y});
        cx<T> ymk = cmul(x_mk, cx<T>{h1.x, h1.y});
        cx<T> P = yk + conj(ymk);
        cx<T> Q = yk - conj(ymk);
        cx<T> cQ = mul_i(cmul(conj(w), Q));
        cx<T> vk = P + cQ;
        re[k] = vk.x;
        im[k] = vk.y;
        if (k != 0 && kk != k) {
            cx<T> vmk = conj(P - cQ);
            re[kk] = vmk.x;
            im[kk] = vmk.y;
        }
    }
    __syncthreads();
}

// Spectrum of a real sequence after fft_lds: H'[k] = X2[k] / (4F), k in [0, M].
template <typename T, int M>
__device__ __forceinline__ void real_spectrum_out(const T* re, const T* im, const typename tw_of<T>::type* tw,
                                                  typename tw_of<T>::type* Hout) {
    const T scale = (T)1 / (T)(8 * M);
    for (int k = threadIdx.x; k <= M; k += NT) {
        const int kk = (M - k) & (M - 1);
        const int ka = k & (M - 1);
        cx<T> za = {re[ka], im[ka]};
        cx<T> zb = {re[kk], im[kk]};
        cx<T> A = za + conj(zb);
        cx<T> Bd = za - conj(zb);
        cx<T> w;
        if (k == M) {
            w = {(T)-1, (T)0};
        } else {
            auto wt = tw[k];
            w = {wt.x, wt.y};
        }
        cx<T> x = A - mul_i(cmul(w, Bd));
        Hout[k] = {x.x * scale, x.y * scale};
    }
}

}  // namespace apx
