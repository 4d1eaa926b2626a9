// Filter bank on matrix cores: y[c][f][t] = sum_n x[c][t-n] h[f][n] for C channels and F <= 32
// filters, as a Hankel-form GEMM per channel:
//   y[t0 + i][f] = sum_k xw[i + k] B[k][f],  xw[j] = x[t0 - (NPAD-1) + j],  B[k][f] = h[f][NPAD-1-k]
// (the taps are reversed so that every row reads ascending samples).  Products run on
// 32x32x16 half-precision MFMA with FP32 accumulation; every operand is split into a high and a
// low half-precision part and three passes (hi*hi, hi*lo, lo*hi) recover close to FP32 accuracy.
// FP16: lo = fp16((v - hi) 2^12) keeps the residual out of the subnormal range, the hi*lo and
// lo*hi products go to a second accumulator scaled back by 2^-12.  BF16: lo = bf16(v - hi).
//
// Tiles: a workgroup of NW waves computes MT = 128 NW consecutive outputs of one channel for
// all 32 filter columns.  Wave w owns rows [128 w, 128 w + 128) as four 32-row MFMA tiles.  In
// Hankel form the A fragment of row tile r at k-step s equals the fragment of row tile 0 at
// step s + 2r, so a wave loads each A fragment once and keeps a ring of seven in registers.
// Unaligned fragment starts are avoided by eight copies of the window shifted by 0..7 samples;
// every lane reads 16-byte aligned chunks of the copy matching its row.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.h"

namespace apx {

typedef _Float16 h8 __attribute__((ext_vector_type(8)));
typedef __bf16 bh8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

template <int PREC>
struct Split;

template <>
struct Split<FB_F16X3> {
    using T = _Float16;
    using V = h8;
    static constexpr float LO_SCALE = 4096.0f;
    static constexpr float LO_INV = 1.0f / 4096.0f;
    __device__ static __forceinline__ void split(float v, T& hi, T& lo) {
        hi = (T)v;
        lo = (T)((v - (float)hi) * LO_SCALE);
    }
    __device__ static __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
    }
};

template <>
struct Split<FB_BF16X3> {
    using T = __bf16;
    using V = bh8;
    static constexpr float LO_SCALE = 1.0f;
    static constexpr float LO_INV = 1.0f;
    __device__ static __forceinline__ void split(float v, T& hi, T& lo) {
        hi = (T)v;
        lo = (T)(v - (float)hi);
    }
    __device__ static __forceinline__ f32x16 mma(V a, V b, f32x16 c) {
        return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
    }
};

// B fragments of the reversed, split taps: frag[(part * KS + s) * 64 + lane] holds
// B[16 s + 8 (lane / 32) + j][lane % 32], j < 8 (part 0 = hi, part 1 = lo).
template <int PREC>
__global__ void __launch_bounds__(NT) k_fb_frag(const float* __restrict__ h, int32_t F, int32_t N, int32_t KS,
                                                typename Split<PREC>::V* __restrict__ frag) {
    using S = Split<PREC>;
    const int idx = blockIdx.x * NT + threadIdx.x;
    if (idx >= KS * 64) return;
    const int s = idx / 64, lane = idx % 64;
    const int f = lane & 31, kh = lane >> 5;
    const int npad = 16 * KS;
    typename S::V hi, lo;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        const int k = 16 * s + 8 * kh + j;
        const int n = npad - 1 - k;
        const float v = (f < F && n < N) ? h[(int64_t)f * N + n] : 0.0f;
        typename S::T a, b;
        S::split(v, a, b);
        hi[j] = a;
        lo[j] = b;
    }
    frag[s * 64 + lane] = hi;
    frag[(KS + s) * 64 + lane] = lo;
}

// Workgroup barrier that orders LDS only: each wave waits for its own LDS operations, not for
// its global stores (__syncthreads would drain a tile's output stores before the next tile).
// The wavefront fences keep the compiler from moving memory accesses across the barrier.
__device__ __forceinline__ void wave_lds_order() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xc07f);  // lgkmcnt(0)
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int KS, int NW>
struct FbGeom {
    static constexpr int NPAD = 16 * KS;
    static constexpr int MT = 128 * NW;     // outputs per tile
    static constexpr int CL = MT + NPAD;     // samples per shifted copy
    static constexpr int CS = CL + 8;        // copy stride in elements (16 B of bank offset)
    static constexpr size_t B_BYTES = (size_t)2 * KS * 64 * 16;
    static constexpr size_t A_BYTES = (size_t)2 * 8 * CS * 2;
    static constexpr int WS = CL + 8;        // raw window samples (the last chunk reads 7 past CL)
    static constexpr size_t W_BYTES = (size_t)4 * WS;
    static constexpr int TS = 36;            // transpose row stride in floats (16 B aligned, banks spread)
    static constexpr size_t T_BYTES = (size_t)NW * 32 * TS * 4;
    static constexpr size_t LDS = B_BYTES + A_BYTES + W_BYTES + T_BYTES;
};

template <int PREC, int KS, int NW>
__global__ void __launch_bounds__(64 * NW) k_fbank(const float* __restrict__ x, int32_t C, int64_t L, int64_t ldx,
                                                   const typename Split<PREC>::V* __restrict__ frag, int32_t F,
                                                   int64_t Lout, float* __restrict__ y, int64_t ldy,
                                                   int64_t ntiles) {
    using S = Split<PREC>;
    using T = typename S::T;
    using V = typename S::V;
    using G = FbGeom<KS, NW>;
    constexpr int NTH = 64 * NW;
    extern __shared__ __attribute__((aligned(16))) char lds[];
    V* Bs = (V*)lds;
    T* As = (T*)(lds + G::B_BYTES);
    float* Ws = (float*)(lds + G::B_BYTES + G::A_BYTES);
    float* Tw = (float*)(lds + G::B_BYTES + G::A_BYTES + G::W_BYTES) + (size_t)(threadIdx.x >> 6) * (32 * G::TS);
    for (int i = threadIdx.x; i < 2 * KS * 64; i += NTH) Bs[i] = frag[i];

    // contiguous range of (channel, tile) items per workgroup
    const int64_t nitems = (int64_t)C * ntiles;
    const int64_t per = (nitems + gridDim.x - 1) / gridDim.x;
    const int64_t it0 = (int64_t)blockIdx.x * per;
    const int64_t it1 = min(nitems, it0 + per);

    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 31, kh = lane >> 5, rl = i & 7;
    const bool vec_store = (ldy % 4) == 0 && (reinterpret_cast<uintptr_t>(y) & 15) == 0;  // 16-byte rows

    // The raw window of the next tile is loaded into registers (RPT samples per thread, coalesced)
    // while the current tile's products run: one workgroup fills a CU's LDS, so no other
    // workgroup would hide these loads.  The copies are then built from an LDS staging row.
    constexpr int RPT = (G::WS + NTH - 1) / NTH;
    float pre[RPT];
    auto fetch = [&](int64_t item) {
        const int c = (int)(item / ntiles);
        const int64_t t0 = (item - (int64_t)c * ntiles) * G::MT;
        const float* xc = x + (int64_t)c * ldx;
        const int64_t g0 = t0 - (G::NPAD - 1);
        const bool inside = g0 >= 0 && g0 + G::WS <= L;
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int m = threadIdx.x + k * NTH;
            const int64_t g = g0 + m;
            pre[k] = 0.0f;
            if (m < G::WS && (inside || (g >= 0 && g < L))) pre[k] = xc[g];
        }
    };
    // the staging row takes the prefetched samples after the products and before the output
    // stores, so that waiting for the loads never waits for this tile's stores
    auto stage = [&]() {
#pragma unroll
        for (int k = 0; k < RPT; ++k) {
            const int m = threadIdx.x + k * NTH;
            if (m < G::WS) Ws[m] = pre[k];
        }
    };
    if (it0 < it1) {
        fetch(it0);
        stage();
    }

    for (int64_t item = it0; item < it1; ++item) {
        const int c = (int)(item / ntiles);
        const int64_t t0 = (item - (int64_t)c * ntiles) * G::MT;
        lds_barrier();  // B and the staged window visible; the previous tile's reads of As are done
        // unconditional (the last tile fetches itself again): a load on every path lets the
        // compiler see that no load is pending at the top of the loop
        fetch(item + 1 < it1 ? item + 1 : item);
        // window copies: copy r, chunk q holds xw[8q + r .. 8q + r + 7] (hi and lo parts)
        for (int ch = threadIdx.x; ch < G::CL; ch += NTH) {
            const int r = ch & 7, q = ch >> 3;
            V hi, lo;
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                T a, b;
                S::split(Ws[ch + j], a, b);
                hi[j] = a;
                lo[j] = b;
            }
            *(V*)(As + (size_t)r * G::CS + 8 * q) = hi;
            *(V*)(As + (size_t)(8 + r) * G::CS + 8 * q) = lo;
        }
        lds_barrier();

        // A fragment of ring index j: xw[128 w + i + 8 kh + 16 j + (0..7)] from copy rl
        const T* ah_base = As + (size_t)rl * G::CS + (128 * w + i - rl + 8 * kh);
        const T* al_base = ah_base + (size_t)8 * G::CS;
        f32x16 accm[4], accc[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                accm[r][e] = 0.0f;
                accc[r][e] = 0.0f;
            }
        }
        V fh[7], fl[7];
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            fh[j] = *(const V*)(ah_base + 16 * j);
            fl[j] = *(const V*)(al_base + 16 * j);
        }
#pragma unroll
        for (int s = 0; s < KS; ++s) {
            // ring slot of fragment j is j % 7; step s uses fragments s, s+2, s+4, s+6
            fh[(s + 6) % 7] = *(const V*)(ah_base + 16 * (s + 6));
            fl[(s + 6) % 7] = *(const V*)(al_base + 16 * (s + 6));
            const V bh = Bs[s * 64 + lane];
            const V bl = Bs[(KS + s) * 64 + lane];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const V a = fh[(s + 2 * r) % 7];
                const V al = fl[(s + 2 * r) % 7];
                accm[r] = S::mma(a, bh, accm[r]);
                accc[r] = S::mma(a, bl, accc[r]);
                accc[r] = S::mma(al, bh, accc[r]);
            }
        }

        stage();  // every wave read Ws before the barrier above the products

        // D[row][f]: lane holds rows 8 (e/4) + 4 kh + (e%4) of each tile, column f = i.  Each
        // 32 x 32 block goes through the wave's own LDS region (row f, stride TS) so that one
        // store instruction writes eight whole 128-byte runs of output rows.
#pragma unroll
        for (int r = 0; r < 4; ++r) {
#pragma unroll
            for (int g = 0; g < 4; ++g) {
                float4 o;
                o.x = accm[r][4 * g + 0] + accc[r][4 * g + 0] * S::LO_INV;
                o.y = accm[r][4 * g + 1] + accc[r][4 * g + 1] * S::LO_INV;
                o.z = accm[r][4 * g + 2] + accc[r][4 * g + 2] * S::LO_INV;
                o.w = accm[r][4 * g + 3] + accc[r][4 * g + 3] * S::LO_INV;
                *(float4*)(Tw + i * G::TS + 8 * g + 4 * kh) = o;
            }
            wave_lds_order();
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                const int f = 8 * k + (lane >> 3), tc = 4 * (lane & 7);
                const float4 o = *(const float4*)(Tw + f * G::TS + tc);
                const int64_t t = t0 + 128 * w + 32 * r + tc;
                if (f < F) {
                    float* yr = y + ((int64_t)c * F + f) * ldy;
                    if (vec_store && t + 3 < Lout) {
                        *(float4*)(yr + t) = o;
                    } else {
                        const float ov[4] = {o.x, o.y, o.z, o.w};
#pragma unroll
                        for (int j = 0; j < 4; ++j)
                            if (t + j < Lout) yr[t + j] = ov[j];
                    }
                }
            }
            wave_lds_order();  // the next block's writes follow this block's reads
        }
    }
}

namespace {

template <int PREC, int KS>
hipError_t fb_launch_ks(const FbLaunch& b, bool query, int* per_cu) {
    constexpr int NW = FB_WAVES;
    using G = FbGeom<KS, NW>;
    auto kern = k_fbank<PREC, KS, NW>;
    if (query) {
        hipError_t e = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)G::LDS);
        if (e != hipSuccess) return e;
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(per_cu, kern, 64 * NW, G::LDS);
    }
    const int64_t ntiles = (b.Lout + G::MT - 1) / G::MT;
    hipLaunchKernelGGL(kern, dim3(b.grid), dim3(64 * NW), G::LDS, b.st, b.x, b.C, b.L, b.ldx,
                       (const typename Split<PREC>::V*)b.frag, b.F, b.Lout, b.y, b.ldy, ntiles);
    return hipGetLastError();
}

template <int PREC>
hipError_t fb_launch_prec(const FbLaunch& b, bool query, int* per_cu) {
    switch (b.KS) {
        case 8: return fb_launch_ks<PREC, 8>(b, query, per_cu);
        case 16: return fb_launch_ks<PREC, 16>(b, query, per_cu);
        case 32: return fb_launch_ks<PREC, 32>(b, query, per_cu);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

int fb_ks_for(int N) {
    if (N <= 128) return 8;
    if (N <= 256) return 16;
    if (N <= 512) return 32;
    return 0;
}

int64_t fb_tile_rows() { return 128 * FB_WAVES; }

hipError_t fb_prepare(const float* h, int32_t F, int32_t N, int32_t KS, int32_t prec, void* frag, hipStream_t st) {
    const int n = KS * 64;
    dim3 g((n + NT - 1) / NT);
    if (prec == FB_F16X3)
        hipLaunchKernelGGL(k_fb_frag<FB_F16X3>, g, dim3(NT), 0, st, h, F, N, KS, (h8*)frag);
    else if (prec == FB_BF16X3)
        hipLaunchKernelGGL(k_fb_frag<FB_BF16X3>, g, dim3(NT), 0, st, h, F, N, KS, (bh8*)frag);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t fb_occupancy(int32_t prec, int32_t KS, int* per_cu) {
    FbLaunch b{};
    b.KS = KS;
    return prec == FB_F16X3 ? fb_launch_prec<FB_F16X3>(b, true, per_cu) : fb_launch_prec<FB_BF16X3>(b, true, per_cu);
}

hipError_t fb_launch(const FbLaunch& b) {
    if (b.C <= 0 || b.Lout <= 0) return hipSuccess;
    return b.prec == FB_F16X3 ? fb_launch_prec<FB_F16X3>(b, false, nullptr)
                              : fb_launch_prec<FB_BF16X3>(b, false, nullptr);
}

}  // namespace apx
