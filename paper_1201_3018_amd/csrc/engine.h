// Host-side handle types of libapx shared by the C ABI (capi.cpp) and the serving engine
// (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <utility>
#include <vector>

#include "apx.h"
#include "internal.h"

constexpr int LOGF_MAX_TABLE = 14;  // twiddle tables up to F = 16384

namespace apx {
// LDS FFT core for one fixed packed mode at its own transform length (2^logmw complex points,
// kernels.hip)
bool fft1_supported(int mode, int logmw);
hipError_t fft1_set_lds(int mode, int logmw);
hipError_t launch_fft1(const RunArgs& a, int mode, int logmw, hipStream_t st);
// integer matrix-core core (kernels.hip)
int i8_ksteps(int N_odd);
int i8_kpad(int N_odd);
int i8_plane_len(int N_odd, int W);
size_t i8_lds_bytes(int plane_len, int W_block);
hipError_t launch_i8_frag(const float* kf, const KState* ks, int mode, int N_odd, int split, void* frag,
                          hipStream_t st);
hipError_t i8_set_lds(int bytes);
hipError_t launch_i8(const RunArgs& a, const void* frag, int split_s, int split_k, int plane_len, hipStream_t st);
}  // namespace apx

using apx::KState;

struct apx_ctx_s {
    int device = 0;
    double2* twd = nullptr;
    float2* twf = nullptr;
    int max_lds = 65536;
    // W_F^t tables (t < F) of any length F, built on first use
    std::map<int, std::pair<double2*, float2*>> tables;
};

struct apx_kernel_s {
    apx_ctx ctx = nullptr;
    int32_t N = 0;       // taps as given
    int32_t N_odd = 0;
    int32_t op = APX_CONV;
    int32_t W_block = 0, W = 0;
    apx_params params{};
    int core = APX_CORE_TIME;
    int logF = 0;
    int fft1_logmw = 0;  // > 0: the fixed packed mode runs k_fft1 at 2^fft1_logmw complex points
    // integer matrix-core core: B fragments (two digit planes), LDS digit-plane length, K split
    int32_t* i8frag = nullptr;
    int i8_plane = 0;
    int i8_splitk = 0;
    int32_t S[4] = {0, 0, 0, 0}, K[4] = {0, 0, 0, 0};
    int64_t R[4] = {0, 0, 0, 0};
    int32_t T[4] = {0, 0, 0, 0};
    int32_t Fw[4] = {0, 0, 0, 0};
    int32_t cand_mask = 0;
    double calib_db = 0.0;
    size_t td_lds = 0;
    bool use[4] = {false, false, false, false};  // FP32, SYM, ASYM2, ASYM3 states needed
    KState* ks = nullptr;
    float* kf = nullptr;
    double* kd = nullptr;
    double* kq[4] = {nullptr, nullptr, nullptr, nullptr};
    int32_t kq_len[4] = {0, 0, 0, 0}, kq_pad[4] = {0, 0, 0, 0};
    int32_t kf_pad = 0;
    double2* spec[4] = {nullptr, nullptr, nullptr, nullptr};
    float2* spec32 = nullptr;
    // wave-per-block FFT core
    bool wave = false;
    bool group = false;  // wave tables, run by the group-of-waves core
    int32_t wM[4] = {0, 0, 0, 0};  // complex points per mode (0 = FP32)
    double2* coef[4] = {nullptr, nullptr, nullptr, nullptr};
    float2* coef32 = nullptr;
    std::vector<void*> allocs;
    size_t dev_bytes = 0;  // device memory owned by (or carved for) this kernel
    // device buffers carved from a caller-owned pool instead of hipMalloc (batched pairs)
    char* pool = nullptr;
    size_t pool_off = 0, pool_cap = 0;
};

