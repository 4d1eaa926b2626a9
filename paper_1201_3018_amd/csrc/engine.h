// Host-side handle types of libapx shared by the C ABI (capi.cpp) and the serving engine
// (server.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
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
// tm: output tiles per pass over the taps, 1 to 3
hipError_t launch_i8(const RunArgs& a, const void* frag, int split_s, int split_k, int plane_len, int tm, hipStream_t st);
int i8_tiles(int N_odd, int W);
}  // namespace apx

using apx::KState;

namespace apx {
// Autotuning table entries: the shape asked for, and the fastest way measured to run it.
struct TuneKey {
    int32_t N_odd, op, mode, W_block;  // W_block 0: the tuner chose the block size too
    bool operator<(const TuneKey& o) const {
        if (N_odd != o.N_odd) return N_odd < o.N_odd;
        if (op != o.op) return op < o.op;
        if (mode != o.mode) return mode < o.mode;
        return W_block < o.W_block;
    }
};
struct TuneVal {
    int32_t core, variant, W_block;
    double ps_per_output;
    int32_t tile = 0;  // integer core: output tiles per pass; time-domain core: outputs per thread
                       // (0: the shape's default)
};
}  // namespace apx

struct apx_ctx_s {
    int device = 0;
    double2* twd = nullptr;
    float2* twf = nullptr;
    int max_lds = 65536;
    // W_F^t tables (t < F) of any length F, built on first use, and their device bytes
    std::map<int, std::pair<double2*, float2*>> tables;
    size_t table_bytes = 0;
    // device address of this device's copy of the library's calibration scratch
    void* scratch = nullptr;
    size_t scratch_bytes = 0;
    // autotuning table of this device's architecture (tune.cpp)
    std::string arch;
    std::map<apx::TuneKey, apx::TuneVal> tuned;
    std::string last_tune;
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
    int i8_tm = 3;  // output tiles per pass (1 to 3)
    int td_tile = 8;  // time-domain core: outputs per thread (4 or 8)
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
    // multi-pass FFT core (transforms beyond one workgroup's LDS): 2^big_logmw complex points per
    // block, its kernel spectrum, and a per-item scratch grown to the longest signal run so far
    int big_logmw = 0;
    void* big_spec = nullptr;
    void* big_scr = nullptr;
    size_t big_scr_bytes = 0;
    std::vector<void*> allocs;
    size_t dev_bytes = 0;  // device memory owned by (or carved for) this kernel
    // device buffers carved from a caller-owned pool instead of hipMalloc (batched pairs)
    char* pool = nullptr;
    size_t pool_off = 0, pool_cap = 0;
    // plan only: count the device bytes (dev_bytes, and the context tables it would add in
    // plan_tables) without allocating or launching anything
    bool plan_only = false;
    std::vector<int> plan_tables;
};

namespace apx {
// Internal entry points used by the serving engine (capi.cpp).
// Arguments of one run of k on s (device, L samples), with the checks of apx_run.
apx_status run_args(apx_kernel k, const float* s, int64_t L, float* out, apx_block_info* info, RunArgs* a);
// The per-call calibration of apx_run_auto on block `block` of a's signal for the target
// a.snr_min_db, enqueued on st; workspace: apx_workspace_bytes() device bytes; *off: device
// address of the offset (followed by the threshold ratio the block kernels compare against).
apx_status calib_on_device(apx_kernel k, const RunArgs& a, int32_t block, void* workspace, const double** off,
                           hipStream_t st);
// One launch of k's block core over every item of the signals whose arguments (item0 set) sit at
// args (device, n entries), item_sig (device, nitems entries) giving each item's signal.
apx_status launch_many(apx_kernel k, const RunArgs& first, const RunArgs* args, const int32_t* item_sig,
                       int64_t nitems, hipStream_t st);
// Device bytes a kernel prepared with these arguments would hold, plus the context tables its
// preparation would add.
apx_status kernel_plan_bytes(apx_ctx ctx, int32_t N, int32_t op, int32_t W_block, const apx_params* p,
                             size_t* bytes);
// Record a failure message for apx_last_error and return st.
apx_status set_error(apx_status st, const char* fmt, ...);
// Autotuning table (tune.cpp): load this device's entries; look one up; the default block size.
void tune_load(apx_ctx ctx);
bool tune_lookup(apx_ctx ctx, int32_t N_odd, int32_t op, int32_t mode, int32_t W_block, TuneVal* out);
int32_t default_block(int32_t N);
// The block size and core a kernel request resolves to: W_block 0 takes the tuned block size (or
// the default rule), and an automatic core and FFT implementation take the tuned ones.
void resolve_tuned(apx_ctx ctx, int32_t N, int32_t op, int32_t* W_block, apx_params* p, int32_t* tile = nullptr);
}  // namespace apx

