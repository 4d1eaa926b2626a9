// Shared between the device kernels and the host engine of libapx.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "apx.h"

namespace apx {

constexpr int NT = 256;  // threads per workgroup for every block kernel

// Table 1, "Companding range" row: largest R_max = N S_q K_q with error-free unpacking in FP64.
constexpr int64_t SYM_BOUND = 97667;
constexpr int64_t ASYM2_BOUND = 43165096;
constexpr int64_t ASYM3_BOUND = 97667;

// Mode indices used inside the library (same numbering as apx_mode).
enum { MD_FULL32 = 0, MD_SYM = 1, MD_ASYM2 = 2, MD_ASYM3 = 3, MD_AUTO = 4, MD_FULL64 = 5 };

// Device-resident statistics of a prepared kernel.
struct KState {
    double kmax;       // ||k||_inf over the N given taps
    double krms;       // root second moment over the N given taps
    double ck[4];      // c_k = K_q / ||k||_inf per packed mode (index = mode)
    int32_t nonfinite; // k holds a NaN or infinity
    int32_t pad;
};

// Everything one launch of a block kernel needs (passed by value).
struct RunArgs {
    const float* s;
    int64_t L;
    float* out;          // r_out, out_len entries
    int64_t out_len;     // L + N - 1 with the N given by the caller
    double* fields;      // debug: r~ at every output instead of r (nullable)
    apx_block_info* info;
    int32_t N;           // odd tap count (N_odd)
    int32_t W_block;
    int32_t W;
    int32_t mode;        // MD_* (MD_AUTO = per-block choice)
    int64_t P;           // blocks
    int32_t cand_mask;   // MD_AUTO: bit m set = mode m is a candidate
    int32_t S[4], K[4];  // companding ranges per packed mode
    int64_t R[4];        // R_max per packed mode
    int32_t T[4];        // asymmetric part stride per mode (W / M rounded up)
    int32_t Fw[4];       // FFT length in words per mode (index 0 = FP32 full precision)
    double thr_lin;      // MD_AUTO: SNR ratio that a candidate's model must reach
    double qs_inv[4];    // per packed mode 1 / (S_q sqrt 12) and 1 / (K_q sqrt 12): sigma_v of eq. (18)
    double qk_inv[4];    //   is ||x||_inf times these
    double eps[4];       // per packed mode eps = 1 / (2 R_max) of eq. (6)
    double inv_wb;       // 1 / W_block
    double calib_db;     // MD_AUTO: offset reported in the block info
    const double* calib_dev;  // MD_AUTO: offset measured on the device for this call (nullable);
    double snr_min_db;        //   then the threshold is formed per block from snr_min_db
    const KState* ks;
    const double* kq[4]; // [1] packed symmetric taps, [2], [3] companded taps (FP64, zero padded)
    int32_t kq_len[4];   // taps per mode before padding
    int32_t kq_pad[4];   // taps per mode after padding to a multiple of 8
    const float* kf;     // FP32 taps, zero padded to kf_pad
    const double* kd;    // FP64 taps, zero padded to kf_pad
    int32_t kf_pad;
    int32_t pad0;
    const double2* spec[4];  // FFT-core kernel spectra per packed mode, Fw/2 + 1 entries
    const float2* spec32;    // FFT-core FP32 kernel spectrum
    const double2* twd;      // twiddle tables: exp(-2 pi i t / F), t < F, at twd + F
    const float2* twf;
    // wave-per-block FFT core: per mode, W_M^t (t < M) tables and real-split coefficients
    const double2* wtw[4];
    const float2* wtwf;
    const double2* coef[4];
    const float2* coef32;
    // multi-wave FFT core: per mode, the table of one wave transform (W_MS^t with its per-pass
    // copies; float2 for index 0, the FP32 slot, double2 otherwise)
    const void* gsub[4];
    double sigma_s;  // > 0: the signal's sigma in the SNR model for every block (else block rms)
    double sigma_k;  // > 0: the kernel's sigma in the SNR model (else the taps' root second moment)
    int64_t nitems;            // work items of the launch: P (time-domain and integer cores) or
                               // P + 1 (FFT cores: block 0's prefix item), or the sum over signals
    // multi-signal launch: the arguments of every signal (built on the host, one RunArgs per
    // signal), the signal of each launch item, and (in a signal's own RunArgs) its first item
    const RunArgs* many;
    const int32_t* many_sig;
    int64_t item0;
};

// Host launchers (kernels.hip).
hipError_t launch_prepare_kernel(const float* k_in, int32_t N_given, int32_t N_odd, int32_t reverse,
                                 KState* ks, float* kf, double* kd, int32_t kf_pad,
                                 double* kq1, double* kq2, double* kq3, const int32_t* K, const int64_t* R,
                                 int32_t kq1_pad, int32_t kq23_pad, hipStream_t st);
hipError_t launch_spectrum(const double* taps, int32_t ntaps, int32_t Fw, const double2* twd,
                           double2* spec, hipStream_t st);
hipError_t launch_spectrum32(const float* taps, int32_t ntaps, int32_t Fw, const float2* twf,
                             float2* spec, hipStream_t st);
hipError_t launch_td(const RunArgs& a, size_t lds_bytes, int tile, hipStream_t st);  // tile: 4 or 8 outputs per thread
hipError_t launch_fft(const RunArgs& a, int logF, hipStream_t st);
hipError_t launch_calib(const RunArgs& a, int64_t block, int32_t Q, double* partial, int32_t nparts,
                        hipStream_t st);
// device address and size of the library's calibration scratch on the current device
hipError_t noalloc_scratch(void** ptr, size_t* bytes);
// marginal fit (model 0 Laplacian, 1 Weibull) of n samples; out: 4 doubles on the device
hipError_t launch_fit_marginal(const float* x, int64_t n, int32_t model, double* out, hipStream_t st);
// offset = measured - model SNR from launch_calib's partials, written to out[0] (device), and the
// SNR ratio a candidate's model must reach for snr_min_db, 10^((snr_min_db - offset) / 10), to
// out[1] (krms_override > 0 replaces the taps' root second moment, as RunArgs::sigma_k)
hipError_t launch_calib_finish(const double* partial, int32_t nparts, const KState* ks, int32_t Q, double* out,
                               double krms_override, double snr_min_db, hipStream_t st);
hipError_t fft_set_lds(int logF);
size_t td_lds_bytes(int mode, int N_odd, int W_block, int T2, int T3);
// wave-per-block FFT core (fftw.hip)
hipError_t upload_dft_constants(const double2* w32, const double2* w24);
bool wave_supported(int ms, int ma2, int ma3, int mf);
hipError_t launch_fftw(const RunArgs& a, int ms, int ma2, int ma3, int mf, hipStream_t st);
// group-of-waves FFT core (fftw.hip): sizes are multiples of 512 points
bool group_supported(int ms, int ma2, int ma3, int mf);
int group_sub_points(int ms, int ma2, int ma3, int mf, int mode);
hipError_t launch_fftg(const RunArgs& a, int ms, int ma2, int ma3, int mf, hipStream_t st);
// multi-pass FFT core (kernels.hip): transforms of 2^logmw complex points per block,
// BIG_LOGMW_MIN <= logmw <= BIG_LOGMW_MAX (BIG_LOGMW_MAX_FP32 for FP32), through a device
// scratch of 2^logmw points per item
constexpr int BIG_LOGMW_MIN = 10, BIG_LOGMW_MAX = 15, BIG_LOGMW_MAX_FP32 = 16;
bool big_supported(int logmw, bool fp32);
size_t big_item_bytes();
hipError_t launch_big_spectrum(const double* h, int32_t nh, int32_t F, const double2* twF, void* spec, bool fp32,
                               hipStream_t st);
hipError_t launch_big(const RunArgs& a, int mode, int logmw, void* items, void* scratch, const void* twF1,
                      const void* twF2, const void* twMW, const void* twF, const void* H, hipStream_t st);
hipError_t launch_coef(const double* h, int32_t nh, int32_t M, const double2* twF, double2* coef, hipStream_t st);
hipError_t launch_coef32(const double* h, int32_t nh, int32_t M, const double2* twF, float2* coef, hipStream_t st);
int fft_max_logF();
int fft_min_logF();

// batched cross-correlation matching (kernels.hip)
struct BatchLaunch {
    int mode, logW;
    const RunArgs* targs;   // one per pair
    const int2* items;      // (pair, block) per item; block P = the prefix item of block 0
    int32_t nitems, chunk, grid, npairs;
    unsigned int* counter;
    unsigned long long* keys;
    const int32_t* Ngiven;  // taps per pair as given
    int64_t* lag;
    float* val;
    hipStream_t st;
};
constexpr int BATCH_LOGW_MIN = 11, BATCH_LOGW_MAX = 14;
size_t batch_lds_bytes(int mode, int logW);
hipError_t batch_occupancy(int mode, int logW, int* per_cu);
hipError_t launch_batch(const BatchLaunch& b);

// filter bank on split-precision MFMA (fbank.hip)
enum { FB_F16X3 = 0, FB_BF16X3 = 1 };
constexpr int FB_WAVES = 8;  // waves per workgroup; 128 outputs per wave and tile
struct FbLaunch {
    int prec, KS;           // precision, k-steps of 16 taps (padded taps = 16 KS)
    const float* x;
    int32_t C;
    int64_t L, ldx;
    const void* frag;       // split tap fragments (fb_prepare)
    int32_t F;
    int64_t Lout;           // L + N - 1
    float* y;
    int64_t ldy;
    int grid;
    hipStream_t st;
};
int fb_ks_for(int N);
int64_t fb_tile_rows();
hipError_t fb_prepare(const float* h, int32_t F, int32_t N, int32_t KS, int32_t prec, void* frag, hipStream_t st);
hipError_t fb_occupancy(int32_t prec, int32_t KS, int* per_cu);
hipError_t fb_launch(const FbLaunch& b);

}  // namespace apx
