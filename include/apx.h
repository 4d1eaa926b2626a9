/*
 * apx -- packed approximate overlap-save convolution and cross-correlation on MI355X (gfx950).
 *
 * Method: Anam & Andreopoulos, "Throughput Scaling Of Convolution For Error-Tolerant
 * Multimedia Applications" (arXiv 1201.3018).  The input is cut into overlapping blocks
 * (Section II); each block is companded to integers with its own scale (eq. 2), packed several
 * samples per FP64 word (symmetric packing eqs. 4-6, asymmetric packing eqs. 7-8), convolved on
 * the packed words by a time-domain or FFT core (eq. 9), unpacked (eqs. 11-15), inverse-companded
 * (eq. 16) and placed (eq. 17).  The packing per block can follow an SNR target (Section IV.D,
 * eqs. 18-19).
 *
 * Conventions for every call below.
 *   - Array pointers are DEVICE pointers unless the comment says "host".  The caller owns every
 *     buffer it passes; the library keeps no caller pointer after the enqueued work completes.
 *   - Signal inputs s_in (and a served request's s) must be 8-byte aligned: the window loaders
 *     read sample pairs.  A misaligned one gives APX_E_INVALID before anything is launched.
 *     (Every device allocation is; a view that starts an odd number of floats into one is not.)
 *     The batch's references may start anywhere.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).  Work is enqueued on it
 *     and the call returns without waiting, unless the comment says the call synchronizes.
 *   - Return codes only; nothing throws across this boundary.  Shape and bound errors are found
 *     on the host before anything is launched.  apx_last_error() gives a message for the last
 *     failure on the calling thread.
 *   - A context is used by one host thread at a time.
 *   - Outputs are FP32.  Blocks whose window holds a NaN or infinity give NaN outputs and set
 *     APX_FLAG_NONFINITE in their block report.
 */
#ifndef APX_H
#define APX_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    APX_OK = 0,
    APX_E_INVALID = -1,      /* bad shape or argument */
    APX_E_BOUND = -2,        /* explicit packed mode with R_max beyond Table 1's range */
    APX_E_NOMEM = -3,        /* device allocation failed */
    APX_E_DEVICE = -4,       /* a HIP call failed (also a fault surfacing from earlier work) */
    APX_E_UNSUPPORTED = -5   /* valid request this build does not handle (e.g. size limits) */
} apx_status;

/* Packing per block (Section III.A options i-iii) */
typedef enum {
    APX_FULL_FP32 = 0,   /* no packing: FP32 overlap-save (option iii) */
    APX_SYM = 1,         /* symmetric packing, eqs. (4)-(6), two samples per FP64 word */
    APX_ASYM2 = 2,       /* asymmetric packing with M = 2, eq. (7) */
    APX_ASYM3 = 3,       /* asymmetric packing with M = 3, eq. (7) */
    APX_AUTO_SNR = 4,    /* per block: symmetric, else asymmetric M=2, else FP32, by the
                            calibrated model SNR of eqs. (18)-(19) against snr_min_db */
    APX_FULL_FP64 = 5    /* no packing, FP64 arithmetic (time-domain core only) */
} apx_mode;

/* Tier-2 convolution core.  APX_CORE_INT8 computes the companded block convolution
   r~ = s~ * k~ (eq. 2 on both operands) of a fixed packed mode's S_q, K_q exactly on the int8
   matrix cores (balanced base-128 digits when S_q or K_q exceed 127, up to 16319), then eq. (16):
   no FP64 packing, so it is exact whatever Table 1's bound says and its outputs equal the packed
   cores' wherever their unpacking is exact.  Fixed packed modes only; one wavefront per block.
   APX_CORE_AUTO: N <= 129 runs a fixed packed mode on APX_CORE_INT8 (when its LDS fits) and other
   modes on the time-domain core; longer kernels run on the FFT core. */
typedef enum { APX_CORE_AUTO = 0, APX_CORE_TIME = 1, APX_CORE_FFT = 2, APX_CORE_INT8 = 3 } apx_core;
typedef enum { APX_CONV = 0, APX_XCORR = 1 } apx_op;

typedef struct {
    int32_t mode;         /* apx_mode */
    int32_t core;         /* apx_core */
    int32_t Sq, Kq;       /* companding ranges of eq. (2) for fixed packed modes; 0 = the
                             largest S_q = K_q whose R_max = N S_q K_q (eq. 3) fits the mode */
    double snr_min_db;    /* APX_AUTO_SNR: required SNR per block */
    double calib_db;      /* APX_AUTO_SNR: offset added to the model SNR (apx_calibrate) */
    int32_t allow_unsafe; /* 1: accept R_max beyond the bound (unpacking may then be wrong) */
    int32_t fft_variant;  /* FFT core implementation: 0 = automatic (the autotuner's entry for
                             the shape if there is one, else 3, else 2, where the sizes are
                             supported, else 1), 1 = one 256-thread workgroup per block with LDS
                             passes, 2 = one wavefront per block, 3 = a group of 512-point
                             wavefront transforms per block (2 and 3: supported sizes only),
                             4 = multi-pass transforms through a device scratch (fixed packed
                             modes, 2^11 to 2^16 words, and FP32, to 2^17 words; taken by
                             itself where a fixed mode's or FP32's words exceed 2^14; one signal
                             per launch, no apx_many) */
    double sigma_s;       /* > 0: the signal's sigma in eq. (18) for every block (a source-level
                             value, e.g. from apx_fit_marginal, Section IV.D); 0 = each block's
                             root second moment.  The block maximum still sets sigma_v. */
    double sigma_k;       /* > 0: the kernel's sigma in eq. (18); 0 = the taps' root second moment */
} apx_params;

#define APX_FLAG_NONFINITE 1
#define APX_FLAG_ZERO 2

/* Per-block report (one per overlap-save block), written by the device. */
typedef struct {
    int32_t mode;         /* apx_mode the block ran in */
    int32_t flags;        /* APX_FLAG_* */
    int32_t Sq, Kq;       /* companding ranges used (0 for full precision) */
    int64_t rmax;         /* R_max of eq. (3) */
    double cs;            /* block companding factor c_s of eq. (2) */
    double smax;          /* ||s||_inf of the block window */
    double rms;           /* root second moment of the block window */
    double snr_pred_db;   /* calibrated model SNR (+inf for full precision) */
} apx_block_info;

typedef struct apx_ctx_s* apx_ctx;
typedef struct apx_kernel_s* apx_kernel;

/* Context on one HIP device (creates no stream).  Builds the twiddle tables.  Synchronizes. */
apx_status apx_create(int device, apx_ctx* out);
apx_status apx_destroy(apx_ctx ctx);

/* Host only.  Overlap-save geometry of Section III: N_odd = N rounded up to odd (one zero tap
 * appended, Section III opening), W = W_block - N_odd - 1 outputs per block (must be even and
 * >= 2 N_odd), P = ceil(L / W) blocks.  Any output pointer may be NULL. */
apx_status apx_geometry(int64_t L, int32_t N, int32_t W_block, int32_t* N_odd, int32_t* W, int64_t* P);

/* Prepare a kernel k (device, N FP32 taps) for one operation and block size (Section IV,
 * "Initialization").  W_block = 0 takes the block size apx_tune chose for this shape, else the
 * default rule (the smallest power of two with W >= 2 N, at least 1024 up to 129 taps); with
 * params->core = APX_CORE_AUTO and fft_variant = 0 the core and FFT implementation are the
 * tuned ones when the context's table has this shape.  The rest of the preparation
 * (Section IV,
 * "Initialization"): ||k||_inf, companding of k (eq. 2) for every mode the parameters can use,
 * symmetric packing of k (eq. 5, with eps^-1 = 2 R_max multiplying the even taps), and, for the
 * FFT core, the kernel spectra, all kept on the device.  APX_XCORR stores the time-reversed
 * taps: correlation c[l] = sum_n s[l+n] k[n] is the convolution with reversed k.  Copies k;
 * the handle owns its buffers.  Enqueued on `stream`. */
apx_status apx_kernel_create(apx_ctx ctx, const float* k, int32_t N, int32_t op, int32_t W_block,
                             const apx_params* params, void* stream, apx_kernel* out);
apx_status apx_kernel_destroy(apx_kernel kern);

/* Run the prepared operation on s_in (device, L FP32 samples, L >= N).
 * r_out (device, L + N - 1 FP32): convolution r_out[m] = sum_n s_in[m-n] k[n] (eq. 1), or for
 * APX_XCORR r_out[i] = c[i - (N-1)], lags -(N-1) .. L-1.
 * info (device, nullable): one apx_block_info per block (P entries, apx_geometry). */
apx_status apx_run(apx_ctx ctx, apx_kernel kern, const float* s_in, int64_t L, float* r_out,
                   apx_block_info* info, void* stream);

/* The integer fields r~ = s~ * k~ of Section III.B at every output position, as exact integers
 * in FP64 (device, L + N - 1 entries), for a kernel prepared in a fixed packed mode.  Runs the
 * same kernels as apx_run with the dequantization replaced by a store of r~. */
apx_status apx_debug_fields(apx_ctx ctx, apx_kernel kern, const float* s_in, int64_t L, double* fields,
                            void* stream);

/* Calibration of the SNR model (Section IV.D): measures on block `block` of s_in the SNR of the
 * companded convolution at S_q = K_q = Q against FP64, subtracts the model SNR of eqs. (18)-(19)
 * at the same Q and stores the difference in the kernel (used by APX_AUTO_SNR when
 * params.calib_db is NaN) and in *offset_db (host).  Synchronizes `stream`. */
apx_status apx_calibrate(apx_ctx ctx, apx_kernel kern, const float* s_in, int64_t L, int32_t block, int32_t Q,
                         void* stream, double* offset_db);

/* Marginal-CDF fit of a source's samples (Section IV.D, Fig. 4), for the sigma of eq. (18).
 * x: device, n FP32 samples.  model: APX_MARGINAL_LAPLACE (zero-mean Laplacian, scale b = mean |x|
 * by maximum likelihood, sigma = sqrt(2) b) or APX_MARGINAL_WEIBULL (two-parameter Weibull of
 * the positive samples by maximum likelihood: Newton's method on the shape equation, then the
 * scale; sigma = lambda sqrt(Gamma(1 + 2/kappa)); samples <= 0 are left out).
 * out (host, 4 doubles): scale (b or lambda), shape (1 or kappa), sigma, samples used.  One
 * workgroup runs the whole fit on the device; synchronizes `stream`.
 * APX_E_INVALID: null pointers, n < 1, unknown model, or fewer than 2 positive samples for a
 * Weibull fit. */
typedef enum { APX_MARGINAL_LAPLACE = 0, APX_MARGINAL_WEIBULL = 1 } apx_marginal;
apx_status apx_fit_marginal(apx_ctx ctx, const float* x, int64_t n, int32_t model, double* out, void* stream);

/* One-shot convolution / correlation: kernel_create + run + kernel_destroy. Synchronizes. */
apx_status apx_conv(apx_ctx ctx, const float* s_in, int64_t L, const float* k, int32_t N, int32_t W_block,
                    const apx_params* params, float* r_out, apx_block_info* info, void* stream);
apx_status apx_xcorr(apx_ctx ctx, const float* s_in, int64_t L, const float* k, int32_t N, int32_t W_block,
                     const apx_params* params, float* r_out, apx_block_info* info, void* stream);

/* apx_run for an APX_AUTO_SNR kernel with the SNR target and the calibration of this call
 * (Section IV.D): the calibration of apx_calibrate (measured against FP64 at S_q = K_q = 8 on
 * block `calib_block` of s_in, minus the model of eqs. 18-19) is computed on the device ahead of
 * the run, on the same stream, and used by this call only; snr_min_db replaces the kernel's
 * target.  A calibration block without quantization error or without signal gives offset 0.
 * workspace: device, apx_workspace_bytes() bytes, owned by the caller; calls that overlap in
 * time need distinct workspaces.  Allocates nothing and never synchronizes, so several requests
 * may share one prepared kernel concurrently on different streams. */
size_t apx_workspace_bytes(void);
apx_status apx_run_auto(apx_ctx ctx, apx_kernel kern, const float* s_in, int64_t L, float* r_out,
                        apx_block_info* info, double snr_min_db, int32_t calib_block, void* workspace,
                        void* stream);

/* apx_run_auto for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the calibration workspace is the
 * library's own device array of 2048 bytes per device (apx_workspace_bytes() must fit it, else
 * APX_E_UNSUPPORTED), so the call allocates nothing and never synchronizes.  Every call on one
 * device shares that array: calls that overlap on one device race and must not be issued
 * (serialize them on one stream, or use apx_run_auto with distinct workspaces).  Nothing in the
 * array needs clearing between calls: each call writes every entry it reads.  Same arguments,
 * results and errors as apx_run_auto otherwise. */
apx_status apx_run_auto_noalloc(apx_ctx ctx, apx_kernel kern, const float* s_in, int64_t L, float* r_out,
                                apx_block_info* info, double snr_min_db, int32_t calib_block, void* stream);

/* ---- Autotuning ---------------------------------------------------------------------------
 * apx_tune: for taps k (device, N FP32), the operation and params->mode (and its companding and
 * SNR settings), prepares the kernel on every core that can run the shape (time-domain core
 * with 4 and 8 outputs per thread, integer matrix cores for fixed packed modes with one to three
 * output tiles per pass over the taps, FFT core with LDS passes / one wavefront per block / a
 * group of wavefronts per block, each with its own radix plan) at W_block, or, for W_block = 0,
 * at the three smallest power-of-two block sizes with W >= 2 N; times each on a synthetic signal
 * of L_hint samples (0: 64 blocks, at least 2^16 samples; the number of blocks a call has decides
 * how much parallelism each core finds, so tune for the length you run) on `stream`, in three
 * rounds that visit every candidate in turn, each candidate keeping its fastest round (the runs
 * rotate over up to 16 copies of the signal, at most 512 MiB, so that inputs come from HBM rather
 * than the last-level cache); records the
 * fastest in the context's table
 * (used by apx_kernel_create for this shape from then on) and in the table file
 * (APX_TUNE_FILE, else $HOME/.cache/apx_tune.txt; entries of other architectures are kept),
 * from which apx_create loads this device's entries.  Allocates a test signal and output,
 * synchronizes `stream`.  out (host): the choice and its time per output.  The packed modes
 * give the same outputs on every core wherever their unpacking is exact; the choice of block
 * size changes the per-block companding, so W_block = 0 is for callers that leave it free.
 * APX_E_UNSUPPORTED: no core runs the shape.
 * apx_tune_describe (host only): the device's table and the last tuning's timings as text. */
typedef struct {
    int32_t core;         /* apx_core */
    int32_t fft_variant;  /* as apx_params.fft_variant (FFT core) */
    int32_t W_block;
    int32_t tile;         /* integer core: output tiles per pass over the taps; time-domain core:
                             outputs per thread, 4 or 8 (0: FFT core) */
    double ps_per_output; /* measured time per output sample, picoseconds */
} apx_tuned;
apx_status apx_tune(apx_ctx ctx, const float* k, int32_t N, int32_t op, int32_t W_block, const apx_params* params,
                    int64_t L_hint, void* stream, apx_tuned* out);
apx_status apx_tune_describe(apx_ctx ctx, char* buf, int32_t size);

/* Host only.  A short description of how a prepared kernel runs (core, FFT kernel and transform
 * sizes, companding ranges per mode) written into buf (host, size bytes, NUL-terminated). */
apx_status apx_kernel_describe(apx_kernel kern, char* buf, int32_t size);

/* ---- Many signals, one kernel -----------------------------------------------------------------
 * n signals s_i (DEVICE, L_i FP32 samples each, 8-byte aligned, L_i >= N) convolved (or, for an
 * APX_XCORR kernel, correlated) with one prepared kernel in ONE launch over every (signal, block)
 * item: the overlap-save blocks of all signals are independent (Section II), so they form one
 * work list.  r_out_i (DEVICE, L_i + N - 1 FP32) receives exactly what apx_run(kern, s_i) writes,
 * and info_i (DEVICE, P_i entries, nullable) its block report.  Fixed modes and APX_AUTO_SNR with
 * the kernel's own calibration (apx_calibrate / params.calib_db), on any core.
 * apx_many_create: s, r_out, info are HOST arrays of n device pointers (info, or any entry of it,
 *   may be NULL), L a host array of n lengths.  Builds the signal table and the per-item signal
 *   index on the device (owned by the handle, 40 + 4 P_i bytes per signal); synchronizes
 *   `stream`.  The pointers are kept: the memory must stay valid until apx_many_destroy, its
 *   contents may change between runs.  The kernel handle must outlive the many handle.
 *   APX_E_INVALID: null or misaligned pointers, n < 1, L_i < N, a geometry error;
 *   APX_E_UNSUPPORTED: more than 2^31 - 1 work items; APX_E_NOMEM: device allocation failed.
 * apx_many_run: one launch of the kernel's block core over all items, enqueued on `stream`;
 *   allocates nothing and can be captured into a HIP graph.  Runs share no scratch memory, so
 *   they may overlap when their outputs do not.
 * apx_many_describe (host only): signals, work items and the kernel's launch as text. */
typedef struct apx_many_s* apx_many;
apx_status apx_many_create(apx_ctx ctx, apx_kernel kern, int32_t n, const float* const* s, const int64_t* L,
                           float* const* r_out, apx_block_info* const* info, void* stream, apx_many* out);
apx_status apx_many_run(apx_ctx ctx, apx_many many, void* stream);
apx_status apx_many_describe(apx_many many, char* buf, int32_t size);
apx_status apx_many_destroy(apx_many many);

/* ---- Batched cross-correlation matching ----------------------------------------------------
 * n pairs (reference s_t of L_t samples, template k_t of N_t taps).  For each pair the
 * correlation c_t[l] = sum_n s_t[l+n] k_t[n], l in [-(N_t-1), L_t-1], is computed exactly as
 * apx_xcorr would with the same fixed mode and the pair's W_block (apx_batch_blocks), and only
 * its maximum is kept: lag_out[t] = the lag of the largest value (ties: smallest lag),
 * val_out[t] = that value (FP32 output of eq. 16).  NaN outputs (blocks whose window holds a NaN
 * or infinity) take no part; with no other output lag_out = INT64_MIN and val_out = NaN.
 * This is the matching use of correlation in the paper's applications (Section IV.B).
 *
 * All pairs share one packed FFT length of 2^logW words (11..14); each pair's block size is the
 * largest one whose packed words fit it (FP32: W_block = 2^logW samples; symmetric: 2^(logW+1);
 * asymmetric M: W = M (2^logW - N + 1) rounded down to even), with W >= 2N (Section III
 * opening).  One persistent launch processes every (pair, block) item.
 *
 * apx_batch_create: refs, tmpl are HOST arrays of n DEVICE pointers (FP32), L and N host arrays.
 *   Pointers are kept by the batch: the reference and template memory must stay valid and
 *   unchanged until apx_batch_destroy (templates are read at create time, references at every
 *   run).  params->mode must be APX_FULL_FP32, APX_SYM, APX_ASYM2 or APX_ASYM3 (else
 *   APX_E_UNSUPPORTED); Sq/Kq/allow_unsafe as for apx_kernel_create.  logW = 0 autotunes: every
 *   FFT length that fits all pairs and a work-grab of 1, 2 or 4 items are timed on `stream`
 *   (this runs the batch several times) and the fastest is kept.  Synchronizes `stream`.
 * apx_batch_run: lag_out (device, n int64), val_out (device, n float).  Enqueued on `stream`;
 *   allocates nothing and launches three kernels (clear, persistent matching, finish), so it can
 *   be captured into a HIP graph.  Runs of one batch must not overlap (they share its counters).
 * apx_batch_blocks (host only): W_block per pair (host array of n, nullable), the FFT length
 *   log2 and the number of work items.
 * apx_batch_describe (host only): kernel, grid, grab size and the tuning table as text. */
typedef struct apx_batch_s* apx_batch;
apx_status apx_batch_create(apx_ctx ctx, int32_t n, const float* const* refs, const int64_t* L,
                            const float* const* tmpl, const int32_t* N, const apx_params* params, int32_t logW,
                            void* stream, apx_batch* out);
apx_status apx_batch_run(apx_ctx ctx, apx_batch batch, int64_t* lag_out, float* val_out, void* stream);
apx_status apx_batch_blocks(apx_batch batch, int32_t* W_block, int32_t* logW, int32_t* nitems);
apx_status apx_batch_describe(apx_batch batch, char* buf, int32_t size);
apx_status apx_batch_destroy(apx_batch batch);
/* One shot: create (autotuned) + run + destroy.  Synchronizes. */
apx_status apx_xcorr_argmax_batch(apx_ctx ctx, int32_t n, const float* const* refs, const int64_t* L,
                                  const float* const* tmpl, const int32_t* N, const apx_params* params,
                                  int64_t* lag_out, float* val_out, void* stream);

/* ---- Filter bank on split-precision matrix cores (the full-precision comparator) ----------------
 * y[(c F + f) ldy + t] = sum_n x[c ldx + t - n] h[f N + n], t in [0, L + N - 1): the direct
 * convolution of eq. (1) for C channels and F filters, computed as a Hankel-form GEMM on
 * half-precision MFMA with FP32 accumulation.  Every sample and tap is split into a high and a
 * low half-precision part and three products (hi*hi, hi*lo, lo*hi) are accumulated:
 *   APX_FB_F16X3  FP16 parts, lo = fp16(2^12 (v - hi)) (accurate to about 2^-21 per product;
 *                 |x| and |h| must stay below 32768),
 *   APX_FB_BF16X3 BF16 parts, lo = bf16(v - hi) (about 2^-16 per product, any FP32 range).
 * apx_fbank_create: h (device, F x N FP32, row-major), 1 <= F <= 32, 1 <= N <= 512.  Copies the
 *   taps into split fragments owned by the handle.  Enqueued on `stream`.
 * apx_fbank_run: x (device, C rows of ldx >= L floats), y (device, C F rows of ldy >= L + N - 1
 *   floats, not overlapping x).  One persistent launch; allocates nothing.  Enqueued on `stream`.
 * apx_fbank_describe (host only): kernel and launch shape as text. */
typedef enum { APX_FB_F16X3 = 0, APX_FB_BF16X3 = 1 } apx_fb_prec;
typedef struct apx_fbank_s* apx_fbank;
apx_status apx_fbank_create(apx_ctx ctx, const float* h, int32_t F, int32_t N, int32_t prec, void* stream,
                            apx_fbank* out);
apx_status apx_fbank_run(apx_ctx ctx, apx_fbank fb, const float* x, int32_t C, int64_t L, int64_t ldx, float* y,
                         int64_t ldy, void* stream);
apx_status apx_fbank_describe(apx_fbank fb, char* buf, int32_t size);
apx_status apx_fbank_destroy(apx_fbank fb);

/* ---- Serving: a request loop with admission by HBM budget and resident kernels ---------------
 * Convolution and correlation requests of mixed L and N (the paper's problem statement,
 * Section II, with the SNR constraint of Section IV.D per request) are queued by
 * apx_server_submit and served by one scheduler thread per server:
 *   - admission in arrival order while the request's device memory (input, output, workspace,
 *     its share of a launch table, and its prepared kernel on a cache miss, sized by a dry run
 *     of the preparation, with any twiddle tables it adds to the context) fits hbm_budget and
 *     fewer than max_inflight requests are on the device; idle cached kernels are evicted
 *     (least recently used) to make room; a request that could never fit is refused at submit
 *     (APX_E_NOMEM);
 *   - continuous batching: the requests admitted together that share a prepared kernel run as
 *     ONE multi-signal launch of its block core (as apx_many_run) after their copies in and
 *     their per-request calibrations, on one of n_streams HIP streams, then their copies out;
 *     batches admitted while others run overlap with them on the device;
 *   - prepared kernels stay resident, keyed by (kernel_key, N, op, W_block, mode).
 * Each request is computed exactly as apx_run_auto (APX_AUTO_SNR, calibration on its own block
 * 0) or apx_run (fixed modes) would compute it alone; the mix changes only timing.
 * While a server exists, the context belongs to its scheduler thread: the caller must not use
 * the same context for other calls. */
typedef struct {
    int64_t hbm_budget;    /* bytes of device memory for requests and cached kernels (>= 1 MiB) */
    int32_t n_streams;     /* 1..64 */
    int32_t max_inflight;  /* requests on the device at once (>= 1) */
} apx_server_config;

typedef struct {
    uint64_t kernel_key;   /* equal keys must carry equal taps */
    const float* k;        /* host, N taps; read when the kernel is not cached */
    int32_t N;
    int32_t op;            /* APX_CONV or APX_XCORR */
    const float* s;        /* host (pinned memory lets the copy overlap), L >= N samples */
    int64_t L;
    float* r_out;          /* host (pinned), L + N - 1 samples, written when the request completes */
    double snr_min_db;     /* APX_AUTO_SNR: per-block target */
    int32_t W_block;       /* 0: the server's choice (time-domain core up to 129 taps, else FFT core,
                              smallest power of two with W >= 2N) */
    int32_t mode;          /* apx_mode; APX_AUTO_SNR for the SNR-driven packing */
} apx_request;
/* s, k and r_out must stay valid until the request's completion has been returned by
 * apx_server_poll (or apx_server_drain returned). */

typedef struct {
    uint64_t ticket;
    int32_t status;        /* APX_OK or the failure */
    int32_t core;          /* apx_core the request ran on */
    int32_t W_block, N;
    int64_t L;
    double t_submit, t_admit, t_done;  /* apx_server_now() clock, seconds */
} apx_completion;

typedef struct {
    int64_t submitted, completed, failed, rejected;
    int64_t kernel_hits, kernel_misses, evictions;
    int64_t peak_bytes;     /* largest budgeted device memory in use */
    int64_t reserved_bytes; /* device memory held by the server's allocator */
    int32_t cached_kernels, pad;
    int64_t launches;       /* block-kernel launches: one per batch of requests sharing a kernel */
} apx_server_counters;

typedef struct apx_server_s* apx_server;
apx_status apx_server_create(apx_ctx ctx, const apx_server_config* cfg, apx_server* out);
/* Thread safe.  *ticket identifies the request's completion. */
apx_status apx_server_submit(apx_server srv, const apx_request* req, uint64_t* ticket);
/* Up to max completions (host array), oldest first; waits up to wait_ms for the first one. */
apx_status apx_server_poll(apx_server srv, apx_completion* out, int32_t max, int32_t* n, int32_t wait_ms);
/* Blocks until every submitted request has completed. */
apx_status apx_server_drain(apx_server srv);
apx_status apx_server_stats(apx_server srv, apx_server_counters* out);
/* Finishes queued work, then releases everything. */
apx_status apx_server_destroy(apx_server srv);
/* The server's clock (steady, seconds). */
double apx_server_now(void);

const char* apx_status_str(apx_status st);
const char* apx_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* APX_H */
