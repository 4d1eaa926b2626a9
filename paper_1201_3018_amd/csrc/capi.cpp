// Host engine and C ABI of libapx: validation, overlap-save geometry, per-kernel device state,
// twiddle tables, launch planning.  Every arithmetic step of the convolution runs in the kernels
// of kernels.hip; the host only plans and launches.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cstdint>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "engine.h"
#include "internal.h"

using namespace apx;

namespace {

thread_local std::string g_err;

apx_status fail(apx_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

#define HIPCHK(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return fail(APX_E_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

int64_t isqrt64(int64_t x) {
    int64_t r = (int64_t)sqrt((double)x);
    while (r * r > x) --r;
    while ((r + 1) * (r + 1) <= x) ++r;
    return r;
}

int64_t bound_of(int m) {
    return m == MD_SYM ? SYM_BOUND : (m == MD_ASYM2 ? ASYM2_BOUND : ASYM3_BOUND);
}

int pad8(int n) { return (n + 7) / 8 * 8; }

int ceil_log2(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

}  // namespace

namespace {

template <typename T>
apx_status dalloc(apx_kernel k, T** p, size_t n) {
    if (k->plan_only) {
        k->dev_bytes += std::max<size_t>(n, 1) * sizeof(T);
        *p = nullptr;
        return APX_OK;
    }
    if (k->pool) {
        const size_t bytes = (std::max<size_t>(n, 1) * sizeof(T) + 255) / 256 * 256;
        if (k->pool_off + bytes > k->pool_cap) return fail(APX_E_NOMEM, "pair buffer pool exhausted");
        *p = (T*)(k->pool + k->pool_off);
        k->pool_off += bytes;
        k->dev_bytes += bytes;
        return APX_OK;
    }
    void* q = nullptr;
    hipError_t e = hipMalloc(&q, std::max<size_t>(n, 1) * sizeof(T));
    if (e != hipSuccess) return fail(APX_E_NOMEM, "hipMalloc(%zu): %s", n * sizeof(T), hipGetErrorString(e));
    k->allocs.push_back(q);
    k->dev_bytes += std::max<size_t>(n, 1) * sizeof(T);
    *p = (T*)q;
    return APX_OK;
}

void free_kernel(apx_kernel k) {
    for (void* p : k->allocs) (void)hipFree(p);
    k->allocs.clear();
    if (k->big_scr) (void)hipFree(k->big_scr);
    k->big_scr = nullptr;
    k->big_scr_bytes = 0;
}

apx_status build_twiddles(apx_ctx c) {
    const int Fmax = 1 << LOGF_MAX_TABLE;
    std::vector<double2> hd(2 * (size_t)Fmax);
    std::vector<float2> hf(2 * (size_t)Fmax);
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (int F = 2; F <= Fmax; F *= 2) {
        for (int t = 0; t < F; ++t) {
            // exp(-2 pi i t / F), angle reduced to the first octant by symmetry for accuracy
            long double ang = two_pi * (long double)t / (long double)F;
            long double cr = cosl(ang), si = -sinl(ang);
            // exact values on the axes
            if (4 * t == F) { cr = 0.0L; si = -1.0L; }
            if (2 * t == F) { cr = -1.0L; si = 0.0L; }
            if (4 * t == 3 * F) { cr = 0.0L; si = 1.0L; }
            hd[F + t] = make_double2((double)cr, (double)si);
            hf[F + t] = make_float2((float)cr, (float)si);
        }
    }
    hd[0] = hd[1] = make_double2(1.0, 0.0);
    hf[0] = hf[1] = make_float2(1.0f, 0.0f);
    HIPCHK(hipMalloc((void**)&c->twd, hd.size() * sizeof(double2)));
    HIPCHK(hipMalloc((void**)&c->twf, hf.size() * sizeof(float2)));
    HIPCHK(hipMemcpy(c->twd, hd.data(), hd.size() * sizeof(double2), hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(c->twf, hf.data(), hf.size() * sizeof(float2), hipMemcpyHostToDevice));
    return APX_OK;
}

long double two_pi_l() { return 6.283185307179586476925286766559005768L; }

// exp(-2 pi i t / F), t < F, in extended precision (exact on the axes), rounded once.
void fill_twiddles(int F, double2* d) {
    for (int t = 0; t < F; ++t) {
        long double cr, si;
        if (t == 0) { cr = 1.0L; si = 0.0L; }
        else if (4 * (int64_t)t == F) { cr = 0.0L; si = -1.0L; }
        else if (2 * (int64_t)t == F) { cr = -1.0L; si = 0.0L; }
        else if (4 * (int64_t)t == 3 * (int64_t)F) { cr = 0.0L; si = 1.0L; }
        else {
            long double ang = two_pi_l() * (long double)t / (long double)F;
            cr = cosl(ang);
            si = -sinl(ang);
        }
        d[t] = make_double2((double)cr, (double)si);
    }
}

// Entries after the F-entry table of a one-wave FFT size (F a multiple of 512): the radix-8
// passes' twiddles in the order the lanes read them, W_F^{8 r k} at (r-1) E + k (k < E = F/64)
// and then W_F^{r j} at 7 E + (r-1) F/8 + j (j < F/8), r = 1..7, copies of the table's values.
int pass_table_len(int F) { return (F % 512 == 0) ? 7 * (F / 64) + 7 * (F / 8) : 0; }

apx_status get_table(apx_ctx c, int F, double2** d, float2** f) {
    auto it = c->tables.find(F);
    if (it == c->tables.end()) {
        const int n = F + pass_table_len(F);
        std::vector<double2> hd(n);
        std::vector<float2> hf(n);
        fill_twiddles(F, hd.data());
        if (n > F) {
            const int E = F / 64, F8 = F / 8;
            for (int r = 1; r < 8; ++r) {
                for (int k = 0; k < E; ++k) hd[F + (r - 1) * E + k] = hd[8 * r * k];
                for (int j = 0; j < F8; ++j) hd[F + 7 * E + (r - 1) * F8 + j] = hd[r * j];
            }
        }
        for (int i = 0; i < n; ++i) hf[i] = make_float2((float)hd[i].x, (float)hd[i].y);
        double2* dd = nullptr;
        float2* ff = nullptr;
        hipError_t e = hipMalloc((void**)&dd, n * sizeof(double2));
        if (e == hipSuccess) e = hipMalloc((void**)&ff, n * sizeof(float2));
        if (e == hipSuccess) e = hipMemcpy(dd, hd.data(), n * sizeof(double2), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(ff, hf.data(), n * sizeof(float2), hipMemcpyHostToDevice);
        if (e != hipSuccess) {
            if (dd) (void)hipFree(dd);
            if (ff) (void)hipFree(ff);
            return fail(APX_E_DEVICE, "twiddle table of %d points: %s", F, hipGetErrorString(e));
        }
        it = c->tables.emplace(F, std::make_pair(dd, ff)).first;
        c->table_bytes += (size_t)n * (sizeof(double2) + sizeof(float2));
    }
    if (d) *d = it->second.first;
    if (f) *f = it->second.second;
    return APX_OK;
}

// smallest complex size the wave core handles that holds `words` real words (2M >= words)
int wave_m_for(int words) {
    const int ms[4] = {512, 1024, 1536, 2048};
    for (int m : ms)
        if (2 * m >= words) return m;
    return 0;
}

apx_status geometry(int64_t L, int32_t N, int32_t W_block, int32_t* N_odd, int32_t* W, int64_t* P) {
    if (N < 1) return fail(APX_E_INVALID, "kernel length N = %d must be >= 1", N);
    if (W_block < 4) return fail(APX_E_INVALID, "W_block = %d too small", W_block);
    const int32_t no = (N % 2) ? N : N + 1;
    const int32_t w = W_block - no - 1;
    if (w < 2 * no || (w % 2) != 0)
        return fail(APX_E_INVALID, "W = W_block - N - 1 = %d must be even and >= 2N = %d (N odd = %d)", w, 2 * no, no);
    if (N_odd) *N_odd = no;
    if (W) *W = w;
    if (P) {
        if (L < 1) return fail(APX_E_INVALID, "input length L = %lld must be >= 1", (long long)L);
        *P = (L + w - 1) / w;
    }
    return APX_OK;
}

RunArgs make_args(apx_kernel k, const float* s, int64_t L, float* out, double* fields, apx_block_info* info,
                  int64_t P) {
    RunArgs a;
    memset(&a, 0, sizeof a);
    a.s = s;
    a.L = L;
    a.out = out;
    a.out_len = L + k->N - 1;
    a.fields = fields;
    a.info = info;
    a.N = k->N_odd;
    a.W_block = k->W_block;
    a.W = k->W;
    a.mode = k->params.mode;
    a.P = P;
    a.nitems = P + (k->core == APX_CORE_FFT ? 1 : 0);  // the FFT cores add block 0's prefix item
    a.cand_mask = k->cand_mask;
    for (int m = 0; m < 4; ++m) {
        a.S[m] = k->S[m];
        a.K[m] = k->K[m];
        a.R[m] = k->R[m];
        a.T[m] = k->T[m];
        a.Fw[m] = k->Fw[m];
        a.kq[m] = k->kq[m];
        a.kq_len[m] = k->kq_len[m];
        a.kq_pad[m] = k->kq_pad[m];
        a.spec[m] = k->spec[m];
    }
    const double calib = isnan(k->params.calib_db) ? k->calib_db : k->params.calib_db;
    a.calib_db = calib;
    a.thr_lin = pow(10.0, (k->params.snr_min_db - calib) / 10.0);
    const double r12 = sqrt(12.0);
    for (int m = 1; m < 4; ++m) {
        a.qs_inv[m] = k->S[m] > 0 ? 1.0 / ((double)k->S[m] * r12) : 0.0;
        a.qk_inv[m] = k->K[m] > 0 ? 1.0 / ((double)k->K[m] * r12) : 0.0;
        a.eps[m] = k->R[m] > 0 ? 1.0 / (2.0 * (double)k->R[m]) : 0.0;
    }
    a.inv_wb = 1.0 / (double)k->W_block;
    a.ks = k->ks;
    a.kf = k->kf;
    a.kd = k->kd;
    a.kf_pad = k->kf_pad;
    a.spec32 = k->spec32;
    a.twd = k->ctx->twd;
    a.twf = k->ctx->twf;
    a.sigma_s = k->params.sigma_s > 0.0 ? k->params.sigma_s : 0.0;
    a.sigma_k = k->params.sigma_k > 0.0 ? k->params.sigma_k : 0.0;
    if (k->wave) {
        for (int m = 0; m < 4; ++m) {
            if (!k->use[m]) continue;
            double2* d = nullptr;
            float2* f = nullptr;
            get_table(k->ctx, k->wM[m], &d, &f);
            if (m == 0) a.wtwf = f;
            else a.wtw[m] = d;
            a.coef[m] = k->coef[m];
            if (k->group) {
                get_table(k->ctx, group_sub_points(k->wM[1], k->wM[2], k->wM[3], k->wM[0], m), &d, &f);
                a.gsub[m] = (m == 0) ? (const void*)f : (const void*)d;
            }
        }
        a.coef32 = k->coef32;
    }
    return a;
}

// The multi-pass FFT core: its per-item scratch (grown here to the signal's items; the
// allocation waits for the device), then its passes.
apx_status launch_big_kernel(apx_kernel k, const RunArgs& a, hipStream_t st) {
    if (a.many) return fail(APX_E_UNSUPPORTED, "the multi-pass FFT core runs one signal per launch");
    if (a.nitems > 65535) return fail(APX_E_UNSUPPORTED, "the multi-pass FFT core runs at most 65535 blocks");
    const int MW = 1 << k->big_logmw, F1 = 1 << (k->big_logmw / 2);
    const bool fp32 = k->params.mode == APX_FULL_FP32;
    const size_t pts = (size_t)a.nitems * MW * (fp32 ? sizeof(float2) : sizeof(double2));
    const size_t need = pts + (size_t)a.nitems * big_item_bytes();
    if (need > k->big_scr_bytes) {
        if (k->big_scr) HIPCHK(hipFree(k->big_scr));
        k->big_scr = nullptr;
        k->big_scr_bytes = 0;
        HIPCHK(hipMalloc(&k->big_scr, need));
        k->big_scr_bytes = need;
    }
    double2 *d1 = nullptr, *d2 = nullptr, *dm = nullptr, *dF = nullptr;
    float2 *f1 = nullptr, *f2 = nullptr, *fm = nullptr, *fF = nullptr;
    apx_status r = get_table(k->ctx, F1, &d1, &f1);
    if (r == APX_OK) r = get_table(k->ctx, MW / F1, &d2, &f2);
    if (r == APX_OK) r = get_table(k->ctx, MW, &dm, &fm);
    if (r == APX_OK) r = get_table(k->ctx, 2 * MW, &dF, &fF);
    if (r != APX_OK) return r;
    const int m = k->params.mode;
    const void* H = fp32 ? (const void*)k->spec32 : (const void*)k->spec[m];
    char* items = (char*)k->big_scr + pts;
    if (fp32)
        HIPCHK(launch_big(a, MD_FULL32, k->big_logmw, items, k->big_scr, f1, f2, fm, fF, H, st));
    else
        HIPCHK(launch_big(a, m, k->big_logmw, items, k->big_scr, d1, d2, dm, dF, H, st));
    return APX_OK;
}

apx_status launch_block_kernel(apx_kernel k, const RunArgs& a, hipStream_t st) {
    if (k->core == APX_CORE_FFT && k->big_logmw) return launch_big_kernel(k, a, st);
    if (k->core == APX_CORE_INT8) {
        HIPCHK(launch_i8(a, k->i8frag, k->S[k->params.mode] > 127, k->i8_splitk, k->i8_plane, k->i8_tm, st));
    } else if (k->core == APX_CORE_FFT && k->group) {
        HIPCHK(launch_fftg(a, k->wM[1], k->wM[2], k->wM[3], k->wM[0], st));
    } else if (k->core == APX_CORE_FFT && k->wave) {
        HIPCHK(launch_fftw(a, k->wM[1], k->wM[2], k->wM[3], k->wM[0], st));
    } else if (k->core == APX_CORE_FFT && k->fft1_logmw > 0) {
        HIPCHK(launch_fft1(a, k->params.mode, k->fft1_logmw, st));
    } else if (k->core == APX_CORE_FFT) {
        HIPCHK(launch_fft(a, k->logF, st));
    } else {
        HIPCHK(launch_td(a, k->td_lds, k->td_tile, st));
    }
    return APX_OK;
}

// The one-wave FFT, time-domain and integer cores read their windows as sample pairs: s_in must
// be 8-byte aligned (blocks start at even sample offsets).  The batched kernel tests alignment
// itself, so references may start anywhere.
static bool aligned8(const float* p) { return (reinterpret_cast<uintptr_t>(p) & 7) == 0; }

apx_status run_impl(apx_ctx ctx, apx_kernel k, const float* s, int64_t L, float* out, double* fields,
                    apx_block_info* info, hipStream_t st) {
    if (!ctx || !k) return fail(APX_E_INVALID, "null context or kernel");
    if (!s || !out) return fail(APX_E_INVALID, "null input or output pointer");
    if (!aligned8(s)) return fail(APX_E_INVALID, "s_in must be 8-byte aligned");
    if (L < k->N) return fail(APX_E_INVALID, "input length L = %lld shorter than the kernel N = %d", (long long)L, k->N);
    int64_t P = 0;
    apx_status r = geometry(L, k->N, k->W_block, nullptr, nullptr, &P);
    if (r != APX_OK) return r;
    if (P > (int64_t)0x7fffffff - 1) return fail(APX_E_UNSUPPORTED, "too many blocks");
    HIPCHK(hipSetDevice(ctx->device));
    RunArgs a = make_args(k, s, L, out, fields, info, P);
    return launch_block_kernel(k, a, st);
}

}  // namespace

extern "C" {

const char* apx_status_str(apx_status st) {
    switch (st) {
        case APX_OK: return "ok";
        case APX_E_INVALID: return "invalid argument";
        case APX_E_BOUND: return "companding range beyond the error-free packing bound";
        case APX_E_NOMEM: return "device allocation failed";
        case APX_E_DEVICE: return "HIP device error";
        case APX_E_UNSUPPORTED: return "unsupported";
    }
    return "unknown status";
}

const char* apx_last_error(void) { return g_err.c_str(); }

apx_status apx_create(int device, apx_ctx* out) {
    if (!out) return fail(APX_E_INVALID, "null output handle");
    *out = nullptr;
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(APX_E_INVALID, "device %d not present (%d devices)", device, n);
    HIPCHK(hipSetDevice(device));
    apx_ctx c = new (std::nothrow) apx_ctx_s;
    if (!c) return fail(APX_E_NOMEM, "host allocation failed");
    c->device = device;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, device) == hipSuccess && lds > 0)
        c->max_lds = lds;
    apx_status r = build_twiddles(c);
    if (r == APX_OK) {
        // the device address of this device's scratch copy, taken once with the device current
        hipError_t e = noalloc_scratch(&c->scratch, &c->scratch_bytes);
        if (e != hipSuccess) r = fail(APX_E_DEVICE, "scratch address: %s", hipGetErrorString(e));
    }
    if (r == APX_OK) apx::tune_load(c);  // this device's autotuning table from earlier processes
    if (r == APX_OK) {
        double2 w32[32], w24[24];
        fill_twiddles(32, w32);
        fill_twiddles(24, w24);
        hipError_t e = upload_dft_constants(w32, w24);
        if (e != hipSuccess) r = fail(APX_E_DEVICE, "constant upload: %s", hipGetErrorString(e));
    }
    if (r != APX_OK) {
        apx_destroy(c);
        return r;
    }
    *out = c;
    return APX_OK;
}

apx_status apx_destroy(apx_ctx c) {
    if (!c) return APX_OK;
    (void)hipSetDevice(c->device);
    if (c->twd) (void)hipFree(c->twd);
    if (c->twf) (void)hipFree(c->twf);
    for (auto& kv : c->tables) {
        (void)hipFree(kv.second.first);
        (void)hipFree(kv.second.second);
    }
    delete c;
    return APX_OK;
}

apx_status apx_geometry(int64_t L, int32_t N, int32_t W_block, int32_t* N_odd, int32_t* W, int64_t* P) {
    return geometry(L, N, W_block, N_odd, W, P);
}

}  // extern "C"

namespace {

// Prepare kernel state into *k (fresh).  fft_words > 0 forces the FFT core with that packed word
// length for every mode (the batched path); 0 = the rules of apx_kernel_create.  On failure the
// device buffers of k are released (pool buffers belong to the pool).
apx_status init_kernel(apx_kernel k, apx_ctx ctx, const float* k_in, int32_t N, int32_t op, int32_t W_block,
                       const apx_params* params, void* stream, int32_t fft_words) {
    if (!ctx || !k_in || !params) return fail(APX_E_INVALID, "null argument");
    if (op != APX_CONV && op != APX_XCORR) return fail(APX_E_INVALID, "unknown op %d", op);
    int32_t N_odd = 0, W = 0;
    apx_status r = geometry(1, N, W_block, &N_odd, &W, nullptr);
    if (r != APX_OK) return r;
    const apx_params p = *params;
    if (p.mode < APX_FULL_FP32 || p.mode > APX_FULL_FP64) return fail(APX_E_INVALID, "unknown mode %d", p.mode);
    if (p.core < APX_CORE_AUTO || p.core > APX_CORE_INT8) return fail(APX_E_INVALID, "unknown core %d", p.core);
    if (p.Sq < 0 || p.Kq < 0) return fail(APX_E_INVALID, "negative companding range");
    if (p.mode == APX_AUTO_SNR && !isfinite(p.snr_min_db)) return fail(APX_E_INVALID, "snr_min_db must be finite");

    k->ctx = ctx;
    k->N = N;
    k->N_odd = N_odd;
    k->op = op;
    k->W_block = W_block;
    k->W = W;
    k->params = p;
    // companding ranges (eq. 3) per packed mode
    for (int m = MD_SYM; m <= MD_ASYM3; ++m) {
        const int64_t qmax = isqrt64(bound_of(m) / N_odd);
        int64_t S = qmax, K = qmax;
        if (p.mode == m) {
            if (p.Sq) S = p.Sq;
            if (p.Kq) K = p.Kq;
        }
        // S, K < 2^31, so S K fits; N_odd S K may not (caller-given ranges)
        int64_t Rm = 0;
        if (__builtin_mul_overflow(S * K, (int64_t)N_odd, &Rm))
            return fail(APX_E_BOUND, "R_max = N S_q K_q overflows 64 bits (N = %d, S_q = %lld, K_q = %lld)", N_odd,
                        (long long)S, (long long)K);
        k->S[m] = (int32_t)S;
        k->K[m] = (int32_t)K;
        k->R[m] = Rm;
        k->T[m] = (m == MD_SYM) ? 0 : (W + (m == MD_ASYM2 ? 2 : 3) - 1) / (m == MD_ASYM2 ? 2 : 3);
    }
    if (p.mode >= APX_SYM && p.mode <= APX_ASYM3) {
        const int m = p.mode;
        if (k->S[m] < 1 || k->K[m] < 1) {
            return fail(APX_E_BOUND, "no companding range S_q = K_q >= 1 fits the bound for N = %d", N_odd);
        }
        // the integer core carries no packing: exact for any S_q, K_q its digits hold
        if (k->R[m] > bound_of(m) && !p.allow_unsafe && p.core != APX_CORE_INT8) {
            int64_t Rm = k->R[m];
            return fail(APX_E_BOUND, "R_max = N S_q K_q = %lld exceeds the bound %lld (Table 1)", (long long)Rm,
                        (long long)bound_of(m));
        }
        if (k->R[m] > ((int64_t)1 << (p.core == APX_CORE_INT8 ? 52 : 40))) {
            return fail(APX_E_UNSUPPORTED, "R_max too large");
        }
        k->use[m] = true;
    } else if (p.mode == APX_AUTO_SNR) {
        k->cand_mask = 0;
        if (k->S[MD_SYM] >= 1) k->cand_mask |= 1 << MD_SYM;
        if (k->S[MD_ASYM2] >= 1) k->cand_mask |= 1 << MD_ASYM2;
        k->use[MD_SYM] = k->S[MD_SYM] >= 1;
        k->use[MD_ASYM2] = k->S[MD_ASYM2] >= 1;
        k->use[0] = true;
    } else {
        k->use[0] = true;
    }
    k->calib_db = 0.0;
    // core choice
    int core = p.core;
    if (p.mode == APX_FULL_FP64) {
        if (core == APX_CORE_FFT) {
            return fail(APX_E_UNSUPPORTED, "FP64 full precision runs on the time-domain core only");
        }
        core = APX_CORE_TIME;
    }
    if (core == APX_CORE_AUTO) {
        // short kernels: the integer matrix cores for a fixed packed mode (the same companded
        // integers as the packed time-domain core, measured several times faster), else the
        // time-domain core; long kernels: the FFT core
        core = (N_odd <= 129) ? APX_CORE_TIME : APX_CORE_FFT;
        if (core == APX_CORE_TIME && p.mode >= APX_SYM && p.mode <= APX_ASYM3 && fft_words == 0 &&
            k->S[p.mode] <= 16319 && k->K[p.mode] <= 16319 &&
            i8_lds_bytes(i8_plane_len(N_odd, W), W_block) <= (size_t)ctx->max_lds)
            core = APX_CORE_INT8;
    }
    if (fft_words > 0) core = APX_CORE_FFT;
    k->core = core;
    if (core == APX_CORE_INT8) {
        if (p.mode < APX_SYM || p.mode > APX_ASYM3)
            return fail(APX_E_UNSUPPORTED, "the integer core runs a fixed packed mode's companding only");
        const int m = p.mode;
        if (k->S[m] > 16319 || k->K[m] > 16319)
            return fail(APX_E_UNSUPPORTED, "the integer core takes S_q, K_q <= 16319 (two int8 digits)");
        if ((int64_t)N_odd + 31 >= (1 << 17)) return fail(APX_E_UNSUPPORTED, "N too large for int32 digit sums");
        k->i8_plane = i8_plane_len(N_odd, W);
        // tiles per pass: as many as the blocks have, at most 3.  Fewer passes win even where the
        // last pass repeats tiles (four tiles on the FFT-block shape: 3 + 1 ran 24.3 us, 2 + 2
        // ran 25.8 us), since every pass reloads the tap fragments.
        k->i8_tm = std::min(3, std::max(1, i8_tiles(N_odd, W)));
        k->i8_splitk = k->K[m] > 127;
        const size_t lds = i8_lds_bytes(k->i8_plane, W_block);
        if (lds > (size_t)ctx->max_lds)
            return fail(APX_E_UNSUPPORTED, "integer core block needs %zu bytes of LDS (> %d)", lds, ctx->max_lds);
    }
    if (fft_words > 0) {
        if (p.mode == APX_AUTO_SNR || p.mode == APX_FULL_FP64)
            return fail(APX_E_UNSUPPORTED, "a forced FFT length needs a fixed mode");
        k->logF = ceil_log2(fft_words);
        if ((1 << k->logF) != fft_words || k->logF > LOGF_MAX_TABLE || k->logF < 8)
            return fail(APX_E_UNSUPPORTED, "FFT length %d", fft_words);
        for (int m = 0; m < 4; ++m) k->Fw[m] = fft_words;
    } else if (core == APX_CORE_FFT) {
        k->logF = std::max(ceil_log2(W_block), fft_min_logF());
        // a fixed packed mode transforms only its own words: W_block / 2 (symmetric) or
        // T + N - 1 (asymmetric), at the shortest power of two that holds them
        const bool fixed_packed = p.mode >= APX_SYM && p.mode <= APX_ASYM3;
        int own_logw = 0;
        // the multi-pass core: asked for (fft_variant 4), or a fixed mode / FP32 whose words
        // exceed the one-workgroup transforms
        const int big_words = fixed_packed ? ((p.mode == MD_SYM) ? W_block / 2 : k->T[p.mode] + N_odd - 1)
                                           : (p.mode == APX_FULL_FP32 ? W_block : 0);
        if (big_words > 0 && (p.fft_variant == 4 || ceil_log2(big_words) > fft_max_logF())) {
            const int logmw = std::max(ceil_log2(big_words), 1) - 1;
            const bool fp32 = p.mode == APX_FULL_FP32;
            if (!big_supported(logmw, fp32))
                return fail(APX_E_UNSUPPORTED, "FFT core: %d words per block (multi-pass transforms of %d to %d words)",
                            big_words, 2 << BIG_LOGMW_MIN, 2 << (fp32 ? BIG_LOGMW_MAX_FP32 : BIG_LOGMW_MAX));
            k->big_logmw = logmw;
            for (int m = 0; m < 4; ++m) k->Fw[m] = 2 << logmw;
        } else if (p.fft_variant == 4) {
            return fail(APX_E_UNSUPPORTED, "the multi-pass FFT core runs a fixed packed mode or FP32");
        } else if (fixed_packed) {
            const int words = (p.mode == MD_SYM) ? W_block / 2 : k->T[p.mode] + N_odd - 1;
            own_logw = std::max(ceil_log2(words), fft_min_logF() - 1);
            if (own_logw > fft_max_logF() || !fft1_supported(p.mode, own_logw - 1))
                return fail(APX_E_UNSUPPORTED, "FFT core: %d packed words per block exceed %d", words,
                            1 << fft_max_logF());
        } else if (k->logF > fft_max_logF()) {
            return fail(APX_E_UNSUPPORTED, "FFT core supports W_block <= %d", 1 << fft_max_logF());
        }
        if (k->logF <= fft_max_logF() && !k->big_logmw) {
            const int F = 1 << k->logF;
            k->Fw[0] = F;
            k->Fw[MD_SYM] = F / 2;
            k->Fw[MD_ASYM2] = F;
            k->Fw[MD_ASYM3] = F;
        }
        if (fixed_packed && !k->big_logmw) {
            k->fft1_logmw = own_logw - 1;
            k->Fw[p.mode] = 1 << own_logw;
        }
        // wave-per-block core: complex points per mode, if an instantiated size set covers them
        int need[4] = {W_block, W_block / 2, k->T[MD_ASYM2] + N_odd - 1, k->T[MD_ASYM3] + N_odd - 1};
        int wm[4];
        bool ok = true;
        for (int m = 0; m < 4; ++m) {
            wm[m] = wave_m_for(need[m]);
            if (k->use[m] && wm[m] == 0) ok = false;
        }
        if (wm[0] == 0) ok = false;  // the FP32 size also sizes the window in LDS
        if (k->big_logmw) ok = false;
        if (ok && p.fft_variant != 1) {
            // modes that are not used may take any size, except the FP32 slot (W_block <= 2 M):
            // look for a compiled set that matches (the launch needs a complete set).  Automatic
            // choice: the group core first (C2: asymmetric M=2 25 vs 30 us, per-block choice at
            // 40 dB 27 vs 32 us, FP32 23.4 vs 24.3 us), then the one-wave core
            const int cand[4] = {512, 1024, 1536, 2048};
            int order[2] = {0, 1};  // 0 = group, 1 = one wave
            int npass = 2;
            if (p.fft_variant == 2 || p.fft_variant == 3) {
                order[0] = p.fft_variant == 3 ? 0 : 1;
                npass = 1;
            }
            for (int oi = 0; oi < npass && !k->wave; ++oi) {
                const int pass = order[oi];
                for (int c = 0; c < 256 && !k->wave; ++c) {
                    const int t4[4] = {cand[c & 3], cand[(c >> 2) & 3], cand[(c >> 4) & 3], cand[(c >> 6) & 3]};
                    bool match = t4[0] == wm[0];
                    for (int m = 1; m < 4; ++m)
                        if (k->use[m] && t4[m] != wm[m]) match = false;
                    const bool sup = pass == 0 ? group_supported(t4[1], t4[2], t4[3], t4[0])
                                               : wave_supported(t4[1], t4[2], t4[3], t4[0]);
                    if (match && sup) {
                        for (int m = 0; m < 4; ++m) k->wM[m] = t4[m];
                        k->wave = true;
                        k->group = pass == 0;
                    }
                }
            }
        }
        if ((p.fft_variant == 2 || p.fft_variant == 3) && !k->wave) {
            return fail(APX_E_UNSUPPORTED, "no compiled %s size set covers W_block = %d, N = %d",
                        p.fft_variant == 2 ? "one-wave" : "group", W_block, N);
        }
        if (p.fft_variant == 3 && !k->group) {
            return fail(APX_E_UNSUPPORTED, "no compiled group size set covers W_block = %d, N = %d", W_block, N);
        }
    } else if (core == APX_CORE_INT8) {
        // sized above
    } else {
        k->td_lds = td_lds_bytes(p.mode, N_odd, W_block, k->T[MD_ASYM2], k->T[MD_ASYM3]);
        if (k->td_lds > (size_t)ctx->max_lds) {
            return fail(APX_E_UNSUPPORTED, "time-domain block needs %zu bytes of LDS (> %d); use the FFT core",
                        k->td_lds, ctx->max_lds);
        }
        // outputs per thread: 4 while one pass of the workgroup's threads covers the longest
        // range the block convolves (outputs, or packed words), else 8
        int range = W_block;  // FP32 / FP64 outputs
        if (p.mode == MD_SYM) range = W_block / 2 + 1;
        if (p.mode == MD_ASYM2 || p.mode == MD_ASYM3) range = k->T[p.mode] + N_odd;
        k->td_tile = range <= 4 * NT ? 4 : 8;
    }
    // device state
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return fail(APX_E_DEVICE, "hipSetDevice failed");
    k->kf_pad = pad8(N_odd);
    const int nsym = (N_odd + 1) / 2;
    k->kq_len[MD_SYM] = nsym;
    k->kq_pad[MD_SYM] = pad8(nsym);
    k->kq_len[MD_ASYM2] = k->kq_len[MD_ASYM3] = N_odd;
    k->kq_pad[MD_ASYM2] = k->kq_pad[MD_ASYM3] = pad8(N_odd);
    r = dalloc(k, &k->ks, 1);
    if (r == APX_OK) r = dalloc(k, &k->kf, k->kf_pad + 8);
    if (r == APX_OK) r = dalloc(k, &k->kd, k->kf_pad + 8);
    if (r == APX_OK && k->use[MD_SYM]) r = dalloc(k, &k->kq[MD_SYM], k->kq_pad[MD_SYM] + 8);
    if (r == APX_OK && k->use[MD_ASYM2]) r = dalloc(k, &k->kq[MD_ASYM2], k->kq_pad[MD_ASYM2] + 8);
    if (r == APX_OK && k->use[MD_ASYM3]) r = dalloc(k, &k->kq[MD_ASYM3], k->kq_pad[MD_ASYM3] + 8);
    if (r == APX_OK && core == APX_CORE_FFT && !k->wave) {
        for (int m = MD_SYM; m <= MD_ASYM3 && r == APX_OK; ++m)
            if (k->use[m]) r = dalloc(k, &k->spec[m], k->Fw[m] / 2 + 1);
        if (r == APX_OK && k->use[0]) r = dalloc(k, &k->spec32, k->Fw[0] / 2 + 1);
    }
    if (r == APX_OK && core == APX_CORE_FFT && k->wave) {
        for (int m = MD_SYM; m <= MD_ASYM3 && r == APX_OK; ++m)
            if (k->use[m]) r = dalloc(k, &k->coef[m], 2 * (size_t)k->wM[m]);
        if (r == APX_OK && k->use[0]) r = dalloc(k, &k->coef32, 2 * (size_t)k->wM[0]);
        auto table = [&](int F) -> apx_status {
            if (!k->plan_only) return get_table(ctx, F, nullptr, nullptr);
            if (!ctx->tables.count(F) && std::find(k->plan_tables.begin(), k->plan_tables.end(), F) == k->plan_tables.end())
                k->plan_tables.push_back(F);
            return APX_OK;
        };
        for (int m = 0; m < 4 && r == APX_OK; ++m) {
            if (!k->use[m]) continue;
            r = table(k->wM[m]);
            if (r == APX_OK) r = table(2 * k->wM[m]);
            if (r == APX_OK && k->group) r = table(group_sub_points(k->wM[1], k->wM[2], k->wM[3], k->wM[0], m));
        }
    }
    if (r == APX_OK && core == APX_CORE_FFT && k->big_logmw) {
        // twiddles of the two transform lengths, of the inter-pass step and of the real split
        const int MW = 1 << k->big_logmw, F1 = 1 << (k->big_logmw / 2);
        for (int F : {F1, MW / F1, MW, 2 * MW}) {
            if (r != APX_OK) break;
            if (!k->plan_only) r = get_table(ctx, F, nullptr, nullptr);
            else if (!ctx->tables.count(F) &&
                     std::find(k->plan_tables.begin(), k->plan_tables.end(), F) == k->plan_tables.end())
                k->plan_tables.push_back(F);
        }
    }
    if (r == APX_OK && core == APX_CORE_INT8) r = dalloc(k, &k->i8frag, (size_t)2 * i8_kpad(N_odd) * 64 * 4);
    if (r != APX_OK) {
        free_kernel(k);
        return r;
    }
    if (k->plan_only) return APX_OK;
    hipError_t e = launch_prepare_kernel(k_in, N, N_odd, op == APX_XCORR, k->ks, k->kf, k->kd, k->kf_pad + 8,
                                         k->kq[MD_SYM], k->kq[MD_ASYM2], k->kq[MD_ASYM3], k->K, k->R,
                                         k->kq_pad[MD_SYM] + 8, k->kq_pad[MD_ASYM2] + 8, st);
    if (e == hipSuccess && core == APX_CORE_FFT && k->big_logmw) {
        // the multi-pass core's spectrum of its one mode, by a direct DFT in FP64
        double2* tF = nullptr;
        get_table(ctx, k->Fw[0], &tF, nullptr);
        for (int m = MD_SYM; m <= MD_ASYM3 && e == hipSuccess; ++m)
            if (k->use[m]) e = launch_big_spectrum(k->kq[m], k->kq_len[m], k->Fw[m], tF, k->spec[m], false, st);
        if (e == hipSuccess && k->use[0]) e = launch_big_spectrum(k->kd, N_odd, k->Fw[0], tF, k->spec32, true, st);
    } else if (e == hipSuccess && core == APX_CORE_FFT && !k->wave) {
        for (int m = MD_SYM; m <= MD_ASYM3 && e == hipSuccess; ++m)
            if (k->use[m]) e = launch_spectrum(k->kq[m], k->kq_len[m], k->Fw[m], ctx->twd, k->spec[m], st);
        if (e == hipSuccess && k->use[0]) e = launch_spectrum32(k->kf, N_odd, k->Fw[0], ctx->twf, k->spec32, st);
    }
    if (e == hipSuccess && core == APX_CORE_FFT && k->wave) {
        for (int m = MD_SYM; m <= MD_ASYM3 && e == hipSuccess; ++m) {
            if (!k->use[m]) continue;
            double2* tF = nullptr;
            get_table(ctx, 2 * k->wM[m], &tF, nullptr);
            e = launch_coef(k->kq[m], k->kq_len[m], k->wM[m], tF, k->coef[m], st);
        }
        if (e == hipSuccess && k->use[0]) {
            double2* tF = nullptr;
            get_table(ctx, 2 * k->wM[0], &tF, nullptr);
            e = launch_coef32(k->kd, N_odd, k->wM[0], tF, k->coef32, st);
        }
    }
    if (e == hipSuccess && core == APX_CORE_INT8) {
        e = launch_i8_frag(k->kf, k->ks, p.mode, N_odd, k->i8_splitk, k->i8frag, st);
        const size_t lds = i8_lds_bytes(k->i8_plane, W_block);
        if (e == hipSuccess && lds > 65536) e = i8_set_lds((int)lds);
    }
    if (e == hipSuccess && core == APX_CORE_FFT && !k->wave && !k->big_logmw && fft_words == 0)
        e = k->fft1_logmw > 0 ? fft1_set_lds(p.mode, k->fft1_logmw) : fft_set_lds(k->logF);
    if (e != hipSuccess) {
        free_kernel(k);
        return fail(APX_E_DEVICE, "kernel preparation launch: %s", hipGetErrorString(e));
    }
    return APX_OK;
}

}  // namespace

extern "C" {

apx_status apx_kernel_create(apx_ctx ctx, const float* k_in, int32_t N, int32_t op, int32_t W_block,
                             const apx_params* params, void* stream, apx_kernel* out) {
    if (!out) return fail(APX_E_INVALID, "null output handle");
    *out = nullptr;
    if (!ctx || !params) return fail(APX_E_INVALID, "null argument");
    if (W_block < 0) return fail(APX_E_INVALID, "W_block = %d", W_block);
    apx_params p = *params;
    int32_t tile = 0;
    apx::resolve_tuned(ctx, N, op, &W_block, &p, &tile);  // W_block 0 and automatic cores take the tuned choice
    apx_kernel k = new (std::nothrow) apx_kernel_s;
    if (!k) return fail(APX_E_NOMEM, "host allocation failed");
    apx_status r = init_kernel(k, ctx, k_in, N, op, W_block, &p, stream, 0);
    if (r != APX_OK) {
        delete k;
        return r;
    }
    if (tile > 0 && k->core == APX_CORE_INT8) k->i8_tm = tile;
    if ((tile == 4 || tile == 8) && k->core == APX_CORE_TIME) k->td_tile = tile;
    *out = k;
    return APX_OK;
}

apx_status apx_kernel_destroy(apx_kernel k) {
    if (!k) return APX_OK;
    (void)hipSetDevice(k->ctx->device);
    free_kernel(k);
    delete k;
    return APX_OK;
}

apx_status apx_run(apx_ctx ctx, apx_kernel k, const float* s, int64_t L, float* out, apx_block_info* info,
                   void* stream) {
    return run_impl(ctx, k, s, L, out, nullptr, info, (hipStream_t)stream);
}

apx_status apx_debug_fields(apx_ctx ctx, apx_kernel k, const float* s, int64_t L, double* fields, void* stream) {
    if (!ctx || !k || !s || !fields) return fail(APX_E_INVALID, "null argument");
    if (L < k->N) return fail(APX_E_INVALID, "input shorter than the kernel");
    if (k->params.mode < APX_SYM || k->params.mode > APX_ASYM3)
        return fail(APX_E_INVALID, "integer fields exist for fixed packed modes only");
    float* tmp = nullptr;
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipMalloc((void**)&tmp, (size_t)(L + k->N - 1) * sizeof(float)));
    apx_status r = run_impl(ctx, k, s, L, tmp, fields, nullptr, (hipStream_t)stream);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    (void)hipFree(tmp);
    if (r != APX_OK) return r;
    if (e != hipSuccess) return fail(APX_E_DEVICE, "debug fields: %s", hipGetErrorString(e));
    return APX_OK;
}

apx_status apx_calibrate(apx_ctx ctx, apx_kernel k, const float* s, int64_t L, int32_t block, int32_t Q, void* stream,
                         double* offset_db) {
    if (!ctx || !k || !s) return fail(APX_E_INVALID, "null argument");
    if (!aligned8(s)) return fail(APX_E_INVALID, "s_in must be 8-byte aligned");
    if (Q < 1) return fail(APX_E_INVALID, "Q must be >= 1");
    int64_t P = 0;
    apx_status r = geometry(L, k->N, k->W_block, nullptr, nullptr, &P);
    if (r != APX_OK) return r;
    if (L < k->N) return fail(APX_E_INVALID, "input shorter than the kernel");
    if (block < 0 || block >= P) return fail(APX_E_INVALID, "block %d outside [0, %lld)", block, (long long)P);
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    const int nparts = 64;
    double* part = nullptr;
    HIPCHK(hipMalloc((void**)&part, (2 * nparts + 2) * sizeof(double)));
    RunArgs a = make_args(k, s, L, nullptr, nullptr, nullptr, P);
    std::vector<double> h(2 * nparts + 2);
    KState ks;
    hipError_t e = launch_calib(a, block, Q, part, nparts, st);
    if (e == hipSuccess) e = hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipMemcpyAsync(&ks, k->ks, sizeof ks, hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(part);
    if (e != hipSuccess) return fail(APX_E_DEVICE, "calibration: %s", hipGetErrorString(e));
    double pr = 0.0, pe = 0.0;
    for (int i = 0; i < nparts; ++i) {
        pr += h[2 * i];
        pe += h[2 * i + 1];
    }
    const double smax = h[2 * nparts], rms = h[2 * nparts + 1];  // rms: the source sigma when one is set
    const double krms = ks.krms > 0.0 && k->params.sigma_k > 0.0 ? k->params.sigma_k : ks.krms;
    if (pe <= 0.0 || pr <= 0.0 || rms <= 0.0 || krms <= 0.0)
        return fail(APX_E_INVALID, "calibration block has no quantization error or no signal");
    const double measured = 10.0 * log10(pr / pe);
    const double r12 = sqrt(12.0);
    const double svs = smax / (Q * r12), svk = ks.kmax / (Q * r12);
    const double D = (rms * svk) * (rms * svk) + (krms * svs) * (krms * svs) + (svk * svs) * (svk * svs);
    const double model = 10.0 * log10((rms * krms) * (rms * krms) / D);
    k->calib_db = measured - model;
    if (offset_db) *offset_db = k->calib_db;
    return APX_OK;
}

size_t apx_workspace_bytes(void) { return 2048; }

apx_status apx_fit_marginal(apx_ctx ctx, const float* x, int64_t n, int32_t model, double* out, void* stream) {
    if (!ctx || !x || !out) return fail(APX_E_INVALID, "null argument");
    if (n < 1) return fail(APX_E_INVALID, "n = %lld samples", (long long)n);
    if (model != APX_MARGINAL_LAPLACE && model != APX_MARGINAL_WEIBULL)
        return fail(APX_E_INVALID, "unknown marginal model %d", model);
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    double* d = nullptr;
    HIPCHK(hipMalloc((void**)&d, 4 * sizeof(double)));
    hipError_t e = launch_fit_marginal(x, n, model, d, st);
    if (e == hipSuccess) e = hipMemcpyAsync(out, d, 4 * sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(d);
    if (e != hipSuccess) return fail(APX_E_DEVICE, "marginal fit: %s", hipGetErrorString(e));
    if (model == APX_MARGINAL_WEIBULL && out[3] < 2.0)
        return fail(APX_E_INVALID, "a Weibull fit needs at least 2 positive samples (%g)", out[3]);
    return APX_OK;
}

}  // extern "C"

namespace apx {

apx_status set_error(apx_status st, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return st;
}

apx_status run_args(apx_kernel k, const float* s, int64_t L, float* out, apx_block_info* info, RunArgs* a) {
    if (!k || !s || !out || !a) return fail(APX_E_INVALID, "null argument");
    if (!aligned8(s)) return fail(APX_E_INVALID, "s_in must be 8-byte aligned");
    if (L < k->N) return fail(APX_E_INVALID, "input length L = %lld shorter than the kernel N = %d", (long long)L, k->N);
    int64_t P = 0;
    apx_status r = geometry(L, k->N, k->W_block, nullptr, nullptr, &P);
    if (r != APX_OK) return r;
    *a = make_args(k, s, L, out, nullptr, info, P);
    return APX_OK;
}

// Workspace layout: 64 per-workgroup partial pairs, the block's ||s||_inf and sigma, the offset.
apx_status calib_on_device(apx_kernel k, const RunArgs& a, int32_t block, void* workspace, const double** off,
                           hipStream_t st) {
    constexpr int nparts = 64, Q = 8;
    if (block < 0 || block >= a.P) return fail(APX_E_INVALID, "calibration block %d outside [0, %lld)", block, (long long)a.P);
    static_assert((2 * nparts + 4) * sizeof(double) <= 2048, "calibration workspace");
    double* part = (double*)workspace;
    double* o = part + 2 * nparts + 2;  // offset, then the threshold ratio for a.snr_min_db
    HIPCHK(launch_calib(a, block, Q, part, nparts, st));
    HIPCHK(launch_calib_finish(part, nparts, k->ks, Q, o, k->params.sigma_k > 0.0 ? k->params.sigma_k : 0.0,
                               a.snr_min_db, st));
    *off = o;
    return APX_OK;
}

apx_status launch_many(apx_kernel k, const RunArgs& first, const RunArgs* args, const int32_t* item_sig, int64_t nitems,
                       hipStream_t st) {
    if (nitems < 1 || nitems > (int64_t)0x7fffffff) return fail(APX_E_UNSUPPORTED, "%lld work items", (long long)nitems);
    RunArgs a = first;
    a.many = args;
    a.many_sig = item_sig;
    a.nitems = nitems;
    a.item0 = 0;
    return launch_block_kernel(k, a, st);
}

apx_status kernel_plan_bytes(apx_ctx ctx, int32_t N, int32_t op, int32_t W_block, const apx_params* p, size_t* bytes) {
    if (!bytes) return fail(APX_E_INVALID, "null argument");
    apx_kernel_s tmp;
    tmp.plan_only = true;
    static const float dummy = 0.0f;  // never read: a plan reads no taps
    apx_params pp = *p;
    resolve_tuned(ctx, N, op, &W_block, &pp);
    apx_status r = init_kernel(&tmp, ctx, &dummy, N, op, W_block, &pp, nullptr, 0);
    if (r != APX_OK) return r;
    size_t tb = 0;
    for (int F : tmp.plan_tables) tb += (size_t)(F + pass_table_len(F)) * (sizeof(double2) + sizeof(float2));
    *bytes = tmp.dev_bytes + tb;
    return APX_OK;
}

}  // namespace apx

extern "C" {

apx_status apx_run_auto(apx_ctx ctx, apx_kernel k, const float* s, int64_t L, float* out, apx_block_info* info,
                        double snr_min_db, int32_t calib_block, void* workspace, void* stream) {
    if (!ctx || !k || !s || !out || !workspace) return fail(APX_E_INVALID, "null argument");
    if (!aligned8(s)) return fail(APX_E_INVALID, "s_in must be 8-byte aligned");
    if (k->params.mode != APX_AUTO_SNR) return fail(APX_E_INVALID, "apx_run_auto needs an APX_AUTO_SNR kernel");
    if (!isfinite(snr_min_db)) return fail(APX_E_INVALID, "snr_min_db must be finite");
    if (L < k->N) return fail(APX_E_INVALID, "input length L = %lld shorter than the kernel N = %d", (long long)L, k->N);
    int64_t P = 0;
    apx_status r = geometry(L, k->N, k->W_block, nullptr, nullptr, &P);
    if (r != APX_OK) return r;
    if (calib_block < 0 || calib_block >= P)
        return fail(APX_E_INVALID, "calibration block %d outside [0, %lld)", calib_block, (long long)P);
    hipStream_t st = (hipStream_t)stream;
    HIPCHK(hipSetDevice(ctx->device));
    RunArgs a = make_args(k, s, L, out, nullptr, info, P);
    a.snr_min_db = snr_min_db;
    const double* off = nullptr;
    r = calib_on_device(k, a, calib_block, workspace, &off, st);
    if (r != APX_OK) return r;
    a.calib_dev = off;
    return launch_block_kernel(k, a, st);
}

apx_status apx_run_auto_noalloc(apx_ctx ctx, apx_kernel k, const float* s, int64_t L, float* out, apx_block_info* info,
                                double snr_min_db, int32_t calib_block, void* stream) {
    if (!ctx) return fail(APX_E_INVALID, "null context");
    if (!ctx->scratch) return fail(APX_E_DEVICE, "no scratch address for device %d", ctx->device);
    if (apx_workspace_bytes() > ctx->scratch_bytes)
        return fail(APX_E_UNSUPPORTED, "the calibration needs %zu bytes, the scratch holds %zu", apx_workspace_bytes(),
                    ctx->scratch_bytes);
    return apx_run_auto(ctx, k, s, L, out, info, snr_min_db, calib_block, ctx->scratch, stream);
}

apx_status apx_kernel_describe(apx_kernel k, char* buf, int32_t size) {
    if (!k || !buf || size < 1) return fail(APX_E_INVALID, "null argument");
    char tmp[512];
    int n;
    if (k->core == APX_CORE_TIME) {
        n = snprintf(tmp, sizeof tmp, "core=time kernel=k_td lds=%zu outputs_per_thread=%d", k->td_lds, k->td_tile);
    } else if (k->core == APX_CORE_INT8) {
        n = snprintf(tmp, sizeof tmp, "core=int8 kernel=k_i8 ksteps=%d lds=%zu split_k=%d tiles_per_pass=%d",
                     i8_ksteps(k->N_odd), i8_lds_bytes(k->i8_plane, k->W_block), k->i8_splitk, k->i8_tm);
    } else if (k->wave) {
        n = snprintf(tmp, sizeof tmp, "core=fft kernel=%s<%d,%d,%d,%d> words(fp32,sym,asym2,asym3)=%d,%d,%d,%d",
                     k->group ? "k_fftg" : "k_fftw", k->wM[1], k->wM[2], k->wM[3], k->wM[0], 2 * k->wM[0],
                     2 * k->wM[1], 2 * k->wM[2], 2 * k->wM[3]);
    } else if (k->big_logmw > 0) {
        n = snprintf(tmp, sizeof tmp, "core=fft kernel=k_big<mode %d, %d x %d points> words=%d", k->params.mode,
                     1 << (k->big_logmw / 2), 1 << (k->big_logmw - k->big_logmw / 2), 2 << k->big_logmw);
    } else if (k->fft1_logmw > 0) {
        n = snprintf(tmp, sizeof tmp, "core=fft kernel=k_fft1<mode %d, %d points> words=%d", k->params.mode,
                     1 << k->fft1_logmw, k->Fw[k->params.mode]);
    } else {
        n = snprintf(tmp, sizeof tmp, "core=fft kernel=k_fft<%d> words(fp32,sym,asym2,asym3)=%d,%d,%d,%d", k->logF,
                     k->Fw[0], k->Fw[1], k->Fw[2], k->Fw[3]);
    }
    snprintf(tmp + n, sizeof tmp - n, " N=%d W_block=%d W=%d SqKq(sym,asym2,asym3)=%d,%d,%d", k->N_odd, k->W_block,
             k->W, k->S[1], k->S[2], k->S[3]);
    snprintf(buf, size, "%s", tmp);
    return APX_OK;
}

static apx_status oneshot(apx_ctx ctx, int op, const float* s, int64_t L, const float* kk, int32_t N, int32_t W_block,
                          const apx_params* params, float* out, apx_block_info* info, void* stream) {
    apx_kernel k = nullptr;
    apx_status r = apx_kernel_create(ctx, kk, N, op, W_block, params, stream, &k);
    if (r != APX_OK) return r;
    r = apx_run(ctx, k, s, L, out, info, stream);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    apx_kernel_destroy(k);
    if (r != APX_OK) return r;
    if (e != hipSuccess) return fail(APX_E_DEVICE, "%s", hipGetErrorString(e));
    return APX_OK;
}

apx_status apx_conv(apx_ctx ctx, const float* s, int64_t L, const float* k, int32_t N, int32_t W_block,
                    const apx_params* params, float* out, apx_block_info* info, void* stream) {
    return oneshot(ctx, APX_CONV, s, L, k, N, W_block, params, out, info, stream);
}

apx_status apx_xcorr(apx_ctx ctx, const float* s, int64_t L, const float* k, int32_t N, int32_t W_block,
                     const apx_params* params, float* out, apx_block_info* info, void* stream) {
    return oneshot(ctx, APX_XCORR, s, L, k, N, W_block, params, out, info, stream);
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// Many signals, one kernel: one launch over every (signal, block) item
// ------------------------------------------------------------------------------------------

struct apx_many_s {
    apx_ctx ctx = nullptr;
    apx_kernel kern = nullptr;
    int32_t n = 0;
    int64_t nitems = 0;
    RunArgs* args = nullptr;      // device, one per signal
    int32_t* item_sig = nullptr;  // device, the signal of each launch item
    RunArgs first;                // host copy of signal 0's arguments: the launch's own
};

namespace {

void many_free(apx_many m) {
    if (!m) return;
    if (m->args) (void)hipFree(m->args);
    if (m->item_sig) (void)hipFree(m->item_sig);
    delete m;
}

}  // namespace

extern "C" {

apx_status apx_many_create(apx_ctx ctx, apx_kernel k, int32_t n, const float* const* s, const int64_t* L,
                           float* const* r_out, apx_block_info* const* info, void* stream, apx_many* out) {
    if (!out) return fail(APX_E_INVALID, "null output handle");
    *out = nullptr;
    if (!ctx || !k || !s || !L || !r_out) return fail(APX_E_INVALID, "null argument");
    if (n < 1) return fail(APX_E_INVALID, "n = %d signals", n);
    if (k->ctx != ctx) return fail(APX_E_INVALID, "the kernel belongs to another context");
    if (k->big_logmw) return fail(APX_E_UNSUPPORTED, "the multi-pass FFT core runs one signal per launch");
    std::vector<RunArgs> ha((size_t)n);
    int64_t total = 0;
    for (int32_t i = 0; i < n; ++i) {
        if (!s[i] || !r_out[i]) return fail(APX_E_INVALID, "signal %d: null pointer", i);
        if (!aligned8(s[i])) return fail(APX_E_INVALID, "signal %d: s must be 8-byte aligned", i);
        if (L[i] < k->N)
            return fail(APX_E_INVALID, "signal %d: length %lld shorter than the kernel N = %d", i, (long long)L[i], k->N);
        int64_t P = 0;
        apx_status r = geometry(L[i], k->N, k->W_block, nullptr, nullptr, &P);
        if (r != APX_OK) return r;
        ha[i] = make_args(k, s[i], L[i], r_out[i], nullptr, info ? info[i] : nullptr, P);
        ha[i].item0 = total;
        total += ha[i].nitems;
        if (total > (int64_t)0x7fffffff) return fail(APX_E_UNSUPPORTED, "more than 2^31 - 1 work items");
    }
    std::vector<int32_t> hi((size_t)total);
    for (int32_t i = 0; i < n; ++i)
        for (int64_t j = ha[i].item0; j < ha[i].item0 + ha[i].nitems; ++j) hi[(size_t)j] = i;
    apx_many m = new (std::nothrow) apx_many_s;
    if (!m) return fail(APX_E_NOMEM, "host allocation failed");
    m->ctx = ctx;
    m->kern = k;
    m->n = n;
    m->nitems = total;
    m->first = ha[0];
    hipStream_t st = (hipStream_t)stream;
    hipError_t e = hipSetDevice(ctx->device);
    if (e == hipSuccess) e = hipMalloc((void**)&m->args, ha.size() * sizeof(RunArgs));
    if (e == hipSuccess) e = hipMalloc((void**)&m->item_sig, hi.size() * sizeof(int32_t));
    if (e == hipSuccess) e = hipMemcpyAsync(m->args, ha.data(), ha.size() * sizeof(RunArgs), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(m->item_sig, hi.data(), hi.size() * sizeof(int32_t), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        many_free(m);
        return fail(e == hipErrorOutOfMemory ? APX_E_NOMEM : APX_E_DEVICE, "signal table: %s", hipGetErrorString(e));
    }
    *out = m;
    return APX_OK;
}

apx_status apx_many_run(apx_ctx ctx, apx_many m, void* stream) {
    if (!ctx || !m) return fail(APX_E_INVALID, "null argument");
    if (ctx != m->ctx) return fail(APX_E_INVALID, "the handle belongs to another context");
    HIPCHK(hipSetDevice(ctx->device));
    RunArgs a = m->first;
    a.many = m->args;
    a.many_sig = m->item_sig;
    a.nitems = m->nitems;
    a.item0 = 0;
    return launch_block_kernel(m->kern, a, (hipStream_t)stream);
}

apx_status apx_many_describe(apx_many m, char* buf, int32_t size) {
    if (!m || !buf || size < 1) return fail(APX_E_INVALID, "null argument");
    char kd[512];
    apx_kernel_describe(m->kern, kd, sizeof kd);
    snprintf(buf, size, "signals=%d items=%lld launch: %s", m->n, (long long)m->nitems, kd);
    return APX_OK;
}

apx_status apx_many_destroy(apx_many m) {
    if (!m) return APX_OK;
    (void)hipSetDevice(m->ctx->device);
    many_free(m);
    return APX_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// Batched cross-correlation matching
// ------------------------------------------------------------------------------------------

struct apx_batch_s {
    apx_ctx ctx = nullptr;
    int32_t n = 0;
    int mode = 0;
    int logW = 0, chunk = 1, grid = 0, per_cu = 0;
    std::vector<apx_kernel_s> kerns;  // per pair; device buffers in `pool`
    char* pool = nullptr;
    RunArgs* d_args = nullptr;
    int2* d_items = nullptr;
    int32_t nitems = 0;
    unsigned int* d_counter = nullptr;
    unsigned long long* d_keys = nullptr;
    int32_t* d_N = nullptr;
    std::vector<int32_t> W_block;
    std::string tune_log;
};

namespace {

void batch_free(apx_batch b) {
    if (!b) return;
    (void)hipSetDevice(b->ctx->device);
    for (void* p : {(void*)b->pool, (void*)b->d_args, (void*)b->d_items, (void*)b->d_counter, (void*)b->d_keys,
                    (void*)b->d_N})
        if (p) (void)hipFree(p);
    delete b;
}

// Largest block for a pair at packed word length `words`: FP32 W_block = words; symmetric two
// samples per word; asymmetric T = W / M parts of T + N - 1 words (T rounded up).  0 if W would
// fall below 2 N (Section III opening).
int32_t batch_block(int mode, int32_t N, int32_t words) {
    const int32_t no = (N % 2) ? N : N + 1;
    int64_t W;
    if (mode == MD_FULL32) W = (int64_t)words - no - 1;
    else if (mode == MD_SYM) W = 2 * (int64_t)words - no - 1;
    else {
        const int M = mode == MD_ASYM2 ? 2 : 3;
        W = (int64_t)M * (words - no + 1);
        W -= W % 2;
    }
    if (W < 2 * (int64_t)no || W % 2) return 0;
    return (int32_t)(W + no + 1);
}

apx_status batch_build(apx_ctx ctx, int32_t n, const float* const* refs, const int64_t* L, const float* const* tmpl,
                       const int32_t* N, const apx_params* params, int32_t logW, hipStream_t st, apx_batch* out) {
    *out = nullptr;
    const int mode = params->mode;
    const int32_t words = 1 << logW;
    apx_batch b = new (std::nothrow) apx_batch_s;
    if (!b) return fail(APX_E_NOMEM, "host allocation failed");
    b->ctx = ctx;
    b->n = n;
    b->mode = mode;
    b->logW = logW;
    b->kerns.resize(n);
    b->W_block.resize(n);
    // pool: per pair KState, FP32 and FP64 taps, companded taps, spectrum, each 256-aligned
    size_t pool_bytes = 0;
    for (int i = 0; i < n; ++i) {
        b->W_block[i] = batch_block(mode, N[i], words);
        if (b->W_block[i] == 0) {
            batch_free(b);
            return fail(APX_E_UNSUPPORTED, "pair %d: N = %d too long for FFT length %d", i, N[i], words);
        }
        const size_t taps = (size_t)pad8(N[i] + 1) + 16;
        pool_bytes += 6 * 256 + sizeof(KState) + taps * (4 + 8 + 8) + ((size_t)words / 2 + 1) * 16;
    }
    apx_status r = APX_OK;
    HIPCHK(hipSetDevice(ctx->device));
    if (hipMalloc((void**)&b->pool, pool_bytes) != hipSuccess) {
        batch_free(b);
        return fail(APX_E_NOMEM, "pair pool of %zu bytes", pool_bytes);
    }
    size_t off = 0;
    std::vector<RunArgs> args(n);
    std::vector<int64_t> P(n);
    for (int i = 0; i < n && r == APX_OK; ++i) {
        apx_kernel k = &b->kerns[i];
        const size_t taps = (size_t)pad8(N[i] + 1) + 16;
        const size_t mine = 6 * 256 + sizeof(KState) + taps * (4 + 8 + 8) + ((size_t)words / 2 + 1) * 16;
        k->pool = b->pool + off;
        k->pool_cap = mine;
        off += mine;
        r = init_kernel(k, ctx, tmpl[i], N[i], APX_XCORR, b->W_block[i], params, st, words);
        if (r == APX_OK) r = geometry(L[i], N[i], b->W_block[i], nullptr, nullptr, &P[i]);
        if (r == APX_OK) args[i] = make_args(k, refs[i], L[i], nullptr, nullptr, nullptr, P[i]);
        if (r != APX_OK) r = fail(r, "pair %d: %s", i, g_err.c_str());
    }
    if (r != APX_OK) {
        batch_free(b);
        return r;
    }
    // work list: pairs in decreasing block count (longest first), blocks in order
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return P[x] > P[y]; });
    std::vector<int2> items;
    int64_t total = 0;
    for (int i = 0; i < n; ++i) total += P[i] + 1;
    if (total > 0x7fffffff / 2) {
        batch_free(b);
        return fail(APX_E_UNSUPPORTED, "%lld blocks in one batch", (long long)total);
    }
    items.reserve(total);
    for (int i : order)
        for (int64_t w = 0; w <= P[i]; ++w) items.push_back(make_int2(i, (int)w));
    b->nitems = (int32_t)items.size();
    hipError_t e = hipMalloc((void**)&b->d_args, sizeof(RunArgs) * n);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_items, sizeof(int2) * items.size());
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_counter, 256);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_keys, sizeof(unsigned long long) * n);
    if (e == hipSuccess) e = hipMalloc((void**)&b->d_N, sizeof(int32_t) * n);
    if (e != hipSuccess) {
        batch_free(b);
        return fail(APX_E_NOMEM, "batch tables: %s", hipGetErrorString(e));
    }
    e = hipMemcpyAsync(b->d_args, args.data(), sizeof(RunArgs) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
        e = hipMemcpyAsync(b->d_items, items.data(), sizeof(int2) * items.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipMemcpyAsync(b->d_N, N, sizeof(int32_t) * n, hipMemcpyHostToDevice, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);  // host staging vectors go out of scope
    if (e == hipSuccess) e = batch_occupancy(mode, logW, &b->per_cu);
    if (e != hipSuccess || b->per_cu < 1) {
        batch_free(b);
        return fail(APX_E_DEVICE, "batch setup: %s", hipGetErrorString(e));
    }
    int cus = 0;
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, ctx->device));
    b->grid = std::max(1, b->per_cu * cus);
    *out = b;
    return APX_OK;
}

BatchLaunch batch_args(apx_batch b, int64_t* lag, float* val, hipStream_t st) {
    BatchLaunch l{};
    l.mode = b->mode;
    l.logW = b->logW;
    l.targs = b->d_args;
    l.items = b->d_items;
    l.nitems = b->nitems;
    l.chunk = b->chunk;
    const int64_t need = (b->nitems + b->chunk - 1) / b->chunk;
    l.grid = (int)std::min<int64_t>(b->grid, std::max<int64_t>(need, 1));
    l.npairs = b->n;
    l.counter = b->d_counter;
    l.keys = b->d_keys;
    l.Ngiven = b->d_N;
    l.lag = lag;
    l.val = val;
    l.st = st;
    return l;
}

}  // namespace

extern "C" {

apx_status apx_batch_create(apx_ctx ctx, int32_t n, const float* const* refs, const int64_t* L,
                            const float* const* tmpl, const int32_t* N, const apx_params* params, int32_t logW,
                            void* stream, apx_batch* out) {
    if (!out) return fail(APX_E_INVALID, "null output handle");
    *out = nullptr;
    if (!ctx || !refs || !L || !tmpl || !N || !params) return fail(APX_E_INVALID, "null argument");
    if (n < 1) return fail(APX_E_INVALID, "batch of %d pairs", n);
    const int mode = params->mode;
    if (mode != APX_FULL_FP32 && mode != APX_SYM && mode != APX_ASYM2 && mode != APX_ASYM3)
        return fail(APX_E_UNSUPPORTED, "batched matching runs a fixed mode (FP32, symmetric or asymmetric)");
    if (logW != 0 && (logW < BATCH_LOGW_MIN || logW > BATCH_LOGW_MAX))
        return fail(APX_E_INVALID, "log2 FFT length %d outside [%d, %d]", logW, BATCH_LOGW_MIN, BATCH_LOGW_MAX);
    for (int i = 0; i < n; ++i) {
        if (!refs[i] || !tmpl[i]) return fail(APX_E_INVALID, "pair %d: null pointer", i);
        if (N[i] < 1 || L[i] < N[i]) return fail(APX_E_INVALID, "pair %d: need 1 <= N <= L", i);
        if (L[i] + N[i] - 1 > (int64_t)0xFFFFFFFEll) return fail(APX_E_UNSUPPORTED, "pair %d: too long", i);
    }
    hipStream_t st = (hipStream_t)stream;
    if (logW != 0) return batch_build(ctx, n, refs, L, tmpl, N, params, logW, st, out);

    // autotuning: every FFT length that fits all pairs, times a grab of 1, 2 or 4 items;
    // each candidate is run once to warm up and once timed on the caller's stream
    apx_batch best = nullptr;
    float best_ms = 0.0f;
    int best_chunk = 1;
    std::string log;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int64_t* lag = nullptr;
    float* val = nullptr;
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    apx_status r = APX_OK;
    if (hipMalloc((void**)&lag, sizeof(int64_t) * n) != hipSuccess ||
        hipMalloc((void**)&val, sizeof(float) * n) != hipSuccess)
        r = fail(APX_E_NOMEM, "tuning outputs");
    for (int lw = BATCH_LOGW_MIN; lw <= BATCH_LOGW_MAX && r == APX_OK; ++lw) {
        bool fits = true;
        for (int i = 0; i < n && fits; ++i) fits = batch_block(mode, N[i], 1 << lw) != 0;
        if (!fits) continue;
        apx_batch b = nullptr;
        apx_status rb = batch_build(ctx, n, refs, L, tmpl, N, params, lw, st, &b);
        if (rb == APX_E_NOMEM || rb == APX_E_UNSUPPORTED) continue;
        if (rb != APX_OK) {
            r = rb;
            break;
        }
        bool kept = false;
        for (int chunk : {1, 2, 4}) {
            b->chunk = chunk;
            hipError_t e = launch_batch(batch_args(b, lag, val, st));
            if (e == hipSuccess) e = hipEventRecord(e0, st);
            if (e == hipSuccess) e = launch_batch(batch_args(b, lag, val, st));
            if (e == hipSuccess) e = hipEventRecord(e1, st);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.0f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                r = fail(APX_E_DEVICE, "tuning run: %s", hipGetErrorString(e));
                break;
            }
            char line[96];
            snprintf(line, sizeof line, "%slogW=%d chunk=%d %.3f ms", log.empty() ? "" : "; ", lw, chunk, ms);
            log += line;
            if (!best || ms < best_ms) {
                if (best && best != b) batch_free(best);
                best = b;
                best_ms = ms;
                best_chunk = chunk;
                kept = true;
            }
        }
        if (!kept) batch_free(b);
    }
    if (lag) (void)hipFree(lag);
    if (val) (void)hipFree(val);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (r != APX_OK) {
        if (best) batch_free(best);
        return r;
    }
    if (!best) return fail(APX_E_UNSUPPORTED, "no FFT length up to %d fits every pair", 1 << BATCH_LOGW_MAX);
    best->chunk = best_chunk;
    best->tune_log = log;
    *out = best;
    return APX_OK;
}

apx_status apx_batch_run(apx_ctx ctx, apx_batch b, int64_t* lag_out, float* val_out, void* stream) {
    if (!ctx || !b || !lag_out || !val_out) return fail(APX_E_INVALID, "null argument");
    if (b->ctx != ctx) return fail(APX_E_INVALID, "batch belongs to another context");
    HIPCHK(hipSetDevice(ctx->device));
    HIPCHK(launch_batch(batch_args(b, lag_out, val_out, (hipStream_t)stream)));
    return APX_OK;
}

apx_status apx_batch_blocks(apx_batch b, int32_t* W_block, int32_t* logW, int32_t* nitems) {
    if (!b) return fail(APX_E_INVALID, "null batch");
    if (W_block) memcpy(W_block, b->W_block.data(), sizeof(int32_t) * b->n);
    if (logW) *logW = b->logW;
    if (nitems) *nitems = b->nitems;
    return APX_OK;
}

apx_status apx_batch_describe(apx_batch b, char* buf, int32_t size) {
    if (!b || !buf || size < 1) return fail(APX_E_INVALID, "null argument");
    snprintf(buf, size, "kernel=k_batch<%d,%d> pairs=%d items=%d chunk=%d grid=%d wg_per_cu=%d lds=%zu tune=[%s]",
             b->mode, b->logW, b->n, b->nitems, b->chunk, b->grid, b->per_cu, batch_lds_bytes(b->mode, b->logW),
             b->tune_log.c_str());
    return APX_OK;
}

apx_status apx_batch_destroy(apx_batch b) {
    batch_free(b);
    return APX_OK;
}

apx_status apx_xcorr_argmax_batch(apx_ctx ctx, int32_t n, const float* const* refs, const int64_t* L,
                                  const float* const* tmpl, const int32_t* N, const apx_params* params,
                                  int64_t* lag_out, float* val_out, void* stream) {
    apx_batch b = nullptr;
    apx_status r = apx_batch_create(ctx, n, refs, L, tmpl, N, params, 0, stream, &b);
    if (r != APX_OK) return r;
    r = apx_batch_run(ctx, b, lag_out, val_out, stream);
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    batch_free(b);
    if (r != APX_OK) return r;
    if (e != hipSuccess) return fail(APX_E_DEVICE, "%s", hipGetErrorString(e));
    return APX_OK;
}

}  // extern "C"

// ------------------------------------------------------------------------------------------
// Filter bank on split-precision matrix cores
// ------------------------------------------------------------------------------------------
struct apx_fbank_s {
    apx_ctx ctx = nullptr;
    int32_t F = 0, N = 0, KS = 0, prec = 0;
    int per_cu = 0, cus = 0;
    void* frag = nullptr;
};

extern "C" {

apx_status apx_fbank_create(apx_ctx ctx, const float* h, int32_t F, int32_t N, int32_t prec, void* stream,
                            apx_fbank* out) {
    if (!out) return fail(APX_E_INVALID, "null output handle");
    *out = nullptr;
    if (!ctx || !h) return fail(APX_E_INVALID, "null argument");
    if (F < 1 || F > 32) return fail(APX_E_INVALID, "F = %d filters: one bank holds 1..32", F);
    if (N < 1) return fail(APX_E_INVALID, "N = %d taps", N);
    if (prec != APX_FB_F16X3 && prec != APX_FB_BF16X3) return fail(APX_E_INVALID, "unknown precision %d", prec);
    const int KS = fb_ks_for(N);
    if (KS == 0) return fail(APX_E_UNSUPPORTED, "N = %d taps: the matrix-core bank takes N <= 512", N);
    HIPCHK(hipSetDevice(ctx->device));
    apx_fbank fb = new (std::nothrow) apx_fbank_s;
    if (!fb) return fail(APX_E_NOMEM, "host allocation failed");
    fb->ctx = ctx;
    fb->F = F;
    fb->N = N;
    fb->KS = KS;
    fb->prec = prec;
    const size_t bytes = (size_t)2 * KS * 64 * 16;
    if (hipMalloc(&fb->frag, bytes) != hipSuccess) {
        delete fb;
        return fail(APX_E_NOMEM, "tap fragments");
    }
    hipError_t e = fb_prepare(h, F, N, KS, prec, fb->frag, (hipStream_t)stream);
    if (e == hipSuccess) e = fb_occupancy(prec, KS, &fb->per_cu);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&fb->cus, hipDeviceAttributeMultiprocessorCount, ctx->device);
    if (e != hipSuccess || fb->per_cu < 1) {
        (void)hipFree(fb->frag);
        delete fb;
        return fail(APX_E_DEVICE, "filter bank setup: %s", hipGetErrorString(e));
    }
    *out = fb;
    return APX_OK;
}

apx_status apx_fbank_run(apx_ctx ctx, apx_fbank fb, const float* x, int32_t C, int64_t L, int64_t ldx, float* y,
                         int64_t ldy, void* stream) {
    if (!ctx || !fb || !x || !y) return fail(APX_E_INVALID, "null argument");
    if (fb->ctx != ctx) return fail(APX_E_INVALID, "bank belongs to another context");
    if (C < 1 || L < 1) return fail(APX_E_INVALID, "C = %d, L = %lld", C, (long long)L);
    if (ldx < L) return fail(APX_E_INVALID, "ldx = %lld < L", (long long)ldx);
    const int64_t Lout = L + fb->N - 1;
    if (ldy < Lout) return fail(APX_E_INVALID, "ldy = %lld < L + N - 1 = %lld", (long long)ldy, (long long)Lout);
    HIPCHK(hipSetDevice(ctx->device));
    FbLaunch b{};
    b.prec = fb->prec;
    b.KS = fb->KS;
    b.x = x;
    b.C = C;
    b.L = L;
    b.ldx = ldx;
    b.frag = fb->frag;
    b.F = fb->F;
    b.Lout = Lout;
    b.y = y;
    b.ldy = ldy;
    const int64_t items = (int64_t)C * ((Lout + fb_tile_rows() - 1) / fb_tile_rows());
    b.grid = (int)std::min<int64_t>((int64_t)fb->per_cu * fb->cus, items);
    b.st = (hipStream_t)stream;
    HIPCHK(fb_launch(b));
    return APX_OK;
}

apx_status apx_fbank_describe(apx_fbank fb, char* buf, int32_t size) {
    if (!fb || !buf || size < 1) return fail(APX_E_INVALID, "null argument");
    snprintf(buf, size, "kernel=k_fbank<%d,%d,%d> F=%d N=%d taps_padded=%d tile_rows=%lld wg_per_cu=%d grid=%d",
             fb->prec, fb->KS, FB_WAVES, fb->F, fb->N, 16 * fb->KS, (long long)fb_tile_rows(), fb->per_cu,
             fb->per_cu * fb->cus);
    return APX_OK;
}

apx_status apx_fbank_destroy(apx_fbank fb) {
    if (!fb) return APX_OK;
    (void)hipSetDevice(fb->ctx->device);
    if (fb->frag) (void)hipFree(fb->frag);
    delete fb;
    return APX_OK;
}

}  // extern "C"
