// Autotuner of the convolution path.  For one kernel shape (taps N, operation, packing mode,
// block size or "choose one") it prepares the kernel on every core and FFT implementation that
// can run the shape, times each on a synthetic signal on the device, and records the fastest in
// the context's table.  apx_kernel_create with core and FFT implementation left automatic, and
// W_block = 0, consult the table.  The table is kept in a text file per user (APX_TUNE_FILE, else
// $HOME/.cache/apx_tune.txt), keyed by the device's architecture, so a later process starts
// with it.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <string>
#include <vector>

#include "engine.h"
#include "internal.h"

namespace {

int odd_of(int32_t N) { return (N % 2) ? N : N + 1; }

// Smallest power-of-two block whose W = W_block - N_odd - 1 holds at least 2 N_odd outputs
// (Section III opening), and the time-domain reach of the default rule.
int32_t min_block(int32_t N) {
    const int32_t no = odd_of(N);
    int32_t wb = 256;
    while (wb - no - 1 < 2 * no) wb *= 2;
    return wb;
}

std::string tune_path() {
    const char* e = getenv("APX_TUNE_FILE");
    if (e && *e) return e;
    const char* h = getenv("HOME");
    return std::string(h && *h ? h : "/tmp") + "/.cache/apx_tune.txt";
}

std::string arch_of(int device) {
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) return "unknown";
    std::string a = p.gcnArchName;
    for (char& c : a)
        if (c == ' ') c = '_';
    return a;
}

// Table line: arch, N_odd, op, mode, W_block asked for (0: chosen too), then core, FFT
// implementation, W_block, picoseconds per output measured and the tile (integer core: output
// tiles per pass, time-domain core: outputs per thread; a line without the field reads as 0,
// the shape's default).
bool parse(const char* line, std::string* arch, apx::TuneKey* k, apx::TuneVal* v) {
    char a[128];
    double us = 0.0;
    int tile = 0;
    const int got = sscanf(line, "%127s %d %d %d %d %d %d %d %lf %d", a, &k->N_odd, &k->op, &k->mode, &k->W_block,
                           &v->core, &v->variant, &v->W_block, &us, &tile);
    if (got < 9) return false;
    *arch = a;
    v->ps_per_output = us;
    const bool ok = v->core == APX_CORE_INT8 ? (tile >= 1 && tile <= 3) : v->core == APX_CORE_TIME && (tile == 4 || tile == 8);
    v->tile = (got == 10 && ok) ? tile : 0;
    return true;
}

void save(apx_ctx ctx) {
    const std::string path = tune_path();
    std::vector<std::string> keep;
    if (FILE* f = fopen(path.c_str(), "r")) {  // other devices' lines stay
        char line[512];
        while (fgets(line, sizeof line, f)) {
            std::string arch;
            apx::TuneKey k;
            apx::TuneVal v;
            if (parse(line, &arch, &k, &v) && arch != ctx->arch) keep.push_back(line);
        }
        fclose(f);
    }
    const size_t slash = path.rfind('/');
    if (slash != std::string::npos) (void)mkdir(path.substr(0, slash).c_str(), 0755);  // e.g. ~/.cache
    const std::string tmp = path + ".tmp" + std::to_string((long long)getpid());
    FILE* f = fopen(tmp.c_str(), "w");
    if (!f) return;  // the table stays in memory only
    for (const std::string& l : keep) fputs(l.c_str(), f);
    for (const auto& kv : ctx->tuned)
        fprintf(f, "%s %d %d %d %d %d %d %d %.3f %d\n", ctx->arch.c_str(), kv.first.N_odd, kv.first.op,
                kv.first.mode, kv.first.W_block, kv.second.core, kv.second.variant, kv.second.W_block,
                kv.second.ps_per_output, kv.second.tile);
    fclose(f);
    if (rename(tmp.c_str(), path.c_str()) != 0) remove(tmp.c_str());
}

// Deterministic test signal: two tones and a linear congruential noise, |x| < 1.
std::vector<float> test_signal(int64_t L) {
    std::vector<float> s((size_t)L);
    uint32_t x = 12345u;
    for (int64_t i = 0; i < L; ++i) {
        x = x * 1664525u + 1013904223u;
        const double noise = ((double)(x >> 8) / 16777216.0 - 0.5) * 0.4;
        s[(size_t)i] = (float)(0.4 * sin(0.031 * (double)i) + 0.2 * sin(0.47 * (double)i) + noise);
    }
    return s;
}

}  // namespace

namespace apx {

void tune_load(apx_ctx ctx) {
    ctx->arch = arch_of(ctx->device);
    FILE* f = fopen(tune_path().c_str(), "r");
    if (!f) return;
    char line[512];
    while (fgets(line, sizeof line, f)) {
        std::string arch;
        TuneKey k;
        TuneVal v;
        if (parse(line, &arch, &k, &v) && arch == ctx->arch) ctx->tuned[k] = v;
    }
    fclose(f);
}

bool tune_lookup(apx_ctx ctx, int32_t N_odd, int32_t op, int32_t mode, int32_t W_block, TuneVal* out) {
    auto it = ctx->tuned.find(TuneKey{N_odd, op, mode, W_block});
    if (it == ctx->tuned.end()) return false;
    *out = it->second;
    return true;
}

int32_t default_block(int32_t N) {
    const int32_t no = odd_of(N);
    int32_t wb = no <= 129 ? 1024 : 512;
    while (wb - no - 1 < 2 * no) wb *= 2;
    return wb;
}

void resolve_tuned(apx_ctx ctx, int32_t N, int32_t op, int32_t* W_block, apx_params* p, int32_t* tile) {
    const int32_t no = odd_of(N);
    const bool auto_core = p->core == APX_CORE_AUTO && p->fft_variant == 0;
    TuneVal v;
    if (*W_block == 0) {
        if (tune_lookup(ctx, no, op, p->mode, 0, &v)) {
            *W_block = v.W_block;
            if (auto_core) {
                p->core = v.core;
                p->fft_variant = v.variant;
                if (tile) *tile = v.tile;
            }
            return;
        }
        *W_block = default_block(N);
    }
    if (auto_core && tune_lookup(ctx, no, op, p->mode, *W_block, &v)) {
        p->core = v.core;
        p->fft_variant = v.variant;
        if (tile) *tile = v.tile;
    }
}

}  // namespace apx

extern "C" {

apx_status apx_tune(apx_ctx ctx, const float* k, int32_t N, int32_t op, int32_t W_block, const apx_params* params,
                    int64_t L_hint, void* stream, apx_tuned* out) {
    if (!ctx || !k || !params || !out) return apx::set_error(APX_E_INVALID, "null argument");
    if (N < 1) return apx::set_error(APX_E_INVALID, "N = %d", N);
    if (op != APX_CONV && op != APX_XCORR) return apx::set_error(APX_E_INVALID, "unknown op %d", op);
    if (W_block < 0) return apx::set_error(APX_E_INVALID, "W_block = %d", W_block);
    if (L_hint < 0 || (L_hint > 0 && L_hint < N)) return apx::set_error(APX_E_INVALID, "L_hint = %lld", (long long)L_hint);
    const int32_t N_odd = odd_of(N);
    std::vector<int32_t> blocks;
    if (W_block > 0) {
        if (apx_geometry(N, N, W_block, nullptr, nullptr, nullptr) != APX_OK) return APX_E_INVALID;
        blocks.push_back(W_block);
    } else {
        const int32_t b0 = min_block(N);
        for (int i = 0; i < 3; ++i) blocks.push_back(b0 << i);
    }
    hipStream_t st = (hipStream_t)stream;
    if (hipSetDevice(ctx->device) != hipSuccess) return apx::set_error(APX_E_DEVICE, "hipSetDevice failed");
    // the caller's signal length, else 64 of the largest blocks' outputs (at least 2^16 samples):
    // how many blocks a call has decides how much parallelism each core finds
    const int32_t wb_max = blocks.back();
    const int64_t L = L_hint > 0 ? L_hint : std::max<int64_t>((int64_t)64 * (wb_max - N_odd - 1), 1 << 16);
    const std::vector<float> hs = test_signal(L);
    // the timed runs rotate over copies of the signal and outputs that together exceed the
    // device's last-level cache (256 MiB on MI355X), so that inputs come from HBM as they do
    // in a real stream of calls
    const int64_t one = (int64_t)(2 * L + N - 1) * 4;
    const int nbuf = (int)std::max<int64_t>(1, std::min<int64_t>(16, ((int64_t)512 << 20) / one));
    float *s = nullptr, *o = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc((void**)&s, (size_t)L * 4 * nbuf);
    if (e == hipSuccess) e = hipMalloc((void**)&o, (size_t)(L + N - 1) * 4 * nbuf);
    for (int b = 0; b < nbuf && e == hipSuccess; ++b)
        e = hipMemcpy(s + (size_t)L * b, hs.data(), (size_t)L * 4, hipMemcpyHostToDevice);
    auto sig = [&](int i) { return s + (size_t)L * (i % nbuf); };
    auto res = [&](int i) { return o + (size_t)(L + N - 1) * (i % nbuf); };
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    apx_tuned best{};
    best.ps_per_output = INFINITY;
    int tried = 0;
    char table[4096];
    int used = 0;
    table[0] = 0;
    // candidates: time-domain core with 4 and 8 outputs per thread, integer core (fixed packed
    // modes) with each count of output tiles per pass up to the tiles a block has, FFT core in
    // each of its implementations (LDS passes; one wave per block; a group of waves per block).
    // Every
    // candidate that runs the shape is prepared first; then rounds of timed runs visit them in
    // turn and each keeps its fastest round, so that a slow moment of the device (another
    // process, a profiler) does not decide the choice.
    const int cores[5][2] = {{APX_CORE_TIME, 0}, {APX_CORE_INT8, 0}, {APX_CORE_FFT, 1}, {APX_CORE_FFT, 2},
                             {APX_CORE_FFT, 3}};
    struct Cand {
        int32_t wb, core, variant, tile;
        apx_kernel kern;
        double ps;
    };
    std::vector<Cand> cands;
    for (int32_t wb : blocks) {
        if (e != hipSuccess) break;
        for (const auto& cv : cores) {
            apx_params p = *params;
            p.core = cv[0];
            p.fft_variant = cv[1];
            int tiles[3] = {0, 0, 0}, ntile = 1;
            if (cv[0] == APX_CORE_INT8) {
                ntile = std::min(3, std::max(1, apx::i8_tiles(N_odd, wb - N_odd - 1)));
                for (int t = 0; t < ntile; ++t) tiles[t] = t + 1;
            } else if (cv[0] == APX_CORE_TIME) {
                ntile = 2;
                tiles[0] = 4;
                tiles[1] = 8;
            }
            for (int ti = 0; ti < ntile; ++ti) {
                const int t = tiles[ti];
                apx_kernel kern = nullptr;
                if (apx_kernel_create(ctx, k, N, op, wb, &p, stream, &kern) != APX_OK) break;  // cannot run it
                if (cv[0] == APX_CORE_INT8) kern->i8_tm = t;
                if (cv[0] == APX_CORE_TIME) kern->td_tile = t;
                bool ok = true;
                for (int i = 0; i < 2 && ok; ++i)
                    ok = apx_run(ctx, kern, sig(i), L, res(i), nullptr, stream) == APX_OK;
                if (!ok) {
                    apx_kernel_destroy(kern);
                    break;
                }
                cands.push_back(Cand{wb, cv[0], cv[1], t, kern, INFINITY});
            }
        }
    }
    constexpr int ROUNDS = 3, REPS = 5;
    int turn = 0;
    for (int round = 0; round < ROUNDS; ++round) {
        for (Cand& c : cands) {
            if (!c.kern) continue;
            float ms = 0.0f;
            bool ok = hipEventRecord(e0, st) == hipSuccess;
            for (int i = 0; i < REPS && ok; ++i) {
                ok = apx_run(ctx, c.kern, sig(turn), L, res(turn), nullptr, stream) == APX_OK;
                ++turn;
            }
            ok = ok && hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
                 hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            if (!ok) {  // drop the candidate
                apx_kernel_destroy(c.kern);
                c.kern = nullptr;
                c.ps = INFINITY;
                continue;
            }
            c.ps = std::min(c.ps, (double)ms * 1e9 / REPS / (double)(L + N - 1));  // picoseconds per output
        }
    }
    for (Cand& c : cands) {
        if (!c.kern) continue;
        apx_kernel_destroy(c.kern);
        ++tried;
        if (used < (int)sizeof table - 64)
            used += snprintf(table + used, sizeof table - used, " [W_block %d core %d impl %d tile %d: %.2f ps/output]",
                             c.wb, c.core, c.variant, c.tile, c.ps);
        if (c.ps < best.ps_per_output) {
            best.core = c.core;
            best.fft_variant = c.variant;
            best.W_block = c.wb;
            best.tile = c.tile;
            best.ps_per_output = c.ps;
        }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (s) (void)hipFree(s);
    if (o) (void)hipFree(o);
    if (e != hipSuccess) return apx::set_error(APX_E_DEVICE, "tuning buffers: %s", hipGetErrorString(e));
    if (tried == 0) return apx::set_error(APX_E_UNSUPPORTED, "no core runs N = %d at the block sizes tried", N);
    ctx->tuned[apx::TuneKey{N_odd, op, params->mode, W_block}] =
        apx::TuneVal{best.core, best.fft_variant, best.W_block, best.ps_per_output, best.tile};
    save(ctx);
    *out = best;
    ctx->last_tune = table;
    return APX_OK;
}

apx_status apx_tune_describe(apx_ctx ctx, char* buf, int32_t size) {
    if (!ctx || !buf || size < 1) return apx::set_error(APX_E_INVALID, "null argument");
    std::string s = "device " + ctx->arch + ", table " + tune_path() + ":";
    for (const auto& kv : ctx->tuned) {
        char line[160];
        snprintf(line, sizeof line,
                 "\n  N=%d op=%d mode=%d W_block=%d -> core %d impl %d W_block %d tile %d (%.2f ps/output)",
                 kv.first.N_odd, kv.first.op, kv.first.mode, kv.first.W_block, kv.second.core, kv.second.variant,
                 kv.second.W_block, kv.second.tile, kv.second.ps_per_output);
        s += line;
    }
    if (!ctx->last_tune.empty()) s += "\nlast tuning:" + ctx->last_tune;
    snprintf(buf, size, "%s", s.c_str());
    return APX_OK;
}

}  // extern "C"
