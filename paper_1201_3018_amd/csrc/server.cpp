// Serving engine of libapx: a request loop for convolution / correlation requests of mixed L
// and N.  One scheduler thread per server:
//   - admits queued requests in arrival order while the device memory they need (input, output,
//     workspace, and the prepared kernel on a cache miss) fits the HBM budget and an in-flight
//     slot is free; idle cached kernels are evicted (least recently used first) to make room;
//   - launches every admitted request at once on one of several HIP streams (copy in, the
//     per-call calibration and the block kernel, copy out), so requests that arrive while
//     others run overlap with them on the device;
//   - keeps prepared kernels (companded / packed taps, spectra or coefficient tables) resident,
//     keyed by the caller's kernel key, so repeated kernels skip their preparation;
//   - retires finished requests by polling their completion events and releases their memory.
// Device buffers come from a caching allocator with power-of-two classes; the budget applies to
// the bytes of the classes in use.
#include <hip/hip_runtime.h>
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "engine.h"
#include "internal.h"

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

size_t size_class(size_t n) {
    size_t c = 4096;
    while (c < n) c <<= 1;
    return c;
}

// Block size the server gives a request: time-domain core up to 129 taps, FFT core above, the
// smallest power of two whose block holds W >= 2N outputs (Section III opening).
int32_t server_block(int32_t N) {
    const int32_t no = (N % 2) ? N : N + 1;
    int32_t wb = no <= 129 ? 1024 : 512;
    while (wb - no - 1 < 2 * no) wb *= 2;
    return wb;
}

// Upper bound of a prepared kernel's device memory (taps in five forms, spectra or coefficient
// tables for every mode), for admission before the kernel exists.
size_t kernel_bytes_bound(int32_t N, int32_t W_block) {
    return (size_t)64 * (N + 64) + (size_t)160 * W_block + 8 * 4096;
}

struct Key {
    uint64_t key;
    int32_t N, op, W_block, mode;
    bool operator==(const Key& o) const {
        return key == o.key && N == o.N && op == o.op && W_block == o.W_block && mode == o.mode;
    }
};
struct KeyHash {
    size_t operator()(const Key& k) const {
        uint64_t h = k.key * 0x9E3779B97F4A7C15ull;
        h ^= ((uint64_t)(uint32_t)k.N << 32) ^ ((uint64_t)(uint32_t)k.W_block << 8) ^ (uint64_t)(k.op * 31 + k.mode);
        return (size_t)(h ^ (h >> 29));
    }
};

struct KEntry {
    apx_kernel k = nullptr;
    float* taps = nullptr;
    size_t taps_cls = 0;
    size_t bytes = 0;
    int refs = 0;
    hipEvent_t ready = nullptr;
    std::list<Key>::iterator lru;
};

struct Req {
    uint64_t ticket = 0;
    apx_request r{};
    double t_submit = 0.0, t_admit = 0.0;
    void *s_dev = nullptr, *o_dev = nullptr, *ws = nullptr;
    size_t s_cls = 0, o_cls = 0, ws_cls = 0;
    KEntry* ke = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    int32_t W_block = 0, core = 0, status = APX_OK;
};

struct DevPool {
    std::map<size_t, std::vector<void*>> free_;
    std::vector<void*> all_;
    std::atomic<size_t> reserved{0};  // read by the stats call on other threads
    void* get(size_t cls) {
        auto& v = free_[cls];
        if (!v.empty()) {
            void* p = v.back();
            v.pop_back();
            return p;
        }
        void* p = nullptr;
        if (hipMalloc(&p, cls) != hipSuccess) return nullptr;
        all_.push_back(p);
        reserved += cls;
        return p;
    }
    void put(void* p, size_t cls) {
        if (p) free_[cls].push_back(p);
    }
    void release() {
        for (void* p : all_) (void)hipFree(p);
        all_.clear();
        free_.clear();
        reserved = 0;
    }
};

}  // namespace

struct apx_server_s {
    apx_ctx ctx = nullptr;
    apx_server_config cfg{};
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    std::vector<hipEvent_t> ev_free;
    DevPool pool;
    std::unordered_map<Key, KEntry, KeyHash> cache;
    std::list<Key> lru;  // front: most recently used
    std::vector<Req*> inflight;
    size_t in_use = 0;
    apx_server_counters st{};
    // shared with the caller's threads
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<Req*> queue;
    std::deque<apx_completion> done;
    uint64_t next_ticket = 1;
    int64_t outstanding = 0;
    bool stop = false;
    std::thread th;

    hipEvent_t event() {
        if (!ev_free.empty()) {
            hipEvent_t e = ev_free.back();
            ev_free.pop_back();
            return e;
        }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
        return e;
    }

    size_t need_of(const Req* q, bool* miss) {
        const apx_request& r = q->r;
        const Key key{r.kernel_key, r.N, r.op, q->W_block, r.mode};
        size_t need = size_class((size_t)r.L * 4) + size_class((size_t)(r.L + r.N - 1) * 4) +
                      size_class(apx_workspace_bytes());
        *miss = cache.find(key) == cache.end();
        if (*miss) need += kernel_bytes_bound(r.N, q->W_block) + size_class((size_t)r.N * 4);
        return need;
    }

    bool evict_one() {
        for (auto it = lru.rbegin(); it != lru.rend(); ++it) {
            auto c = cache.find(*it);
            if (c->second.refs > 0) continue;
            KEntry& e = c->second;
            (void)hipEventSynchronize(e.ready);
            apx_kernel_destroy(e.k);
            pool.put(e.taps, e.taps_cls);
            ev_free.push_back(e.ready);
            in_use -= e.bytes;
            lru.erase(std::next(it).base());
            cache.erase(c);
            st.evictions++;
            return true;
        }
        return false;
    }

    void finish(Req* q, int status) {
        pool.put(q->s_dev, q->s_cls);
        pool.put(q->o_dev, q->o_cls);
        pool.put(q->ws, q->ws_cls);
        in_use -= q->s_cls + q->o_cls + q->ws_cls;
        if (q->ke) q->ke->refs--;
        if (q->done) ev_free.push_back(q->done);
        apx_completion c{};
        c.ticket = q->ticket;
        c.status = status;
        c.core = q->core;
        c.W_block = q->W_block;
        c.t_submit = q->t_submit;
        c.t_admit = q->t_admit;
        c.t_done = now_s();
        c.L = q->r.L;
        c.N = q->r.N;
        {
            std::lock_guard<std::mutex> g(mu);
            done.push_back(c);
            outstanding--;
            if (status == APX_OK) st.completed++;
            else st.failed++;
        }
        cv_done.notify_all();
        delete q;
    }

    // Enqueue everything of an admitted request on one stream.
    int launch(Req* q) {
        const apx_request& r = q->r;
        hipStream_t s = streams[next_stream];
        next_stream = (next_stream + 1) % (int)streams.size();
        q->stream = s;
        const Key key{r.kernel_key, r.N, r.op, q->W_block, r.mode};
        auto it = cache.find(key);
        if (it == cache.end()) {
            KEntry e;
            e.taps_cls = size_class((size_t)r.N * 4);
            e.taps = (float*)pool.get(e.taps_cls);
            if (!e.taps) return APX_E_NOMEM;
            apx_params prm{};
            prm.mode = r.mode;
            prm.core = APX_CORE_AUTO;
            prm.snr_min_db = isfinite(r.snr_min_db) ? r.snr_min_db : 0.0;
            prm.calib_db = NAN;
            apx_kernel k = nullptr;
            int rc = APX_E_DEVICE;
            if (hipMemcpyAsync(e.taps, r.k, (size_t)r.N * 4, hipMemcpyHostToDevice, s) == hipSuccess)
                rc = apx_kernel_create(ctx, e.taps, r.N, r.op, q->W_block, &prm, s, &k);
            e.ready = event();
            if (rc == APX_OK && (!e.ready || hipEventRecord(e.ready, s) != hipSuccess)) rc = APX_E_DEVICE;
            if (rc != APX_OK) {
                if (k) apx_kernel_destroy(k);
                if (e.ready) ev_free.push_back(e.ready);
                (void)hipStreamSynchronize(s);
                pool.put(e.taps, e.taps_cls);
                return rc;
            }
            e.k = k;
            e.bytes = k->dev_bytes + e.taps_cls;
            in_use += e.bytes;
            lru.push_front(key);
            e.lru = lru.begin();
            {
                // the stats call reads the cache and the counters under the same lock
                std::lock_guard<std::mutex> g(mu);
                it = cache.emplace(key, e).first;
                st.kernel_misses++;
            }
        } else {
            {
                std::lock_guard<std::mutex> g(mu);
                st.kernel_hits++;
            }
            lru.splice(lru.begin(), lru, it->second.lru);
            if (hipStreamWaitEvent(s, it->second.ready, 0) != hipSuccess) return APX_E_DEVICE;
        }
        KEntry& e = it->second;
        e.refs++;
        q->ke = &e;
        q->core = e.k->core;
        q->s_cls = size_class((size_t)r.L * 4);
        q->o_cls = size_class((size_t)(r.L + r.N - 1) * 4);
        q->ws_cls = size_class(apx_workspace_bytes());
        q->s_dev = pool.get(q->s_cls);
        q->o_dev = pool.get(q->o_cls);
        q->ws = pool.get(q->ws_cls);
        in_use += q->s_cls + q->o_cls + q->ws_cls;
        if (!q->s_dev || !q->o_dev || !q->ws) return APX_E_NOMEM;
        q->done = event();
        if (!q->done) return APX_E_DEVICE;
        if (hipMemcpyAsync(q->s_dev, r.s, (size_t)r.L * 4, hipMemcpyHostToDevice, s) != hipSuccess) return APX_E_DEVICE;
        int rc;
        if (r.mode == APX_AUTO_SNR)
            rc = apx_run_auto(ctx, e.k, (const float*)q->s_dev, r.L, (float*)q->o_dev, nullptr, r.snr_min_db, 0, q->ws,
                              s);
        else
            rc = apx_run(ctx, e.k, (const float*)q->s_dev, r.L, (float*)q->o_dev, nullptr, s);
        if (rc != APX_OK) return rc;
        if (hipMemcpyAsync(r.r_out, q->o_dev, (size_t)(r.L + r.N - 1) * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
            return APX_E_DEVICE;
        if (hipEventRecord(q->done, s) != hipSuccess) return APX_E_DEVICE;
        return APX_OK;
    }

    void loop() {
        (void)hipSetDevice(ctx->device);
        for (;;) {
            // retire finished requests
            for (size_t i = 0; i < inflight.size();) {
                hipError_t e = hipEventQuery(inflight[i]->done);
                if (e == hipErrorNotReady) {
                    ++i;
                    continue;
                }
                Req* q = inflight[i];
                inflight[i] = inflight.back();
                inflight.pop_back();
                finish(q, e == hipSuccess ? APX_OK : APX_E_DEVICE);
            }
            // admit in arrival order
            bool admitted = false;
            for (;;) {
                Req* q = nullptr;
                {
                    std::lock_guard<std::mutex> g(mu);
                    if (queue.empty() || (int)inflight.size() >= cfg.max_inflight) break;
                    q = queue.front();
                    bool miss = false;
                    size_t need = need_of(q, &miss);
                    while (in_use + need > (size_t)cfg.hbm_budget && evict_one()) {
                    }
                    if (in_use + need > (size_t)cfg.hbm_budget) break;  // wait for memory
                    queue.pop_front();
                }
                q->t_admit = now_s();
                int rc = launch(q);
                {
                    std::lock_guard<std::mutex> g(mu);
                    st.peak_bytes = std::max<int64_t>(st.peak_bytes, (int64_t)in_use);
                }
                if (rc != APX_OK) {
                    // work may be enqueued on the stream: let it end before the buffers go back
                    if (q->stream) (void)hipStreamSynchronize(q->stream);
                    finish(q, rc);
                    continue;
                }
                inflight.push_back(q);
                admitted = true;
            }
            std::unique_lock<std::mutex> lk(mu);
            if (stop && queue.empty() && inflight.empty()) break;
            if (inflight.empty()) {
                cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            } else if (!admitted) {
                cv_work.wait_for(lk, std::chrono::microseconds(50));
            }
        }
    }
};

extern "C" {

apx_status apx_server_create(apx_ctx ctx, const apx_server_config* cfg, apx_server* out) {
    if (!out) return APX_E_INVALID;
    *out = nullptr;
    if (!ctx || !cfg) return APX_E_INVALID;
    if (cfg->hbm_budget < (1 << 20) || cfg->n_streams < 1 || cfg->n_streams > 64 || cfg->max_inflight < 1)
        return APX_E_INVALID;
    if (hipSetDevice(ctx->device) != hipSuccess) return APX_E_DEVICE;
    apx_server srv = new (std::nothrow) apx_server_s;
    if (!srv) return APX_E_NOMEM;
    srv->ctx = ctx;
    srv->cfg = *cfg;
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t t : srv->streams) (void)hipStreamDestroy(t);
            delete srv;
            return APX_E_DEVICE;
        }
        srv->streams.push_back(s);
    }
    srv->th = std::thread([srv] { srv->loop(); });
    *out = srv;
    return APX_OK;
}

double apx_server_now(void) { return now_s(); }

apx_status apx_server_submit(apx_server srv, const apx_request* r, uint64_t* ticket) {
    if (!srv || !r) return APX_E_INVALID;
    if (!r->s || !r->k || !r->r_out || r->N < 1 || r->L < r->N) return APX_E_INVALID;
    if (reinterpret_cast<uintptr_t>(r->s) & 7) return APX_E_INVALID;  // s_in must be 8-byte aligned
    if (r->op != APX_CONV && r->op != APX_XCORR) return APX_E_INVALID;
    if (r->mode < APX_FULL_FP32 || r->mode > APX_FULL_FP64) return APX_E_INVALID;
    if (r->mode == APX_AUTO_SNR && !isfinite(r->snr_min_db)) return APX_E_INVALID;
    Req* q = new (std::nothrow) Req;
    if (!q) return APX_E_NOMEM;
    q->r = *r;
    q->W_block = r->W_block > 0 ? r->W_block : server_block(r->N);
    q->t_submit = now_s();
    {
        std::lock_guard<std::mutex> g(srv->mu);
        const size_t need = size_class((size_t)r->L * 4) + size_class((size_t)(r->L + r->N - 1) * 4) +
                            size_class(apx_workspace_bytes()) + kernel_bytes_bound(r->N, q->W_block) +
                            size_class((size_t)r->N * 4);
        if (need > (size_t)srv->cfg.hbm_budget) {
            srv->st.rejected++;
            delete q;
            return APX_E_NOMEM;
        }
        q->ticket = srv->next_ticket++;
        srv->queue.push_back(q);
        srv->outstanding++;
        srv->st.submitted++;
    }
    srv->cv_work.notify_one();
    if (ticket) *ticket = q->ticket;
    return APX_OK;
}

apx_status apx_server_poll(apx_server srv, apx_completion* out, int32_t max, int32_t* n, int32_t wait_ms) {
    if (!srv || !out || !n || max < 1) return APX_E_INVALID;
    std::unique_lock<std::mutex> lk(srv->mu);
    if (srv->done.empty() && wait_ms > 0)
        srv->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), [&] { return !srv->done.empty(); });
    int32_t k = 0;
    while (k < max && !srv->done.empty()) {
        out[k++] = srv->done.front();
        srv->done.pop_front();
    }
    *n = k;
    return APX_OK;
}

apx_status apx_server_drain(apx_server srv) {
    if (!srv) return APX_E_INVALID;
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->outstanding == 0; });
    return APX_OK;
}

apx_status apx_server_stats(apx_server srv, apx_server_counters* out) {
    if (!srv || !out) return APX_E_INVALID;
    std::lock_guard<std::mutex> g(srv->mu);
    *out = srv->st;
    out->reserved_bytes = (int64_t)srv->pool.reserved.load();
    out->cached_kernels = (int32_t)srv->cache.size();
    return APX_OK;
}

apx_status apx_server_destroy(apx_server srv) {
    if (!srv) return APX_OK;
    {
        std::lock_guard<std::mutex> g(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->th.joinable()) srv->th.join();
    (void)hipSetDevice(srv->ctx->device);
    for (hipStream_t s : srv->streams) (void)hipStreamSynchronize(s);
    for (auto& kv : srv->cache) {
        apx_kernel_destroy(kv.second.k);
        if (kv.second.ready) (void)hipEventDestroy(kv.second.ready);
    }
    srv->cache.clear();
    for (hipEvent_t e : srv->ev_free) (void)hipEventDestroy(e);
    srv->pool.release();
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
    delete srv;
    return APX_OK;
}

}  // extern "C"
