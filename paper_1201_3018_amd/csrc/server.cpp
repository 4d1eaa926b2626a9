// Serving engine of libapx: a request loop for convolution / correlation requests of mixed L
// and N.  One scheduler thread per server:
//   - admits queued requests in arrival order while the device memory they need (input,
//     output, calibration workspace, their share of the launch table, and the prepared kernel
//     on a cache miss, sized exactly by a dry run of its preparation) fits the HBM budget and
//     fewer than max_inflight requests are on the device; idle cached kernels are evicted
//     (least recently used first) to make room;
//   - batches the requests admitted together: requests that use the same prepared kernel go
//     to the device as ONE multi-signal launch of its block core over all their (signal, block)
//     items, after their copies in and per-request calibrations, on one of several HIP
//     streams, so batches that arrive while others run overlap with them on the device;
//   - keeps prepared kernels (companded / packed taps, spectra or coefficient tables)
//     resident, keyed by the caller's kernel key, so repeated kernels skip their preparation;
//   - retires finished batches by polling their completion events and releases their memory.
// Each request is computed exactly as apx_run_auto (or apx_run for fixed modes) computes it
// alone: the multi-signal launch runs every block of every signal as the single-signal launch
// does, with the request's own calibration and SNR target.
// Device buffers come from a caching allocator with power-of-two classes; the budget applies to
// the bytes of the classes in use, and cached free buffers are released before the allocator's
// holdings would pass the budget.
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

// Bytes of one request's entries in a launch table: its arguments and one signal index per
// work item (P blocks and block 0's prefix item).
size_t table_share(int64_t L, int32_t N, int32_t W_block) {
    int64_t P = 0;
    apx_geometry(L, N, W_block, nullptr, nullptr, &P);
    return sizeof(apx::RunArgs) + 4 * (size_t)(P + 1);
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
    int refs = 0;  // admitted requests that use it (it is not evicted while > 0)
    hipEvent_t ready = nullptr;
    std::list<Key>::iterator lru;
};

struct Req {
    uint64_t ticket = 0;
    apx_request r{};
    Key key{};
    double t_submit = 0.0, t_admit = 0.0;
    void *s_dev = nullptr, *o_dev = nullptr, *ws = nullptr;
    size_t s_cls = 0, o_cls = 0, ws_cls = 0, tab_share = 0;
    size_t kern_plan = 0;  // planned bytes of the prepared kernel this request's admission reserved
    int32_t W_block = 0, core = 0;
};

struct Batch {
    std::vector<Req*> reqs;
    KEntry* ke = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* tab_dev = nullptr;
    void* tab_host = nullptr;
    size_t tab_cls = 0;
    bool holds_refs = false;  // the kernel entry counts this batch's requests in its refs
};

// Device buffers by power-of-two class; free buffers are kept for reuse and released (smallest
// classes first) before an allocation would take the holdings past `cap`.
struct DevPool {
    std::map<size_t, std::vector<void*>> free_;
    std::atomic<size_t> reserved{0};  // read by the stats call on other threads
    size_t cap = 0;
    void* get(size_t cls) {
        auto& v = free_[cls];
        if (!v.empty()) {
            void* p = v.back();
            v.pop_back();
            return p;
        }
        if (reserved + cls > cap) trim(reserved + cls - cap);
        void* p = nullptr;
        if (hipMalloc(&p, cls) != hipSuccess) return nullptr;
        reserved += cls;
        return p;
    }
    void put(void* p, size_t cls) {
        if (p) free_[cls].push_back(p);
    }
    void trim(size_t want) {
        size_t got = 0;
        for (auto& kv : free_) {
            while (!kv.second.empty() && got < want) {
                (void)hipFree(kv.second.back());
                kv.second.pop_back();
                reserved -= kv.first;
                got += kv.first;
            }
        }
    }
    void release() {
        for (auto& kv : free_)
            for (void* p : kv.second) (void)hipFree(p);
        free_.clear();
        reserved = 0;
    }
};

// Pinned host staging buffers (launch tables) by class, kept for reuse.
struct HostPool {
    std::map<size_t, std::vector<void*>> free_;
    void* get(size_t cls) {
        auto& v = free_[cls];
        if (!v.empty()) {
            void* p = v.back();
            v.pop_back();
            return p;
        }
        void* p = nullptr;
        if (hipHostMalloc(&p, cls, hipHostMallocDefault) != hipSuccess) return nullptr;
        return p;
    }
    void put(void* p, size_t cls) {
        if (p) free_[cls].push_back(p);
    }
    void release() {
        for (auto& kv : free_)
            for (void* p : kv.second) (void)hipHostFree(p);
        free_.clear();
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
    HostPool hpool;
    // the scheduler thread's own state (no lock)
    std::unordered_map<Key, KEntry, KeyHash> cache;
    std::list<Key> lru;  // front: most recently used
    std::vector<Batch*> inflight;
    int inflight_reqs = 0;
    size_t in_use = 0;
    size_t tables_seen = 0;  // context twiddle-table bytes already counted in in_use
    // shared with the caller's threads
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    apx_server_counters st{};
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

    apx_params kernel_params(const apx_request& r) const {
        apx_params prm{};
        prm.mode = r.mode;
        prm.core = APX_CORE_AUTO;
        prm.snr_min_db = isfinite(r.snr_min_db) ? r.snr_min_db : 0.0;
        prm.calib_db = NAN;
        return prm;
    }

    // Evict the least recently used kernel that no admitted request uses.  Runs on the
    // scheduler thread without the lock, so submitters and pollers are never held up by the
    // wait for the kernel's preparation or by its release.
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
            std::lock_guard<std::mutex> g(mu);
            st.evictions++;
            st.cached_kernels = (int32_t)cache.size();
            return true;
        }
        return false;
    }

    void complete(Req* q, int status) {
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

    // Release everything a batch holds (its stream has finished with it) and complete its
    // requests.
    void finish(Batch* b, int status) {
        for (Req* q : b->reqs) {
            pool.put(q->s_dev, q->s_cls);
            pool.put(q->o_dev, q->o_cls);
            pool.put(q->ws, q->ws_cls);
            in_use -= q->s_cls + q->o_cls + q->ws_cls + q->tab_share;
            in_use -= q->kern_plan;  // only a request whose kernel failed to appear still holds it
            if (b->ke && b->holds_refs) b->ke->refs--;
            inflight_reqs--;
            complete(q, status);
        }
        pool.put(b->tab_dev, b->tab_cls);
        hpool.put(b->tab_host, b->tab_cls);
        if (b->done) ev_free.push_back(b->done);
        delete b;
    }

    // Make sure the batch's kernel is resident (prepared on its stream on a miss).
    int ensure_kernel(Batch* b) {
        Req* q0 = b->reqs[0];
        const apx_request& r = q0->r;
        auto it = cache.find(q0->key);
        if (it != cache.end()) {
            b->ke = &it->second;
            b->holds_refs = true;  // taken at admission
            lru.splice(lru.begin(), lru, it->second.lru);
            std::lock_guard<std::mutex> g(mu);
            st.kernel_hits += (int64_t)b->reqs.size();
            return hipStreamWaitEvent(b->stream, it->second.ready, 0) == hipSuccess ? APX_OK : APX_E_DEVICE;
        }
        KEntry e;
        e.taps_cls = size_class((size_t)r.N * 4);
        e.taps = (float*)pool.get(e.taps_cls);
        if (!e.taps) return APX_E_NOMEM;
        const apx_params prm = kernel_params(r);
        apx_kernel k = nullptr;
        int rc = APX_E_DEVICE;
        if (hipMemcpyAsync(e.taps, r.k, (size_t)r.N * 4, hipMemcpyHostToDevice, b->stream) == hipSuccess)
            rc = apx_kernel_create(ctx, e.taps, r.N, r.op, q0->W_block, &prm, b->stream, &k);
        e.ready = event();
        if (rc == APX_OK && (!e.ready || hipEventRecord(e.ready, b->stream) != hipSuccess)) rc = APX_E_DEVICE;
        if (rc != APX_OK) {
            if (k) apx_kernel_destroy(k);
            if (e.ready) ev_free.push_back(e.ready);
            (void)hipStreamSynchronize(b->stream);
            pool.put(e.taps, e.taps_cls);
            return rc;
        }
        e.k = k;
        e.bytes = k->dev_bytes + e.taps_cls;
        // the admission reserved the planned bytes on every request that missed; the entry now
        // holds the kernel's actual bytes, plus any twiddle tables its preparation added
        for (Req* q : b->reqs) {
            in_use -= q->kern_plan;
            q->kern_plan = 0;
        }
        in_use += e.bytes;
        if (ctx->table_bytes > tables_seen) {
            in_use += ctx->table_bytes - tables_seen;
            tables_seen = ctx->table_bytes;
        }
        lru.push_front(q0->key);
        e.lru = lru.begin();
        e.refs = (int)b->reqs.size();
        it = cache.emplace(q0->key, e).first;
        b->ke = &it->second;
        b->holds_refs = true;
        std::lock_guard<std::mutex> g(mu);
        st.kernel_misses++;
        st.kernel_hits += (int64_t)b->reqs.size() - 1;
        st.cached_kernels = (int32_t)cache.size();
        return APX_OK;
    }

    // Enqueue a batch: copies in, per-request calibrations, one launch over every request's
    // blocks, copies out, completion event.
    int launch(Batch* b) {
        b->stream = streams[next_stream];
        next_stream = (next_stream + 1) % (int)streams.size();
        int rc = ensure_kernel(b);
        if (rc != APX_OK) return rc;
        apx_kernel k = b->ke->k;
        const hipStream_t s = b->stream;
        std::vector<apx::RunArgs> args;
        args.reserve(b->reqs.size());
        int64_t items = 0;
        for (Req* q : b->reqs) {
            const apx_request& r = q->r;
            q->core = k->core;
            q->s_dev = pool.get(q->s_cls);
            q->o_dev = pool.get(q->o_cls);
            q->ws = pool.get(q->ws_cls);
            if (!q->s_dev || !q->o_dev || !q->ws) return APX_E_NOMEM;
            if (hipMemcpyAsync(q->s_dev, r.s, (size_t)r.L * 4, hipMemcpyHostToDevice, s) != hipSuccess)
                return APX_E_DEVICE;
            apx::RunArgs a;
            rc = apx::run_args(k, (const float*)q->s_dev, r.L, (float*)q->o_dev, nullptr, &a);
            if (rc != APX_OK) return rc;
            if (r.mode == APX_AUTO_SNR) {
                const double* off = nullptr;
                a.snr_min_db = r.snr_min_db;
                rc = apx::calib_on_device(k, a, 0, q->ws, &off, s);
                if (rc != APX_OK) return rc;
                a.calib_dev = off;
            }
            a.item0 = items;
            items += a.nitems;
            args.push_back(a);
        }
        const size_t args_bytes = args.size() * sizeof(apx::RunArgs);
        const size_t bytes = args_bytes + (size_t)items * sizeof(int32_t);
        b->tab_cls = size_class(bytes);
        b->tab_dev = pool.get(b->tab_cls);
        b->tab_host = hpool.get(b->tab_cls);
        if (!b->tab_dev || !b->tab_host) return APX_E_NOMEM;
        memcpy(b->tab_host, args.data(), args_bytes);
        int32_t* sig = reinterpret_cast<int32_t*>((char*)b->tab_host + args_bytes);
        for (size_t i = 0; i < args.size(); ++i)
            for (int64_t j = 0; j < args[i].nitems; ++j) *sig++ = (int32_t)i;
        if (hipMemcpyAsync(b->tab_dev, b->tab_host, bytes, hipMemcpyHostToDevice, s) != hipSuccess) return APX_E_DEVICE;
        const apx::RunArgs* dargs = reinterpret_cast<const apx::RunArgs*>(b->tab_dev);
        const int32_t* dsig = reinterpret_cast<const int32_t*>((const char*)b->tab_dev + args_bytes);
        rc = apx::launch_many(k, args[0], dargs, dsig, items, s);
        if (rc != APX_OK) return rc;
        for (Req* q : b->reqs) {
            const apx_request& r = q->r;
            if (hipMemcpyAsync(r.r_out, q->o_dev, (size_t)(r.L + r.N - 1) * 4, hipMemcpyDeviceToHost, s) != hipSuccess)
                return APX_E_DEVICE;
        }
        b->done = event();
        if (!b->done || hipEventRecord(b->done, s) != hipSuccess) return APX_E_DEVICE;
        std::lock_guard<std::mutex> g(mu);
        st.launches++;
        return APX_OK;
    }

    // Bytes a queued request needs to be admitted; `planned` carries the kernels already
    // reserved by requests admitted earlier in the same tick.
    size_t need_of(Req* q, std::vector<Key>& planned, size_t* kern_plan) {
        const apx_request& r = q->r;
        size_t need = q->s_cls + q->o_cls + q->ws_cls + q->tab_share;
        *kern_plan = 0;
        if (cache.find(q->key) == cache.end() && std::find(planned.begin(), planned.end(), q->key) == planned.end()) {
            const apx_params prm = kernel_params(r);
            size_t kb = 0;
            if (apx::kernel_plan_bytes(ctx, r.N, r.op, q->W_block, &prm, &kb) != APX_OK) kb = 0;
            *kern_plan = kb + size_class((size_t)r.N * 4);
            need += *kern_plan;
        }
        return need;
    }

    void loop() {
        (void)hipSetDevice(ctx->device);
        for (;;) {
            // retire finished batches
            for (size_t i = 0; i < inflight.size();) {
                hipError_t e = hipEventQuery(inflight[i]->done);
                if (e == hipErrorNotReady) {
                    ++i;
                    continue;
                }
                Batch* b = inflight[i];
                inflight[i] = inflight.back();
                inflight.pop_back();
                finish(b, e == hipSuccess ? APX_OK : APX_E_DEVICE);
            }
            // admit in arrival order (only this thread pops the queue, so its front stays put
            // between the look and the pop)
            std::vector<Req*> adm;
            std::vector<Key> planned;
            for (;;) {
                Req* q = nullptr;
                {
                    std::lock_guard<std::mutex> g(mu);
                    if (queue.empty() || inflight_reqs + (int)adm.size() >= cfg.max_inflight) break;
                    q = queue.front();
                }
                size_t kplan = 0;
                size_t need = need_of(q, planned, &kplan);
                auto hit = cache.find(q->key);
                if (hit != cache.end()) hit->second.refs++;  // keep it from eviction below
                while (in_use + need > (size_t)cfg.hbm_budget && evict_one()) {
                }
                if (hit != cache.end()) hit->second.refs--;
                if (in_use + need > (size_t)cfg.hbm_budget) break;  // wait for memory
                {
                    std::lock_guard<std::mutex> g(mu);
                    queue.pop_front();
                }
                in_use += need;
                q->kern_plan = kplan;
                if (kplan) planned.push_back(q->key);
                q->t_admit = now_s();
                if (hit != cache.end()) hit->second.refs++;  // released when its batch retires
                adm.push_back(q);
                std::lock_guard<std::mutex> g(mu);
                st.peak_bytes = std::max<int64_t>(st.peak_bytes, (int64_t)in_use);
            }
            // one batch per prepared kernel, in order of first arrival
            std::vector<Batch*> batches;
            for (Req* q : adm) {
                Batch* b = nullptr;
                for (Batch* x : batches)
                    if (x->reqs[0]->key == q->key) b = x;
                if (!b) {
                    b = new Batch;
                    batches.push_back(b);
                }
                b->reqs.push_back(q);
            }
            for (Batch* b : batches) {
                inflight_reqs += (int)b->reqs.size();
                const int rc = launch(b);
                {
                    std::lock_guard<std::mutex> g(mu);
                    st.peak_bytes = std::max<int64_t>(st.peak_bytes, (int64_t)in_use);
                }
                if (rc != APX_OK) {
                    // work may be enqueued on the stream: let it end before the buffers go back
                    if (b->stream) (void)hipStreamSynchronize(b->stream);
                    finish(b, rc);
                    continue;
                }
                inflight.push_back(b);
            }
            std::unique_lock<std::mutex> lk(mu);
            if (stop && queue.empty() && inflight.empty()) break;
            if (inflight.empty()) {
                cv_work.wait(lk, [&] { return stop || !queue.empty(); });
            } else if (adm.empty()) {
                cv_work.wait_for(lk, std::chrono::microseconds(50));
            }
        }
    }
};

extern "C" {

apx_status apx_server_create(apx_ctx ctx, const apx_server_config* cfg, apx_server* out) {
    if (!out) return apx::set_error(APX_E_INVALID, "null output handle");
    *out = nullptr;
    if (!ctx || !cfg) return apx::set_error(APX_E_INVALID, "null argument");
    if (cfg->hbm_budget < (1 << 20) || cfg->n_streams < 1 || cfg->n_streams > 64 || cfg->max_inflight < 1)
        return apx::set_error(APX_E_INVALID, "server configuration out of range");
    if (hipSetDevice(ctx->device) != hipSuccess) return apx::set_error(APX_E_DEVICE, "hipSetDevice failed");
    apx_server srv = new (std::nothrow) apx_server_s;
    if (!srv) return apx::set_error(APX_E_NOMEM, "host allocation failed");
    srv->ctx = ctx;
    srv->cfg = *cfg;
    srv->pool.cap = (size_t)cfg->hbm_budget;
    srv->tables_seen = ctx->table_bytes;  // tables built before the server are not its memory
    for (int i = 0; i < cfg->n_streams; ++i) {
        hipStream_t s = nullptr;
        if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
            for (hipStream_t t : srv->streams) (void)hipStreamDestroy(t);
            delete srv;
            return apx::set_error(APX_E_DEVICE, "stream creation failed");
        }
        srv->streams.push_back(s);
    }
    srv->th = std::thread([srv] { srv->loop(); });
    *out = srv;
    return APX_OK;
}

double apx_server_now(void) { return now_s(); }

apx_status apx_server_submit(apx_server srv, const apx_request* r, uint64_t* ticket) {
    if (!srv || !r) return apx::set_error(APX_E_INVALID, "null argument");
    if (!r->s || !r->k || !r->r_out) return apx::set_error(APX_E_INVALID, "null buffer in the request");
    if (r->N < 1 || r->L < r->N)
        return apx::set_error(APX_E_INVALID, "request shape L = %lld, N = %d", (long long)r->L, r->N);
    if (reinterpret_cast<uintptr_t>(r->s) & 7) return apx::set_error(APX_E_INVALID, "s must be 8-byte aligned");
    if (r->op != APX_CONV && r->op != APX_XCORR) return apx::set_error(APX_E_INVALID, "unknown op %d", r->op);
    if (r->mode < APX_FULL_FP32 || r->mode > APX_FULL_FP64) return apx::set_error(APX_E_INVALID, "unknown mode %d", r->mode);
    if (r->mode == APX_AUTO_SNR && !isfinite(r->snr_min_db))
        return apx::set_error(APX_E_INVALID, "snr_min_db must be finite");
    const int32_t W_block = r->W_block > 0 ? r->W_block : server_block(r->N);
    if (apx_geometry(r->L, r->N, W_block, nullptr, nullptr, nullptr) != APX_OK)
        return apx::set_error(APX_E_INVALID, "block geometry: W_block = %d, N = %d", W_block, r->N);
    Req* q = new (std::nothrow) Req;
    if (!q) return apx::set_error(APX_E_NOMEM, "host allocation failed");
    q->r = *r;
    q->W_block = W_block;
    q->key = Key{r->kernel_key, r->N, r->op, W_block, r->mode};
    q->t_submit = now_s();
    q->s_cls = size_class((size_t)r->L * 4);
    q->o_cls = size_class((size_t)(r->L + r->N - 1) * 4);
    q->ws_cls = size_class(apx_workspace_bytes());
    // a launch table holds at least this request's share; its class at most doubles it (and is
    // at least one 4 KiB class)
    q->tab_share = std::max<size_t>(4096, 2 * table_share(r->L, r->N, W_block));
    {
        std::lock_guard<std::mutex> g(srv->mu);
        const size_t need = q->s_cls + q->o_cls + q->ws_cls + q->tab_share + size_class((size_t)r->N * 4);
        if (need > (size_t)srv->cfg.hbm_budget) {
            srv->st.rejected++;
            delete q;
            return apx::set_error(APX_E_NOMEM, "request needs %zu bytes, beyond the budget of %lld", need,
                                  (long long)srv->cfg.hbm_budget);
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
    if (!srv || !out || !n || max < 1) return apx::set_error(APX_E_INVALID, "null argument or max < 1");
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
    if (!srv) return apx::set_error(APX_E_INVALID, "null server");
    std::unique_lock<std::mutex> lk(srv->mu);
    srv->cv_done.wait(lk, [&] { return srv->outstanding == 0; });
    return APX_OK;
}

apx_status apx_server_stats(apx_server srv, apx_server_counters* out) {
    if (!srv || !out) return apx::set_error(APX_E_INVALID, "null argument");
    std::lock_guard<std::mutex> g(srv->mu);
    *out = srv->st;
    out->reserved_bytes = (int64_t)srv->pool.reserved.load();
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
    srv->hpool.release();
    for (hipStream_t s : srv->streams) (void)hipStreamDestroy(s);
    delete srv;
    return APX_OK;
}

}  // extern "C"
