// serve.cpp -- a serving engine for Triple-DES ECB requests with continuous batching.
//
// The paper encrypts one file with its whole data staged on the GPU (Listing
// 1.1); a server instead receives many requests of mixed sizes, each under one
// of many resident keys.  The engine keeps every key schedule on the device
// (one table upload), admits queued requests in arrival order while their
// input and output fit in a device-memory budget, and runs the admitted ones
// as one batched launch (batch.cpp) per step.  Several steps are in flight at
// once on their own streams, so requests that arrive while the GPU is busy are
// admitted into the next step as soon as a step slot and memory are free.
//
// Threads: an engine thread runs the loop below; submit, cancel, poll and
// release may be called from any thread (one mutex guards the queues).
//
// Engine loop:
//   1. retire steps whose completion event has fired: stamp the requests'
//      completion time, free their inputs (and outputs unless kept), and
//      queue their completion records;
//   2. if a step slot is idle, admit queued requests (first come, first
//      served; a request that does not fit blocks those behind it so large
//      requests are not starved), up to the per-step job and block limits;
//   3. launch the step: generate or copy the inputs, one batched cipher
//      launch, copy out host outputs, record the step's event.
//
// The steps' batch contexts launch the 120-VGPR variant of the batch kernel:
// beside its four waves per SIMD the payload fills of the next steps find
// registers to run in, instead of waiting for a batch kernel's workgroups to
// retire (the fills then no longer sit between two steps' ciphers).
#include <stdint.h>
#include <string.h>

#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "internal.h"

namespace {

constexpr uint64_t kAlign = 256;
constexpr uint32_t kMaxInflight = 8;

uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

// Best-fit allocator over one device range, with coalescing of free ranges.
class Pool {
  public:
    void init(uint64_t size) {
        size_ = size;
        by_off_.clear();
        by_size_.clear();
        insert(0, size);
        used_ = peak_ = 0;
    }
    bool alloc(uint64_t bytes, uint64_t *off) {
        bytes = round_up(bytes ? bytes : 1, kAlign);
        auto it = by_size_.lower_bound(bytes);
        if (it == by_size_.end()) return false;
        const uint64_t o = it->second, s = it->first;
        erase(o, s);
        if (s > bytes) insert(o + bytes, s - bytes);
        *off = o;
        used_ += bytes;
        if (used_ > peak_) peak_ = used_;
        return true;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = round_up(bytes ? bytes : 1, kAlign);
        used_ -= bytes;
        uint64_t o = off, s = bytes;
        auto next = by_off_.lower_bound(o);
        if (next != by_off_.end() && next->first == o + s) {
            s += next->second;
            erase(next->first, next->second);
        }
        auto prev = by_off_.lower_bound(o);
        if (prev != by_off_.begin()) {
            --prev;
            if (prev->first + prev->second == o) {
                o = prev->first;
                s += prev->second;
                erase(prev->first, prev->second);
            }
        }
        insert(o, s);
    }
    uint64_t used() const { return used_; }
    uint64_t peak() const { return peak_; }
    uint64_t size() const { return size_; }

  private:
    void insert(uint64_t o, uint64_t s) {
        by_off_[o] = s;
        by_size_.emplace(s, o);
    }
    void erase(uint64_t o, uint64_t s) {
        by_off_.erase(o);
        auto range = by_size_.equal_range(s);
        for (auto it = range.first; it != range.second; ++it)
            if (it->second == o) {
                by_size_.erase(it);
                break;
            }
    }
    uint64_t size_ = 0, used_ = 0, peak_ = 0;
    std::map<uint64_t, uint64_t> by_off_;
    std::multimap<uint64_t, uint64_t> by_size_;
};

struct Request {
    tdes_request r;
    double t_arrival = 0, t_admit = 0, t_launch = 0, t_done = 0;
    uint64_t in_off = 0, out_off = 0, bytes = 0;
    bool admitted = false, canceled = false, has_output = false;
};

struct Step {
    tdes_ctx *ctx = nullptr;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    std::vector<uint64_t> ids;
    std::vector<tdes_job> jobs;
    std::vector<tdes_request> rq;  // copies of the admitted requests, read without the lock
    std::vector<tdes::FillTile> fills;
    tdes::FillTile *h_fill = nullptr;  // pinned staging
    tdes::FillTile *d_fill = nullptr;
    size_t fill_cap = 0;
    hipEvent_t fill_staged = nullptr;  // the last fill-tile upload has read h_fill
};

}  // namespace

struct tdes_server {
    tdes_serve_config cfg{};
    const void *sched = nullptr;
    uint64_t n_scheds = 0;
    int device = 0;
    uint8_t *d_pool = nullptr;
    Pool pool;
    std::chrono::steady_clock::time_point epoch;

    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<uint64_t> pending;
    uint64_t pending_blocks = 0;  // blocks of the queued requests that are not canceled
    std::unordered_map<uint64_t, Request> reqs;
    std::deque<tdes_completion> completed;
    uint64_t next_id = 1;
    uint64_t outstanding = 0;  // submitted, not yet completed

    std::vector<Step> steps;
    std::thread engine;
    std::atomic<bool> stop{false};
    std::atomic<int> engine_error{TDES_OK};
    tdes_serve_stats stats{};

    double now() const {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - epoch).count();
    }
};

namespace {

void complete_locked(tdes_server *s, uint64_t id, Request &q, int status) {
    tdes_completion c{};
    c.id = id;
    c.user_tag = q.r.user_tag;
    c.status = status;
    c.t_arrival = q.t_arrival;
    c.t_admit = q.t_admit;
    c.t_launch = q.t_launch;
    c.t_complete = q.t_done;
    c.dev_out = (status == TDES_OK && q.has_output) ? s->d_pool + q.out_off : nullptr;
    s->completed.push_back(c);
    if (!q.has_output) s->reqs.erase(id);
    s->outstanding--;
    s->cv_done.notify_all();
}

// Retire finished steps.  Returns whether any step finished.
bool retire(tdes_server *s) {
    bool any = false;
    for (Step &st : s->steps) {
        if (!st.busy) continue;
        const hipError_t q = hipEventQuery(st.done);
        if (q == hipErrorNotReady) continue;
        if (q != hipSuccess) {
            s->engine_error = TDES_ERR_HIP;
            continue;
        }
        const double t = s->now();
        std::lock_guard<std::mutex> lk(s->mu);
        for (uint64_t id : st.ids) {
            Request &r = s->reqs[id];
            r.t_done = t;
            s->pool.release(r.in_off, r.bytes);
            const bool keep = s->cfg.keep_outputs && !r.r.host_out;
            if (!keep) s->pool.release(r.out_off, r.bytes);
            r.has_output = keep;
            s->stats.completed++;
            s->stats.bytes += r.bytes;
            complete_locked(s, id, r, TDES_OK);
        }
        st.ids.clear();
        st.busy = false;
        any = true;
    }
    if (any) s->cv_work.notify_all();
    return any;
}

// Admit queued requests into an idle step.  Returns the number admitted.
size_t admit(tdes_server *s, Step &st) {
    std::lock_guard<std::mutex> lk(s->mu);
    const double t = s->now();
    uint64_t blocks = 0;
    // A long queue is served in larger steps: up to its share per step in flight, within the backlog cap.
    uint64_t cap = s->cfg.max_step_blocks;
    if (s->cfg.backlog_step_blocks > cap) {
        const uint64_t share = s->pending_blocks / s->cfg.max_inflight;
        if (share > cap) cap = share < s->cfg.backlog_step_blocks ? share : s->cfg.backlog_step_blocks;
    }
    while (!s->pending.empty() && st.ids.size() < s->cfg.max_step_jobs) {
        const uint64_t id = s->pending.front();
        auto it = s->reqs.find(id);
        if (it == s->reqs.end() || it->second.canceled) {
            s->pending.pop_front();
            continue;
        }
        Request &r = it->second;
        if (!st.ids.empty() && blocks + r.r.n_blocks > cap) break;
        uint64_t in_off, out_off;
        if (!s->pool.alloc(r.bytes, &in_off)) break;  // first come, first served: wait for memory
        if (!s->pool.alloc(r.bytes, &out_off)) {
            s->pool.release(in_off, r.bytes);
            break;
        }
        s->pending.pop_front();
        s->pending_blocks -= r.r.n_blocks;
        r.in_off = in_off;
        r.out_off = out_off;
        r.admitted = true;
        r.t_admit = t;
        blocks += r.r.n_blocks;
        st.ids.push_back(id);
    }
    const uint64_t used = s->pool.used();
    if (used > s->stats.peak_pool_bytes) s->stats.peak_pool_bytes = used;
    return st.ids.size();
}

int ensure_fill_cap(Step &st, size_t n) {
    if (n <= st.fill_cap) return TDES_OK;
    if (st.fill_staged && hipEventSynchronize(st.fill_staged) != hipSuccess) return TDES_ERR_HIP;
    if (st.h_fill) (void)hipHostFree(st.h_fill);
    if (st.d_fill) (void)hipFree(st.d_fill);
    st.h_fill = nullptr;
    st.d_fill = nullptr;
    const size_t cap = n < 1024 ? 1024 : n * 2;
    if (hipHostMalloc(&st.h_fill, cap * sizeof(tdes::FillTile), hipHostMallocDefault) != hipSuccess) return TDES_ERR_NOMEM;
    if (hipMalloc(&st.d_fill, cap * sizeof(tdes::FillTile)) != hipSuccess) return TDES_ERR_NOMEM;
    st.fill_cap = cap;
    return TDES_OK;
}

// Generate or copy inputs, launch the batch, copy host outputs, record the event.
int launch_step(tdes_server *s, Step &st) {
    st.jobs.clear();
    st.rq.clear();
    st.fills.clear();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (uint64_t id : st.ids) {
            const Request &r = s->reqs[id];
            st.rq.push_back(r.r);
            tdes_job j{};
            j.in_off = r.in_off;
            j.out_off = r.out_off;
            j.n_blocks = r.r.n_blocks;
            j.sched_idx = r.r.key_id;
            j.direction = r.r.direction;
            st.jobs.push_back(j);
        }
    }
    // Inputs: host payloads are copied in; the others are generated from each request's seed.
    for (size_t i = 0; i < st.ids.size(); i++) {
        const tdes_request &rq = st.rq[i];
        const tdes_job &j = st.jobs[i];
        if (rq.host_in) {
            if (hipMemcpyAsync(s->d_pool + j.in_off, rq.host_in, j.n_blocks * 8, hipMemcpyHostToDevice, st.stream) !=
                hipSuccess)
                return TDES_ERR_HIP;
            continue;
        }
        for (uint64_t w = 0; w < j.n_blocks; w += tdes::kFillTileWords) {
            const uint64_t n = j.n_blocks - w < tdes::kFillTileWords ? j.n_blocks - w : tdes::kFillTileWords;
            st.fills.push_back({j.in_off + 8 * w, rq.seed, w, (uint32_t)n, 0});
        }
    }
    if (!st.fills.empty()) {
        int rc = ensure_fill_cap(st, st.fills.size());
        if (rc != TDES_OK) return rc;
        if (hipEventSynchronize(st.fill_staged) != hipSuccess) return TDES_ERR_HIP;
        memcpy(st.h_fill, st.fills.data(), st.fills.size() * sizeof(tdes::FillTile));
        if (hipMemcpyAsync(st.d_fill, st.h_fill, st.fills.size() * sizeof(tdes::FillTile), hipMemcpyHostToDevice,
                           st.stream) != hipSuccess ||
            hipEventRecord(st.fill_staged, st.stream) != hipSuccess ||
            tdes::launch_fill_tiles(st.d_fill, (uint32_t)st.fills.size(), s->d_pool, st.stream) != hipSuccess)
            return TDES_ERR_HIP;
    }
    int rc = tdes_ecb_batch(st.ctx, st.jobs.data(), (uint32_t)st.jobs.size(), s->sched, s->n_scheds, s->d_pool, 0,
                            st.stream);
    if (rc != TDES_OK) return rc;
    for (size_t i = 0; i < st.ids.size(); i++) {
        const tdes_request &rq = st.rq[i];
        if (rq.host_out &&
            hipMemcpyAsync(rq.host_out, s->d_pool + st.jobs[i].out_off, st.jobs[i].n_blocks * 8, hipMemcpyDeviceToHost,
                           st.stream) != hipSuccess)
            return TDES_ERR_HIP;
    }
    if (hipEventRecord(st.done, st.stream) != hipSuccess) return TDES_ERR_HIP;
    const double t = s->now();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (uint64_t id : st.ids) s->reqs[id].t_launch = t;
        s->stats.steps++;
        if (st.ids.size() > s->stats.max_step_jobs) s->stats.max_step_jobs = st.ids.size();
    }
    st.busy = true;
    return TDES_OK;
}

void engine_loop(tdes_server *s) {
    if (hipSetDevice(s->device) != hipSuccess) {
        s->engine_error = TDES_ERR_HIP;
        return;
    }
    while (!s->stop.load()) {
        bool progress = retire(s);
        for (Step &st : s->steps) {
            if (st.busy) continue;
            if (admit(s, st) == 0) break;
            const int rc = launch_step(s, st);
            if (rc != TDES_OK) {
                s->engine_error = rc;
                // Work already enqueued for this step may still touch its buffers.
                (void)hipStreamSynchronize(st.stream);
                // Fail the admitted requests rather than leave them pending.
                std::lock_guard<std::mutex> lk(s->mu);
                for (uint64_t id : st.ids) {
                    Request &r = s->reqs[id];
                    s->pool.release(r.in_off, r.bytes);
                    s->pool.release(r.out_off, r.bytes);
                    r.has_output = false;
                    r.t_done = s->now();
                    complete_locked(s, id, r, rc);
                }
                st.ids.clear();
                continue;
            }
            progress = true;
        }
        if (!progress) {
            bool busy = false;
            for (const Step &st : s->steps) busy |= st.busy;
            std::unique_lock<std::mutex> lk(s->mu);
            if (busy)
                s->cv_work.wait_for(lk, std::chrono::microseconds(20));  // poll the GPU events
            else if (s->pending.empty())
                s->cv_work.wait_for(lk, std::chrono::milliseconds(5), [s] { return s->stop.load() || !s->pending.empty(); });
        }
    }
}

void destroy_steps(tdes_server *s) {
    for (Step &st : s->steps) {
        if (st.stream) (void)hipStreamSynchronize(st.stream);
        if (st.ctx) tdes_ctx_destroy(st.ctx);
        if (st.done) (void)hipEventDestroy(st.done);
        if (st.fill_staged) (void)hipEventDestroy(st.fill_staged);
        if (st.h_fill) (void)hipHostFree(st.h_fill);
        if (st.d_fill) (void)hipFree(st.d_fill);
        if (st.stream) (void)hipStreamDestroy(st.stream);
    }
    s->steps.clear();
}

}  // namespace

extern "C" int tdes_server_create(tdes_server **out, const tdes_serve_config *cfg, const void *dev_sched_table,
                                  uint64_t n_scheds) {
    if (!out || !cfg || !dev_sched_table) return TDES_ERR_NULL;
    *out = nullptr;
    if (n_scheds == 0 || n_scheds > (1ull << 32) / (TDES_SCHED_BYTES / 4)) return TDES_ERR_SIZE;
    if (cfg->budget_bytes < 2 * kAlign || cfg->max_inflight == 0 || cfg->max_inflight > kMaxInflight ||
        cfg->max_step_jobs == 0 || cfg->max_step_blocks == 0)
        return TDES_ERR_ARG;
    // The batch tuning (tdes_ctx_set_tuning's ranges), checked before anything is allocated.
    if (cfg->threads && (cfg->threads > 256 || cfg->threads % 64 || cfg->groups_per_cu == 0 ||
                         cfg->groups_per_cu > 64 || cfg->wave_remainder > 2048 || cfg->tiles_per_draw > 16))
        return TDES_ERR_ARG;
    tdes_server *s = new (std::nothrow) tdes_server;
    if (!s) return TDES_ERR_NOMEM;
    s->cfg = *cfg;
    s->cfg.budget_bytes = round_up(cfg->budget_bytes, kAlign);
    s->sched = dev_sched_table;
    s->n_scheds = n_scheds;
    s->epoch = std::chrono::steady_clock::now();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return TDES_ERR_HIP;
    }
    if (hipMalloc(&s->d_pool, s->cfg.budget_bytes) != hipSuccess) {
        delete s;
        return TDES_ERR_NOMEM;
    }
    s->pool.init(s->cfg.budget_bytes);
    s->steps.resize(cfg->max_inflight);
    for (Step &st : s->steps) {
        if (tdes_ctx_create(&st.ctx, s->device) != TDES_OK ||
            (cfg->threads && tdes_ctx_set_tuning(st.ctx, cfg->threads, cfg->groups_per_cu, cfg->wave_remainder,
                                                 cfg->tiles_per_draw) != TDES_OK) ||
            hipStreamCreateWithFlags(&st.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&st.done, hipEventDisableTiming) != hipSuccess ||
            hipEventCreateWithFlags(&st.fill_staged, hipEventDisableTiming) != hipSuccess) {
            destroy_steps(s);
            (void)hipFree(s->d_pool);
            delete s;
            return TDES_ERR_HIP;
        }
        tdes::ctx_set_capped(st.ctx, true);
    }
    s->engine = std::thread(engine_loop, s);
    *out = s;
    return TDES_OK;
}

extern "C" int tdes_server_destroy(tdes_server *s) {
    if (!s) return TDES_OK;
    s->stop = true;
    s->cv_work.notify_all();
    if (s->engine.joinable()) s->engine.join();
    destroy_steps(s);
    if (s->d_pool) (void)hipFree(s->d_pool);
    delete s;
    return TDES_OK;
}

extern "C" double tdes_server_now(const tdes_server *s) { return s ? s->now() : 0.0; }

static int submit_at(tdes_server *s, const tdes_request *r, double t_arrival, uint64_t *id_out) {
    if (!s || !r) return TDES_ERR_NULL;
    if (r->direction != TDES_ENCRYPT && r->direction != TDES_DECRYPT) return TDES_ERR_ARG;
    if (r->key_id >= s->n_scheds) return TDES_ERR_SIZE;
    if (r->n_blocks == 0 || r->n_blocks > (1ull << 32)) return TDES_ERR_SIZE;
    const uint64_t bytes = r->n_blocks * 8;
    if (2 * round_up(bytes, kAlign) > s->cfg.budget_bytes) return TDES_ERR_BUDGET;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->engine_error != TDES_OK) return s->engine_error;
    const uint64_t id = s->next_id++;
    Request q;
    q.r = *r;
    q.t_arrival = t_arrival;
    q.bytes = bytes;
    s->reqs.emplace(id, q);
    s->pending.push_back(id);
    s->pending_blocks += r->n_blocks;
    s->outstanding++;
    s->stats.submitted++;
    if (id_out) *id_out = id;
    s->cv_work.notify_one();
    return TDES_OK;
}

extern "C" int tdes_server_submit(tdes_server *s, const tdes_request *r, uint64_t *id) {
    if (!s) return TDES_ERR_NULL;
    return submit_at(s, r, s->now(), id);
}

extern "C" int tdes_server_cancel(tdes_server *s, uint64_t id) {
    if (!s) return TDES_ERR_NULL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || it->second.admitted || it->second.canceled) return TDES_ERR_STATE;
    Request &r = it->second;
    r.canceled = true;
    s->pending_blocks -= r.r.n_blocks;
    r.t_done = s->now();
    s->stats.canceled++;
    complete_locked(s, id, r, TDES_ERR_STATE);
    return TDES_OK;
}

extern "C" int tdes_server_poll(tdes_server *s, tdes_completion *out, uint32_t max, uint32_t *n) {
    if (!s || !n || (max && !out)) return TDES_ERR_NULL;
    std::lock_guard<std::mutex> lk(s->mu);
    uint32_t k = 0;
    while (k < max && !s->completed.empty()) {
        out[k++] = s->completed.front();
        s->completed.pop_front();
    }
    *n = k;
    return s->engine_error;
}

extern "C" int tdes_server_wait_idle(tdes_server *s, double timeout_s) {
    if (!s) return TDES_ERR_NULL;
    std::unique_lock<std::mutex> lk(s->mu);
    const bool ok = s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s),
                                        [s] { return s->outstanding == 0 || s->engine_error != TDES_OK; });
    if (s->engine_error != TDES_OK) return s->engine_error;
    return ok ? TDES_OK : TDES_ERR_STATE;
}

extern "C" int tdes_server_release(tdes_server *s, uint64_t id) {
    if (!s) return TDES_ERR_NULL;
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || !it->second.has_output || it->second.t_done == 0) return TDES_ERR_STATE;
    s->pool.release(it->second.out_off, it->second.bytes);
    s->reqs.erase(it);
    s->cv_work.notify_all();
    return TDES_OK;
}

extern "C" int tdes_server_stats(tdes_server *s, tdes_serve_stats *out) {
    if (!s || !out) return TDES_ERR_NULL;
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    out->pool_bytes_in_use = s->pool.used();
    out->pending = s->pending.size();
    return s->engine_error;
}

extern "C" int tdes_server_run_trace(tdes_server *s, const tdes_request *reqs, const double *arrival, uint64_t n,
                                     tdes_completion *out) {
    if (!s || (n && (!reqs || !arrival || !out))) return TDES_ERR_NULL;
    for (uint64_t i = 1; i < n; i++)
        if (arrival[i] < arrival[i - 1]) return TDES_ERR_ARG;
    std::unordered_map<uint64_t, uint64_t> index;
    index.reserve(n * 2);
    std::vector<tdes_completion> buf(4096);
    uint64_t got = 0;
    auto drain = [&]() -> int {
        uint32_t k = 0;
        const int rc = tdes_server_poll(s, buf.data(), (uint32_t)buf.size(), &k);
        for (uint32_t i = 0; i < k; i++) {
            auto it = index.find(buf[i].id);
            if (it != index.end()) {
                out[it->second] = buf[i];
                got++;
            }
        }
        return rc;
    };
    const double t0 = s->now();
    for (uint64_t i = 0; i < n; i++) {
        const double due = t0 + arrival[i];
        // Open loop: wait for the arrival time, then submit with that arrival time.
        for (;;) {
            const double t = s->now();
            if (t >= due) break;
            if (due - t > 200e-6) std::this_thread::sleep_for(std::chrono::microseconds(50));
        }
        uint64_t id = 0;
        int rc = submit_at(s, &reqs[i], due, &id);
        if (rc != TDES_OK) {
            memset(&out[i], 0, sizeof out[i]);
            out[i].status = rc;
            out[i].t_arrival = due;
            got++;
            continue;
        }
        index[id] = i;
        if ((i & 63) == 0) {
            rc = drain();
            if (rc != TDES_OK) return rc;
        }
    }
    while (got < n) {
        const int rc = drain();
        if (rc != TDES_OK) return rc;
        if (got < n) {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_done.wait_for(lk, std::chrono::milliseconds(1));
        }
    }
    return TDES_OK;
}
