// Continuous-batching server.  A scheduler thread admits queued jobs while
// the device bytes of the admitted jobs stay within the budget and fewer than
// max_slots run, packs every admission round into one persistent launch on
// one of a few streams (so a new launch overlaps launches still running),
// and completes jobs as their launch's read-back event fires.  Device memory
// comes from one pool of the budget's size, allocated once.
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <list>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>

#include "batch_host.h"

namespace tn {

namespace {

double now_s() {
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit sub-allocator over one device block.
struct Pool {
    unsigned char* base = nullptr;
    uint64_t bytes = 0;
    uint64_t used = 0, peak = 0;         // bytes handed out now / at most
    std::map<uint64_t, uint64_t> free_;  // offset -> size
    void init(void* b, uint64_t n) {
        base = (unsigned char*)b;
        bytes = n;
        used = peak = 0;
        free_.clear();
        free_[0] = n;
    }
    void* alloc(uint64_t n) {
        n = (n + 255) & ~(uint64_t)255;
        for (auto it = free_.begin(); it != free_.end(); ++it)
            if (it->second >= n) {
                uint64_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > n) free_[off + n] = sz - n;
                used += n;
                peak = std::max(peak, used);
                return base + off;
            }
        return nullptr;
    }
    void release(void* p, uint64_t n) {
        n = (n + 255) & ~(uint64_t)255;
        used -= n;
        uint64_t off = (uint64_t)((unsigned char*)p - base);
        auto it = free_.emplace(off, n).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
};

}  // namespace

// Device bytes one job takes inside a persistent launch (all its passes).
uint64_t job_device_bytes(const Net& net, const Plan& plan, const tn_solve_opts& o) {
    std::vector<PassSpec> passes;
    if (make_passes(net, o, passes) != TN_OK) return 0;
    auto a = [](uint64_t x) { return (x + 255) & ~(uint64_t)255; };
    uint64_t total = a(sizeof(float) * net.wdev.size());
    for (auto& ps : passes) {
        uint64_t pb0 = plane_bytes(ps.dsr, 0), pb1 = plane_bytes(ps.dsr, 1);
        uint64_t E = (uint64_t)std::max<int64_t>(plan.arena_entries_dag, 64);
        uint64_t Pe = 0;  // every split node has its own partials in the dependency-graph executor
        for (auto& np : plan.prog) {
            GemmShape g = choose_gemm_shape(ps.dsr, np.lb, np.li, np.lj, np.lk, np.a_t, np.b_t, true);
            if (g.lsplit) Pe += ((1ull << (g.lsplit + np.lb + np.li + np.lj)) + 63) & ~63ull;
        }
        total += a(E * pb0) + a(E * pb1) + a(Pe * pb0) + a(Pe * pb1) + a(sizeof(TensorMeta) * plan.nodes.size()) + a(16);
    }
    return total;
}

}  // namespace tn

using namespace tn;

struct ServerJob {
    uint64_t id = 0;
    const Net* net = nullptr;
    const Plan* plan = nullptr;
    tn_solve_opts opts{};
    uint64_t bytes = 0;
    // a tree with much work runs alone on per-node launches over the whole
    // chip (a persistent launch keeps each job on one chiplet)
    bool large = false;
    DevProgram* dp = nullptr;
    std::vector<PassSpec> passes;
    SolveLayout layout;
    double t_submit = 0;
    int state = 0;  // 0 queued, 1 running, 2 done
    tn_result res{};
    tn_status st = TN_OK;
    double latency = 0;
};

struct InFlight {
    BatchLaunch L;
    std::vector<uint64_t> ids;
    hipEvent_t ev = nullptr;
    uint64_t bytes = 0;
    int stream = 0;
    // a large job's per-node launches: its buffer in the pool, pinned staging
    bool large = false;
    unsigned char* base = nullptr;
    void* stage = nullptr;
};

struct tn_server {
    tn_ctx* ctx = nullptr;
    uint64_t budget = 0;
    int max_slots = 0;
    std::mutex mu;   // jobs, queue, counters
    std::mutex dev;  // context (device programs, staging)
    std::condition_variable cv, done_cv;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, ServerJob> jobs;
    uint64_t next_id = 1;
    uint64_t admitted = 0;
    int running = 0;
    std::vector<hipStream_t> streams;
    int next_stream = 0;
    Pool pool;
    void* pool_mem = nullptr;
    uint64_t pool_bytes = 0;
    std::list<InFlight> inflight;
    std::thread th;
    bool stop = false;
    // after the pool could not hold an admission round: admit nothing more
    // until fewer launches than this are in flight (a completion frees memory)
    size_t blocked_at = 0;
    tn_server_stats_t stats{};
};

static const uint64_t kTableReserve = 64ull << 20;  // task tables of in-flight launches

static void complete(tn_server* s, InFlight& f) {
    std::vector<tn_result> res;
    std::vector<tn_status> sts;
    if (f.large) {
        tn_solve_opts o;
        std::vector<PassSpec> passes;
        SolveLayout L;
        {
            std::lock_guard<std::mutex> g(s->mu);  // the job table may rehash while submits come in
            const ServerJob& j = s->jobs[f.ids[0]];
            o = j.opts;
            passes = j.passes;
            L = j.layout;
        }
        std::vector<unsigned char> all((unsigned char*)f.stage, (unsigned char*)f.stage + L.acc_bytes);
        res.assign(1, tn_result{});
        sts.push_back(decode_root(o, passes, all, L.nent, 0, res[0]));
        std::lock_guard<std::mutex> g(s->dev);
        s->pool.release(f.base, L.need);
        pinned_release(s->ctx, f.stage);
    } else {
        batch_finish(f.L, res);
        for (auto& it : f.L.items) sts.push_back(it.status);
        std::lock_guard<std::mutex> g(s->dev);
        batch_release(f.L);
    }
    double t = now_s();
    std::lock_guard<std::mutex> g(s->mu);
    for (size_t k = 0; k < f.ids.size(); k++) {
        ServerJob& j = s->jobs[f.ids[k]];
        j.res = res[k];
        j.st = sts[k];
        j.res.seconds = t - j.t_submit;
        j.latency = t - j.t_submit;
        j.state = 2;
        s->stats.completed++;
        if (j.st != TN_OK) s->stats.failed++;
    }
    s->admitted -= f.bytes;
    s->running -= (int)f.ids.size();
    s->done_cv.notify_all();
}

static void scheduler(tn_server* s) {
    (void)hipSetDevice(s->ctx->device);
    for (;;) {
        // 1. complete launches whose read-back has landed
        for (auto it = s->inflight.begin(); it != s->inflight.end();) {
            if (hipEventQuery(it->ev) == hipSuccess) {
                complete(s, *it);
                (void)hipEventDestroy(it->ev);
                it = s->inflight.erase(it);
                std::lock_guard<std::mutex> g(s->mu);
                if (s->blocked_at && s->inflight.size() < s->blocked_at) s->blocked_at = 0;
            } else {
                ++it;
            }
        }
        // 2. admit: FIFO while the budget and the slots allow.  At most one
        // launch per stream is in flight: while all are busy, arrivals wait
        // in the queue and go out together in the next launch (one launch's
        // host work then serves many jobs when the device is saturated)
        std::vector<uint64_t> ids;
        uint64_t bytes = 0;
        {
            std::unique_lock<std::mutex> g(s->mu);
            if (s->stop && s->queue.empty() && s->inflight.empty()) break;
            const bool busy = s->inflight.size() >= s->streams.size() || s->blocked_at != 0;
            while (!busy && !s->queue.empty()) {
                ServerJob& j = s->jobs[s->queue.front()];
                if (s->running + (int)ids.size() >= s->max_slots) break;
                if (s->admitted + bytes + j.bytes > s->budget) break;
                if (j.large && !ids.empty()) break;  // a large job goes out alone
                bytes += j.bytes;
                ids.push_back(j.id);
                s->queue.pop_front();
                if (j.large) break;
            }
            if (ids.empty()) {
                // nothing admissible: sleep until a submit or a completion poll
                auto wait = s->inflight.empty() ? std::chrono::microseconds(2000) : std::chrono::microseconds(50);
                s->cv.wait_for(g, wait);
                continue;
            }
            s->admitted += bytes;
            s->running += (int)ids.size();
            if (s->admitted > s->stats.peak_admitted_bytes) s->stats.peak_admitted_bytes = s->admitted;
            if (s->running > s->stats.peak_running) s->stats.peak_running = s->running;
            for (auto id : ids) s->jobs[id].state = 1;
        }
        // 3. one persistent launch for this admission round (or a large job's
        // per-node launches)
        std::vector<BatchItem> items;
        ServerJob lj;  // a copy of the large job's launch data (the table may rehash)
        bool is_large = false;
        {
            std::lock_guard<std::mutex> g(s->mu);
            for (auto id : ids) {
                ServerJob& j = s->jobs[id];
                items.push_back({j.net, j.plan, j.opts});
                if (j.large) {
                    lj = j;
                    is_large = true;
                }
            }
        }
        InFlight f;
        f.ids = ids;
        f.bytes = bytes;
        f.large = is_large;
        DevAllocFn alloc;
        alloc.alloc = [s](size_t n) { return s->pool.alloc(n); };
        alloc.free = [s](void* p, size_t n) { s->pool.release(p, n); };
        tn_status st;
        // a stream with no launch in flight (one exists: admission above
        // stops while every stream is busy)
        int si = s->next_stream;
        for (int k = 0; k < (int)s->streams.size(); k++) {
            const int c = (s->next_stream + k) % (int)s->streams.size();
            bool used = false;
            for (const InFlight& o : s->inflight) used = used || o.stream == c;
            if (!used) {
                si = c;
                break;
            }
        }
        s->next_stream = (si + 1) % (int)s->streams.size();
        hipStream_t stream = s->streams[si];
        f.stream = si;
        {
            std::lock_guard<std::mutex> g(s->dev);
            if (is_large) {
                const SolveLayout& L = lj.layout;
                f.base = (unsigned char*)s->pool.alloc(L.need);
                f.stage = f.base ? pinned_acquire(s->ctx, std::max<size_t>(L.acc_bytes, sizeof(float) *
                                                                                         lj.net->wdev.size()) + 64)
                                 : nullptr;
                if (!f.base || !f.stage) {
                    if (f.base) s->pool.release(f.base, L.need);
                    f.base = nullptr;
                    st = TN_ENOMEM;
                } else {
                    st = run_solve_on(s->ctx, stream, true, *lj.net, *lj.plan, lj.opts, lj.passes, lj.dp, f.base, L,
                                      0, 1, f.stage, nullptr);
                }
            } else {
                st = batch_prepare(s->ctx, items, f.L, alloc);
                if (st == TN_OK) st = batch_launch(s->ctx, f.L, stream);
            }
        }
        if (st == TN_ENOMEM) {  // pool fragmented: requeue at the front, retry after completions
            std::lock_guard<std::mutex> g(s->dev);
            batch_release(f.L);
            std::lock_guard<std::mutex> g2(s->mu);
            for (auto it = ids.rbegin(); it != ids.rend(); ++it) {
                s->jobs[*it].state = 0;
                s->queue.push_front(*it);
            }
            s->admitted -= bytes;
            s->running -= (int)ids.size();
            s->stats.requeued += ids.size();
            if (!s->inflight.empty()) s->blocked_at = s->inflight.size();  // wait for a completion
            if (s->inflight.empty()) {  // nothing will free memory: fail the head job
                ServerJob& j = s->jobs[s->queue.front()];
                s->queue.pop_front();
                j.st = TN_ENOMEM;
                j.state = 2;
                j.res.semiring = -1;
                s->stats.completed++;
                s->stats.failed++;
                s->done_cv.notify_all();
            }
            continue;
        }
        if (st != TN_OK) {
            {
                std::lock_guard<std::mutex> g(s->dev);
                (void)hipStreamSynchronize(stream);
                batch_release(f.L);
                if (f.base) s->pool.release(f.base, lj.layout.need);
                if (f.stage) pinned_release(s->ctx, f.stage);
            }
            std::lock_guard<std::mutex> g(s->mu);
            for (auto id : ids) {
                ServerJob& j = s->jobs[id];
                j.st = st;
                j.state = 2;
                j.res.semiring = -1;
                s->stats.completed++;
                s->stats.failed++;
            }
            s->admitted -= bytes;
            s->running -= (int)ids.size();
            s->done_cv.notify_all();
            continue;
        }
        (void)hipEventCreateWithFlags(&f.ev, hipEventDisableTiming);
        (void)hipEventRecord(f.ev, stream);
        s->inflight.push_back(std::move(f));
        {
            std::lock_guard<std::mutex> g(s->mu);
            s->stats.launches++;
            s->stats.peak_inflight = std::max<int32_t>(s->stats.peak_inflight, (int32_t)s->inflight.size());
            s->stats.peak_pool_bytes = std::max<uint64_t>(s->stats.peak_pool_bytes, s->pool.peak);
        }
    }
}

extern "C" {

tn_status tn_server_create(tn_ctx* ctx, uint64_t budget, int32_t max_slots, tn_server** out) {
    try {
        if (!ctx || !out || budget == 0 || max_slots <= 0) return fail(TN_EINVAL, "invalid server arguments");
        *out = nullptr;
        auto* s = new tn_server();
        s->ctx = ctx;
        s->budget = budget;
        s->max_slots = max_slots;
        s->pool_bytes = budget + kTableReserve;
        s->pool_mem = dev_alloc(ctx, s->pool_bytes);
        if (!s->pool_mem) {
            delete s;
            return fail(TN_ENOMEM, "server pool allocation failed");
        }
        if (hipStreamSynchronize(ctx->stream) != hipSuccess) {
            dev_free(ctx, s->pool_mem, s->pool_bytes);
            delete s;
            return fail(TN_EDEVICE, "stream synchronisation failed");
        }
        s->pool.init(s->pool_mem, s->pool_bytes);
        for (int k = 0; k < 3; k++) {  // default-priority streams
            hipStream_t st;
            if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) break;
            s->streams.push_back(st);
        }
        if (s->streams.empty()) {
            dev_free(ctx, s->pool_mem, s->pool_bytes);
            delete s;
            return fail(TN_EDEVICE, "stream creation failed");
        }
        s->th = std::thread(scheduler, s);
        *out = s;
        return TN_OK;
    } catch (...) {
        return fail(TN_ENOMEM, "server creation failed");
    }
}

tn_status tn_server_submit(tn_server* s, const tn_net* net, const tn_plan* plan, const tn_solve_opts* o,
                           uint64_t* job_id) {
    try {
        if (!s || !net || !plan || !o || !job_id) return fail(TN_EINVAL, "NULL argument");
        if (plan->plan.fingerprint != net->net.fingerprint) return fail(TN_EINVAL, "plan was built for a different network");
        if (!plan->plan.sliced.empty()) return fail(TN_EINVAL, "served jobs must not be sliced");
        if (o->semiring < TN_TROPICAL_I32 || o->semiring > TN_PARTITION_BF16) return fail(TN_EINVAL, "unknown semiring");
        std::vector<PassSpec> passes;
        tn_status st = make_passes(net->net, *o, passes);
        if (st != TN_OK) return st;
        const bool large = !use_persistent_shared(plan->plan, o->semiring);
        DevProgram* dp = nullptr;
        SolveLayout layout;
        {
            // upload the plan's device program now, on the caller's thread
            std::lock_guard<std::mutex> g(s->dev);
            if (plan->plan.nleaf() > 0) {
                st = get_program(s->ctx, plan->plan, dp);
                if (st != TN_OK) return st;
                for (auto& ps : passes) node_launches(*dp, plan->plan, ps.dsr, !large);
            }
            if (large) layout = solve_layout(net->net, plan->plan, passes, dp, false);
        }
        uint64_t bytes = large ? layout.need : job_device_bytes(net->net, plan->plan, *o);
        if (bytes > s->budget) {
            std::lock_guard<std::mutex> g(s->mu);
            s->stats.rejected++;
            return fail(TN_ETOOBIG, "job needs " + std::to_string(bytes) + " device bytes, above the budget");
        }
        std::lock_guard<std::mutex> g(s->mu);
        if (s->stop) return fail(TN_ECANCELED, "server is shutting down");
        ServerJob j;
        j.id = s->next_id++;
        j.net = &net->net;
        j.plan = &plan->plan;
        j.opts = *o;
        j.opts.primes = nullptr;  // the default primes; caller arrays may not outlive the call
        if (o->primes) return fail(TN_EINVAL, "served jobs use the default primes");
        j.bytes = bytes;
        j.large = large;
        j.dp = dp;
        j.passes = passes;
        j.layout = layout;
        j.t_submit = now_s();
        s->jobs[j.id] = j;
        s->queue.push_back(j.id);
        s->stats.submitted++;
        *job_id = j.id;
        s->cv.notify_one();
        return TN_OK;
    } catch (...) {
        return fail(TN_ENOMEM, "submit failed");
    }
}

tn_status tn_server_poll(tn_server* s, uint64_t job_id, tn_result* out, int32_t* done, double* latency_s) {
    if (!s || !done) return fail(TN_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(TN_EINVAL, "unknown job id");
    *done = it->second.state == 2 ? 1 : 0;
    if (*done) {
        if (out) *out = it->second.res;
        if (latency_s) *latency_s = it->second.latency;
        tn_status st = it->second.st;
        s->jobs.erase(it);
        if (st == TN_ECANCELED) return fail(st, "job was cancelled");
        if (st != TN_OK) return fail(st, "job failed");
    }
    return TN_OK;
}

tn_status tn_server_job_bytes(const tn_net* net, const tn_plan* plan, const tn_solve_opts* o, uint64_t* bytes) {
    try {
        if (!net || !plan || !o || !bytes) return fail(TN_EINVAL, "NULL argument");
        std::vector<PassSpec> passes;
        tn_status st = make_passes(net->net, *o, passes);
        if (st != TN_OK) return st;
        if (use_persistent_shared(plan->plan, o->semiring)) {
            *bytes = job_device_bytes(net->net, plan->plan, *o);
        } else {
            DevProgram host_only;  // launch shapes only: nothing goes to the device
            *bytes = solve_layout(net->net, plan->plan, passes, plan->plan.nleaf() > 0 ? &host_only : nullptr, false).need;
        }
        return TN_OK;
    } catch (...) {
        return fail(TN_ENOMEM, "job size failed");
    }
}

tn_status tn_server_cancel(tn_server* s, uint64_t job_id) {
    if (!s) return fail(TN_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> g(s->mu);
    auto it = s->jobs.find(job_id);
    if (it == s->jobs.end()) return fail(TN_EINVAL, "unknown job id");
    ServerJob& j = it->second;
    if (j.state == 1) return fail(TN_EBUSY, "the job is already on the device");
    if (j.state == 2) return fail(TN_EINVAL, "the job has already finished");
    for (auto q = s->queue.begin(); q != s->queue.end(); ++q)
        if (*q == job_id) {
            s->queue.erase(q);
            break;
        }
    j.state = 2;
    j.st = TN_ECANCELED;
    j.res.semiring = -1;
    j.latency = now_s() - j.t_submit;
    s->stats.completed++;
    s->stats.canceled++;
    s->done_cv.notify_all();
    return TN_OK;
}

tn_status tn_server_drain(tn_server* s) {
    if (!s) return fail(TN_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> g(s->mu);
    s->done_cv.wait(g, [&] { return s->queue.empty() && s->running == 0; });
    return TN_OK;
}

tn_status tn_server_stats(tn_server* s, tn_server_stats_t* st) {
    if (!s || !st) return fail(TN_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> g(s->mu);
    *st = s->stats;
    return TN_OK;
}

tn_status tn_server_destroy(tn_server* s) {
    if (!s) return TN_OK;
    {
        std::lock_guard<std::mutex> g(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    if (s->th.joinable()) s->th.join();
    for (auto st : s->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    dev_free(s->ctx, s->pool_mem, s->pool_bytes);
    (void)hipStreamSynchronize(s->ctx->stream);
    delete s;
    return TN_OK;
}

}  // extern "C"
