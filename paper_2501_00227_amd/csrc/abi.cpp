// extern "C" entry points (include/tn.h).  No exception crosses this file:
// every call is wrapped and reports a tn_status plus a thread-local message.
#include <algorithm>
#include <cmath>
#include <atomic>
#include <new>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <mutex>
#include "batch_host.h"
#include "exec.h"

namespace tn {
const char* last_error_cstr();
}

using namespace tn;

#define TN_GUARD_BEGIN try {
#define TN_GUARD_END                                        \
    }                                                       \
    catch (const std::bad_alloc&) {                         \
        return fail(TN_ENOMEM, "host allocation failed");   \
    }                                                       \
    catch (const std::exception& e) {                       \
        return fail(TN_EINVAL, e.what());                   \
    }                                                       \
    catch (...) {                                           \
        return fail(TN_EINVAL, "unexpected internal error"); \
    }

static std::atomic<uint64_t> g_plan_uid{1};
static std::atomic<uint64_t> g_net_uid{1};

extern "C" {

const char* tn_last_error(void) { return last_error_cstr(); }

tn_status tn_ctx_create(int device, void* stream, const tn_allocator* alloc, tn_ctx** out) {
    TN_GUARD_BEGIN
    if (!out) return fail(TN_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0) return fail(TN_EDEVICE, "no HIP device available");
    if (device < 0 || device >= n) return fail(TN_EINVAL, "device id out of range");
    if (hipSetDevice(device) != hipSuccess) return fail(TN_EDEVICE, "hipSetDevice failed");
    noalloc_init_device(device);  // with the device current
    {
        tn_status ts = tune_env_load();  // TN_TUNE_FILE, once per process
        if (ts != TN_OK) return ts;
    }
    auto* c = new tn_ctx();
    c->device = device;
    if (alloc) {
        if (!alloc->alloc || !alloc->free) {
            delete c;
            return fail(TN_EINVAL, "allocator needs alloc and free");
        }
        c->alloc = *alloc;
        c->has_alloc = true;
    }
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail(TN_EDEVICE, "hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    *out = c;
    return TN_OK;
    TN_GUARD_END
}

void tn_ctx_destroy(tn_ctx* c) {
    if (!c) return;
    try {
        (void)hipSetDevice(c->device);
        (void)hipStreamSynchronize(c->stream);
        batch_cache_drop(c);
        for (auto& kv : c->progs)
            if (kv.second.wide_buf) dev_free(c, kv.second.wide_buf, kv.second.wide_bytes);
        for (auto& b : c->prog_bufs) dev_free(c, b.first, b.second);
        (void)hipStreamSynchronize(c->stream);
        for (auto& pr : c->pending) {
            (void)hipEventDestroy(pr.start);
            (void)hipEventDestroy(pr.stop);
        }
        for (auto e : c->event_pool) (void)hipEventDestroy(e);
        if (c->pinned) (void)hipHostFree(c->pinned);
        for (auto& b : c->pinned_pool) (void)hipHostFree(b.p);
        for (auto& b : c->batch_overflow) dev_free(c, b.first, b.second);
        if (c->batch_dev) dev_free(c, c->batch_dev, c->batch_dev_cap);
        (void)hipStreamSynchronize(c->stream);
        if (c->own_stream) (void)hipStreamDestroy(c->stream);
    } catch (...) {
    }
    delete c;
}

tn_status tn_ctx_set_profiling(tn_ctx* c, int enabled) {
    if (!c) return fail(TN_EINVAL, "ctx is NULL");
    c->profiling = enabled != 0;
    return TN_OK;
}

tn_status tn_ctx_synchronize(tn_ctx* c) {
    if (!c) return fail(TN_EINVAL, "ctx is NULL");
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(TN_EDEVICE, "hipStreamSynchronize failed");
    return TN_OK;
}

tn_status tn_ctx_profile(tn_ctx* c, tn_kernel_record* recs, int32_t cap, int32_t* n, int clear) {
    TN_GUARD_BEGIN
    if (!c || !n) return fail(TN_EINVAL, "ctx or n is NULL");
    if (hipStreamSynchronize(c->stream) != hipSuccess) return fail(TN_EDEVICE, "hipStreamSynchronize failed");
    for (auto& pr : c->pending) {
        float ms = 0;
        (void)hipEventElapsedTime(&ms, pr.start, pr.stop);
        pr.rec.ms = ms;
        c->records.push_back(pr.rec);
        c->event_pool.push_back(pr.start);
        c->event_pool.push_back(pr.stop);
    }
    c->pending.clear();
    *n = (int32_t)c->records.size();
    if (recs)
        for (int32_t k = 0; k < cap && k < *n; k++) recs[k] = c->records[k];
    if (clear) c->records.clear();
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_ctx_task_trace(tn_ctx* c, tn_task_record* recs, int32_t cap, int32_t* n, int clear) {
    TN_GUARD_BEGIN
    if (!c || !n) return fail(TN_EINVAL, "ctx or n is NULL");
    *n = (int32_t)c->task_trace.size();
    if (recs)
        for (int32_t k = 0; k < cap && k < *n; k++) recs[k] = c->task_trace[k];
    if (clear) c->task_trace.clear();
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_net_spin_glass(int32_t nv, int32_t ne, const int32_t* edges, const float* J, const float* h,
                            tn_net** out) {
    TN_GUARD_BEGIN
    if (!out) return fail(TN_EINVAL, "out is NULL");
    *out = nullptr;
    auto* n = new tn_net();
    tn_status st = make_spin_glass(nv, ne, edges, J, h, n->net);
    if (st != TN_OK) {
        delete n;
        return st;
    }
    n->net.uid = g_net_uid.fetch_add(1);
    *out = n;
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_net_independent_set(int32_t nv, int32_t ne, const int32_t* edges, const float* weights,
                                 tn_net** out) {
    TN_GUARD_BEGIN
    if (!out) return fail(TN_EINVAL, "out is NULL");
    *out = nullptr;
    auto* n = new tn_net();
    tn_status st = make_net(nv, ne, edges, weights, n->net);
    if (st != TN_OK) {
        delete n;
        return st;
    }
    n->net.uid = g_net_uid.fetch_add(1);
    *out = n;
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_net_condition(const tn_net* src, int32_t n, const int32_t* vertices, const int32_t* values,
                           tn_net** out) {
    TN_GUARD_BEGIN
    if (!src || !out) return fail(TN_EINVAL, "NULL argument");
    *out = nullptr;
    auto* c = new tn_net();
    tn_status st = condition_net(src->net, n, vertices, values, c->net);
    if (st != TN_OK) {
        delete c;
        return st;
    }
    c->net.uid = g_net_uid.fetch_add(1);
    *out = c;
    return TN_OK;
    TN_GUARD_END
}

void tn_net_destroy(tn_net* n) { delete n; }

tn_status tn_net_info(const tn_net* n, int32_t* nv, int32_t* ne) {
    if (!n) return fail(TN_EINVAL, "net is NULL");
    if (nv) *nv = n->net.nv;
    if (ne) *ne = (int32_t)n->net.edges.size();
    return TN_OK;
}

tn_status tn_net_flat_complexity(const tn_net* n, double* tc, double* sc, double* rwc) {
    if (!n) return fail(TN_EINVAL, "net is NULL");
    double a, b, c;
    flat_complexity(n->net, a, b, c);
    if (tc) *tc = a;
    if (sc) *sc = b;
    if (rwc) *rwc = c;
    return TN_OK;
}

void tn_plan_opts_default(tn_plan_opts* o) {
    if (!o) return;
    PlanOptions d;
    o->method = d.method;
    o->alpha = d.alpha;
    o->temperature = d.temperature;
    o->nrepeat = d.nrepeat;
    o->seed = d.seed;
    o->sc_target = d.sc_target;
    o->sc_weight = d.sc_weight;
    o->rw_weight = d.rw_weight;
    o->beta_start = d.beta_start;
    o->beta_step = d.beta_step;
    o->beta_stop = d.beta_stop;
    o->ntrials = d.ntrials;
    o->niters = d.niters;
    o->nslices = d.nslices;
    o->absorb_vertices = d.absorb ? 1 : 0;
    o->nthreads = d.nthreads;
    o->nopen = 0;
    o->open = nullptr;
}

static tn_status to_options(const tn_plan_opts* o, PlanOptions& p) {
    if (!o) return TN_OK;
    p.method = o->method;
    p.alpha = o->alpha;
    p.temperature = o->temperature;
    p.nrepeat = o->nrepeat;
    p.seed = o->seed;
    p.sc_target = o->sc_target;
    p.sc_weight = o->sc_weight;
    p.rw_weight = o->rw_weight;
    p.beta_start = o->beta_start;
    p.beta_step = o->beta_step;
    p.beta_stop = o->beta_stop;
    p.ntrials = o->ntrials;
    p.niters = o->niters;
    p.nslices = o->nslices;
    p.absorb = o->absorb_vertices != 0;
    p.nthreads = o->nthreads;
    if (o->nopen < 0 || o->nopen > kMaxOpen || (o->nopen > 0 && !o->open))
        return fail(TN_EINVAL, "nopen must be 0 .. 16, with open given");
    p.open.assign(o->open, o->open + o->nopen);
    if (p.method < 0 || p.method > 2) return fail(TN_EINVAL, "method must be 0 (greedy), 1 (TreeSA) or 2 (automatic)");
    if (p.temperature < 0 || p.nrepeat < 0 || p.ntrials < 0 || p.niters < 0 || p.nslices < 0)
        return fail(TN_EINVAL, "negative optimizer parameter");
    if (p.method != 0 && (p.beta_step <= 0 || p.beta_stop < p.beta_start))
        return fail(TN_EINVAL, "TreeSA needs beta_step > 0 and beta_stop >= beta_start");
    return TN_OK;
}

tn_status tn_plan_create(const tn_net* n, const tn_plan_opts* o, tn_plan** out) {
    TN_GUARD_BEGIN
    if (!n || !out) return fail(TN_EINVAL, "net or out is NULL");
    *out = nullptr;
    PlanOptions po;
    tn_status st = to_options(o, po);
    if (st != TN_OK) return st;
    auto* p = new tn_plan();
    st = plan_create(n->net, po, p->plan);
    if (st != TN_OK) {
        delete p;
        return st;
    }
    p->plan.uid = g_plan_uid.fetch_add(1);
    *out = p;
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_plan_from_tree(const tn_net* n, int32_t nleaf, const int32_t* fac_off, const int32_t* fac,
                            int32_t ninner, const int32_t* left, const int32_t* right, int32_t nsliced,
                            const int32_t* sliced, tn_plan** out) {
    TN_GUARD_BEGIN
    if (!n || !out || nleaf < 1 || ninner < 0 || nsliced < 0 || !fac_off || !fac)
        return fail(TN_EINVAL, "invalid tree arguments");
    *out = nullptr;
    std::vector<Leaf> leaves(nleaf);
    for (int l = 0; l < nleaf; l++) {
        if (fac_off[l + 1] < fac_off[l]) return fail(TN_EINVAL, "fac_off must be non-decreasing");
        for (int q = fac_off[l]; q < fac_off[l + 1]; q++) leaves[l].factors.push_back(fac[q]);
    }
    std::vector<int> L(left, left + ninner), R(right, right + ninner), S;
    if (nsliced) S.assign(sliced, sliced + nsliced);
    auto* p = new tn_plan();
    tn_status st = plan_from_tree(n->net, leaves, L, R, S, p->plan);
    if (st != TN_OK) {
        delete p;
        return st;
    }
    p->plan.uid = g_plan_uid.fetch_add(1);
    *out = p;
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_plan_complexity(const tn_plan* p, double* tc, double* sc, double* rwc) {
    if (!p) return fail(TN_EINVAL, "plan is NULL");
    if (tc) *tc = p->plan.tc;
    if (sc) *sc = p->plan.sc;
    if (rwc) *rwc = p->plan.rwc;
    return TN_OK;
}

tn_status tn_plan_info(const tn_plan* p, tn_plan_info_t* info) {
    if (!p || !info) return fail(TN_EINVAL, "plan or info is NULL");
    info->nleaf = p->plan.nleaf();
    info->ninner = p->plan.ninner();
    info->nsliced = (int32_t)p->plan.sliced.size();
    info->max_rank = p->plan.max_rank;
    info->tc_log2 = p->plan.tc;
    info->sc_log2 = p->plan.sc;
    info->rwc_log2 = p->plan.rwc;
    info->arena_entries = (uint64_t)p->plan.arena_entries;
    info->npermutes = p->plan.npermutes;
    return TN_OK;
}

tn_status tn_plan_gemm_shapes(const tn_plan* p, tn_semiring sr, int32_t cap, int32_t* rows, int32_t* nrows) {
    TN_GUARD_BEGIN
    if (!p || !nrows || cap < 0 || (cap > 0 && !rows)) return fail(TN_EINVAL, "invalid arguments");
    std::vector<int> dsrs;
    switch (sr) {
    case TN_TROPICAL_I32: dsrs = {DSR_TROP_I32}; break;
    case TN_TROPICAL_F32: dsrs = {DSR_TROP_F32}; break;
    case TN_COUNTING_TROPICAL: dsrs = {DSR_CTROP}; break;
    case TN_COUNT_EXACT: dsrs = {DSR_MODP}; break;
    case TN_PARTITION_F32: dsrs = {DSR_Z_F32}; break;
    case TN_PARTITION_BF16: dsrs = {DSR_Z_BF16}; break;
    default: return fail(TN_EINVAL, "unknown semiring");
    }
    const Plan& pl = p->plan;
    int32_t n = 0;
    for (size_t a = 0; a < dsrs.size(); a++)
        for (const NodeProg& np : pl.prog) {
            GemmShape g = choose_gemm_shape(dsrs[a], np.lb, np.li, np.lj, np.lk, np.a_t, np.b_t);
            const int kind = g.mode == GEMM_THIN  ? TN_K_GEMM_THIN
                             : g.mode == GEMM_DOT ? TN_K_GEMM_DOT
                             : g.mfma             ? TN_K_GEMM_MFMA
                             : g.rm == 8          ? TN_K_GEMM_BIG
                                                  : TN_K_GEMM;
            const int32_t row[TN_SHAPE_ROW] = {(int32_t)a, np.node, g.lb, g.li, g.lj, g.lk, g.a_t, g.b_t, g.tb,
                                               g.ti, g.tj, g.tk, g.rm, g.rn, g.lsplit, kind,
                                               gemm_shape_valid(dsrs[a], g) ? 1 : 0, 0};
            if (n < cap) std::memcpy(rows + (size_t)n * TN_SHAPE_ROW, row, sizeof row);
            n++;
        }
    *nrows = n;
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_plan_peak_bytes(const tn_plan* p, tn_semiring sr, uint64_t* bytes) {
    TN_GUARD_BEGIN
    if (!p || !bytes) return fail(TN_EINVAL, "plan or bytes is NULL");
    int dsr;
    switch (sr) {
    case TN_TROPICAL_I32: dsr = DSR_TROP_I32; break;
    case TN_TROPICAL_F32: dsr = DSR_TROP_F32; break;
    case TN_COUNTING_TROPICAL: dsr = DSR_CTROP; break;
    case TN_COUNT_EXACT: dsr = DSR_MODP; break;
    case TN_PARTITION_F32: dsr = DSR_Z_F32; break;
    case TN_PARTITION_BF16: dsr = DSR_Z_BF16; break;
    default: return fail(TN_EINVAL, "unknown semiring");
    }
    const Plan& pl = p->plan;
    uint64_t eb = (uint64_t)plane_bytes(dsr, 0) + (uint64_t)plane_bytes(dsr, 1);
    const bool dag = use_persistent(pl);  // the dependency-graph executor keeps every partial separate
    uint64_t part = 0;
    for (auto& np : pl.prog) {
        GemmShape g = choose_gemm_shape(dsr, np.lb, np.li, np.lj, np.lk, np.a_t, np.b_t, dag);
        if (!g.lsplit) continue;
        uint64_t n = 1ull << (g.lsplit + np.lb + np.li + np.lj);
        part = dag ? part + ((n + 63) & ~63ull) : std::max<uint64_t>(part, n);
    }
    uint64_t e = (uint64_t)std::max<int64_t>(dag ? pl.arena_entries_dag : pl.arena_entries, 64);
    *bytes = (e + part) * eb + sizeof(TensorMeta) * pl.nodes.size() + 4ull * pl.nv + 4096 + 8192;
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_plan_export(const tn_plan* pp, int32_t* nleaf, int32_t* ninner, int32_t* nfac, int32_t* nidx,
                         int32_t* nsliced, int32_t* fac_off, int32_t* fac, int32_t* left, int32_t* right,
                         int32_t* idx_off, int32_t* idx, int32_t* sliced) {
    TN_GUARD_BEGIN
    if (!pp) return fail(TN_EINVAL, "plan is NULL");
    const Plan& p = pp->plan;
    int nl = p.nleaf(), ni = p.ninner();
    int nf = 0, nx = 0;
    for (auto& l : p.leaves) nf += (int)l.factors.size();
    for (auto& n : p.nodes) nx += (int)n.out.size();
    if (nleaf) *nleaf = nl;
    if (ninner) *ninner = ni;
    if (nfac) *nfac = nf;
    if (nidx) *nidx = nx;
    if (nsliced) *nsliced = (int32_t)p.sliced.size();
    if (fac_off && fac) {
        int q = 0;
        for (int l = 0; l < nl; l++) {
            fac_off[l] = q;
            for (int f : p.leaves[l].factors) fac[q++] = f;
        }
        fac_off[nl] = q;
    }
    if (left && right)
        for (int t = 0; t < ni; t++) {
            left[t] = p.nodes[nl + t].left;
            right[t] = p.nodes[nl + t].right;
        }
    if (idx_off && idx) {
        int q = 0;
        for (size_t x = 0; x < p.nodes.size(); x++) {
            idx_off[x] = q;
            for (int v : p.nodes[x].out) idx[q++] = v;
        }
        idx_off[p.nodes.size()] = q;
    }
    if (sliced)
        for (size_t k = 0; k < p.sliced.size(); k++) sliced[k] = p.sliced[k];
    return TN_OK;
    TN_GUARD_END
}

void tn_plan_destroy(tn_plan* p) { delete p; }

void tn_solve_opts_default(tn_solve_opts* o) {
    if (!o) return;
    o->semiring = TN_TROPICAL_I32;
    o->beta = 0.0;
    o->nprimes = 0;
    o->primes = nullptr;
    o->slice_begin = 0;
    o->slice_end = 0;
    o->executor = 0;
}

static bool public_semiring(int s) { return s >= TN_TROPICAL_I32 && s <= TN_PARTITION_BF16; }

// TN_LOG=<path>: one JSON line per tn_solve appended to the file: the plan's
// complexity, the slice range, the executor, the status, the result's key
// values and the call's wall time (the variable is read at every call).
static void log_solve(const tn_plan* p, const tn_solve_opts& o, bool persistent, tn_status st, const tn_result& r) {
    const char* path = std::getenv("TN_LOG");
    if (!path || !*path) return;
    static std::mutex mu;
    std::lock_guard<std::mutex> lock(mu);
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f,
                 "{\"call\": \"tn_solve\", \"status\": %d, \"semiring\": %d, \"executor\": \"%s\", "
                 "\"tc_log2\": %.4f, \"sc_log2\": %.4f, \"rwc_log2\": %.4f, \"nsliced\": %d, "
                 "\"slice_begin\": %lld, \"slice_end\": %lld",
                 (int)st, (int)o.semiring, persistent ? "persistent" : "per-node", p->plan.tc, p->plan.sc, p->plan.rwc,
                 (int)p->plan.sliced.size(), (long long)o.slice_begin, (long long)o.slice_end);
    if (st == TN_OK) {
        std::fprintf(f, ", \"seconds\": %.6g", r.seconds);
        switch (o.semiring) {
        case TN_TROPICAL_I32: std::fprintf(f, ", \"size\": %d", r.size_i32); break;
        case TN_TROPICAL_F32: std::fprintf(f, ", \"size\": %.9g", (double)r.size_f32); break;
        case TN_COUNTING_TROPICAL:
            std::fprintf(f, ", \"size\": %d, \"count_mod_2_64\": %llu", r.size_i32,
                         (unsigned long long)r.count_mod_2_64);
            break;
        case TN_COUNT_EXACT:
            std::fprintf(f, ", \"count_mod_2_64\": %llu, \"count_limbs\": %d", (unsigned long long)r.count_mod_2_64,
                         r.count_nlimbs);
            break;
        case TN_PARTITION_F32:
        case TN_PARTITION_BF16:
            std::fprintf(f, ", \"log_z\": %.17g, \"z_range_log2\": %.6g", r.log_z, r.z_range_log2);
            break;
        default: break;
        }
    }
    std::fprintf(f, "}\n");
    std::fclose(f);
}

tn_status tn_result_combine(const tn_result* a, const tn_result* b, tn_result* out) {
    TN_GUARD_BEGIN
    if (!a || !b || !out) return fail(TN_EINVAL, "NULL argument");
    tn_result r;
    tn_status st = combine_results(*a, *b, r);
    if (st == TN_OK) *out = r;
    return st;
    TN_GUARD_END
}

tn_status tn_solve(tn_ctx* c, const tn_net* n, const tn_plan* p, const tn_solve_opts* o, tn_result* out) {
    TN_GUARD_BEGIN
    if (!c || !n || !p || !o || !out) return fail(TN_EINVAL, "NULL argument");
    if (!public_semiring(o->semiring)) return fail(TN_EINVAL, "unknown semiring");
    if (hipSetDevice(c->device) != hipSuccess) return fail(TN_EDEVICE, "hipSetDevice failed");
    if (o->executor < 0 || o->executor > 2) return fail(TN_EINVAL, "executor must be 0, 1 or 2");
    bool persistent = o->executor == 2 || (o->executor == 0 && use_persistent(p->plan));
    if (o->executor == 2 && (!p->plan.sliced.empty() || o->slice_begin || o->slice_end))
        return fail(TN_EINVAL, "the persistent executor runs unsliced plans only");
    tn_status st;
    if (persistent && o->slice_begin == 0 && o->slice_end == 0) {
        std::vector<BatchItem> items{{&n->net, &p->plan, *o}};
        std::vector<tn_result> res;
        st = solve_batch_sync(c, items, res);
        if (!res.empty()) *out = res[0];
    } else {
        persistent = false;
        st = solve_one(c, n->net, p->plan, *o, *out);
    }
    log_solve(p, *o, persistent, st, *out);
    return st;
    TN_GUARD_END
}

tn_status tn_ctx_set_wait_limit(tn_ctx* c, double seconds) {
    TN_GUARD_BEGIN
    if (!c || !(seconds > 0) || !std::isfinite(seconds)) return fail(TN_EINVAL, "the wait limit must be a positive time");
    c->wait_limit_s = seconds;
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_tune_plan(tn_ctx* c, const tn_plan* p, int32_t semiring, double min_log2_ops, int32_t reps,
                       int32_t* ntuned) {
    TN_GUARD_BEGIN
    if (!c || !p) return fail(TN_EINVAL, "NULL argument");
    if (!public_semiring(semiring)) return fail(TN_EINVAL, "unknown semiring");
    if (hipSetDevice(c->device) != hipSuccess) return fail(TN_EDEVICE, "hipSetDevice failed");
    tn_net dummy;  // make_passes reads only the network's weights and kind
    dummy.net.integer_weights = true;
    tn_solve_opts o;
    tn_solve_opts_default(&o);
    o.semiring = semiring;
    o.nprimes = 2;
    std::vector<PassSpec> passes;
    tn_status st = make_passes(dummy.net, o, passes);
    if (st != TN_OK) return st;
    std::vector<int> dsrs;
    for (auto& ps : passes)
        if (std::find(dsrs.begin(), dsrs.end(), ps.dsr) == dsrs.end()) dsrs.push_back(ps.dsr);
    return tune_plan(c, p->plan, dsrs, min_log2_ops, reps, ntuned);
    TN_GUARD_END
}

tn_status tn_tune_save(const char* path, int32_t* nentries) {
    TN_GUARD_BEGIN
    if (!path) return fail(TN_EINVAL, "NULL path");
    return tune_save(path, nentries);
    TN_GUARD_END
}

tn_status tn_tune_load(const char* path, int32_t* nentries) {
    TN_GUARD_BEGIN
    if (!path) return fail(TN_EINVAL, "NULL path");
    return tune_load(path, nentries);
    TN_GUARD_END
}

void tn_tune_clear(void) {
    try {
        tune_clear();
    } catch (...) {
    }
}

tn_status tn_tune_records(tn_tune_record* recs, int32_t cap, int32_t* n) {
    TN_GUARD_BEGIN
    if (!n || cap < 0 || (cap > 0 && !recs)) return fail(TN_EINVAL, "bad arguments");
    *n = tune_records(recs, cap);
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_solve_noalloc(tn_ctx* c, const tn_net* n, const tn_plan* p, const tn_solve_opts* o, tn_result* out) {
    TN_GUARD_BEGIN
    if (!c || !n || !p || !o || !out) return fail(TN_EINVAL, "NULL argument");
    if (!public_semiring(o->semiring)) return fail(TN_EINVAL, "unknown semiring");
    if (o->executor != 0 && o->executor != 1) return fail(TN_EINVAL, "the scratch-free solve runs per-node launches only");
    if (hipSetDevice(c->device) != hipSuccess) return fail(TN_EDEVICE, "hipSetDevice failed");
    auto t0 = std::chrono::steady_clock::now();
    tn_status st = solve_noalloc(c, n->net, p->plan, *o, *out);
    out->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return st;
    TN_GUARD_END
}

tn_status tn_solve_batch(tn_ctx* c, int32_t n, const tn_net* const* nets, const tn_plan* const* plans,
                         const tn_solve_opts* opts, tn_result* out) {
    TN_GUARD_BEGIN
    if (!c || n < 0 || (n > 0 && (!nets || !plans || !opts || !out))) return fail(TN_EINVAL, "NULL argument");
    if (hipSetDevice(c->device) != hipSuccess) return fail(TN_EDEVICE, "hipSetDevice failed");
    // jobs with much work run one after the other on per-node launches over
    // the whole chip (a persistent launch keeps a job on one chiplet); the
    // rest share one persistent launch (use_persistent_shared: the small trees
    // of tn_solve's rule, and mid-size trees of the exact algebras, whose
    // results do not depend on the route).
    std::vector<BatchItem> items;
    std::vector<int32_t> in_batch, alone;
    for (int32_t i = 0; i < n; i++) {
        if (!nets[i] || !plans[i]) return fail(TN_EINVAL, "NULL network or plan in the batch");
        if (!public_semiring(opts[i].semiring)) return fail(TN_EINVAL, "unknown semiring");
        const Plan& pl = plans[i]->plan;
        const bool per_node = pl.sliced.empty() && opts[i].slice_begin == 0 && opts[i].slice_end == 0 &&
                              (opts[i].executor == 1 ||
                               (opts[i].executor == 0 && !use_persistent_shared(pl, opts[i].semiring)));
        if (per_node) {
            alone.push_back(i);
        } else {
            in_batch.push_back(i);
            items.push_back({&nets[i]->net, &pl, opts[i]});
        }
    }
    tn_status st = TN_OK;
    if (!items.empty()) {
        std::vector<tn_result> res;
        st = solve_batch_sync(c, items, res);
        for (size_t k = 0; k < in_batch.size() && k < res.size(); k++) out[in_batch[k]] = res[k];
    }
    for (int32_t i : alone) {
        tn_status s2 = solve_one(c, nets[i]->net, plans[i]->plan, opts[i], out[i]);
        if (s2 != TN_OK) {
            out[i].semiring = -1;
            if (st == TN_OK) st = s2;
        }
    }
    return st;
    TN_GUARD_END
}

tn_status tn_solve_max_k(tn_ctx* c, const tn_net* n, const tn_plan* p, int32_t k, int32_t* sizes, int32_t limbs,
                         uint32_t* counts) {
    TN_GUARD_BEGIN
    if (!c || !n || !p || !sizes || k < 1 || k > 64 || (counts && limbs < 1))
        return fail(TN_EINVAL, "invalid arguments (k in 1..64, sizes required, limbs >= 1 with counts)");
    if (p->plan.fingerprint != n->net.fingerprint || p->plan.nv != n->net.nv)
        return fail(TN_EINVAL, "plan was built for a different network");
    if (hipSetDevice(c->device) != hipSuccess) return fail(TN_EDEVICE, "hipSetDevice failed");
    const int nv = n->net.nv, L = nv / 32 + 2;
    std::vector<uint32_t> poly((size_t)(nv + 1) * L);
    int deg = 0;
    tn_status st = solve_polynomial(c, n->net, p->plan, L, poly.data(), &deg);
    if (st != TN_OK) return st;
    auto coeff_small = [&](int s) -> uint64_t {  // saturating: only compared with k <= 64
        if (s < 0 || s > deg) return 0;
        for (int l = 2; l < L; l++)
            if (poly[(size_t)s * L + l]) return ~0ull;
        return (uint64_t)poly[(size_t)s * L] | ((uint64_t)poly[(size_t)s * L + 1] << 32);
    };
    int filled = 0;
    for (int s = deg; s >= 0 && filled < k; s--)
        for (uint64_t m = coeff_small(s); m > 0 && filled < k; m--) sizes[filled++] = s;
    for (; filled < k; filled++) sizes[filled] = INT32_MIN;
    if (counts) {
        std::memset(counts, 0, sizeof(uint32_t) * (size_t)k * limbs);
        for (int d = 0; d < k; d++) {
            const int s = deg - d;
            if (s < 0) break;
            int used = L;
            while (used > 0 && !poly[(size_t)s * L + used - 1]) used--;
            if (used > limbs) return fail(TN_EOVERFLOW, "a count needs more limbs than given");
            for (int l = 0; l < used; l++) counts[(size_t)d * limbs + l] = poly[(size_t)s * L + l];
        }
    }
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_solve_open(tn_ctx* c, const tn_net* n, const tn_plan* p, const tn_solve_opts* o, int64_t cap,
                        tn_result* out) {
    TN_GUARD_BEGIN
    if (!c || !n || !p || !o || !out) return fail(TN_EINVAL, "NULL argument");
    if (!public_semiring(o->semiring)) return fail(TN_EINVAL, "unknown semiring");
    const int64_t need = (int64_t)1 << p->plan.open.size();
    if (cap < need) return fail(TN_EINVAL, "out must hold 2^nopen results");
    if (o->executor == 2) return fail(TN_EINVAL, "open plans run on the stream executor");
    if (hipSetDevice(c->device) != hipSuccess) return fail(TN_EDEVICE, "hipSetDevice failed");
    std::vector<tn_result> t;
    tn_result first;
    tn_status st = solve_one(c, n->net, p->plan, *o, first, &t);
    if (st == TN_OK)
        for (int64_t e = 0; e < need; e++) out[e] = t[(size_t)e];
    return st;
    TN_GUARD_END
}

tn_status tn_solve_size_max_k(tn_ctx* c, const tn_net* n, const tn_plan* p, int32_t k, int32_t executor,
                              float* sizes) {
    TN_GUARD_BEGIN
    if (!c || !n || !p || !sizes || k < 1 || k > 8) return fail(TN_EINVAL, "invalid arguments (k in 1..8, sizes required)");
    if (executor < 0 || executor > 2) return fail(TN_EINVAL, "executor must be 0, 1 or 2");
    if (executor == 2 && !p->plan.sliced.empty())
        return fail(TN_EINVAL, "the persistent executor runs unsliced plans only");
    if (p->plan.fingerprint != n->net.fingerprint || p->plan.nv != n->net.nv)
        return fail(TN_EINVAL, "plan was built for a different network");
    if (hipSetDevice(c->device) != hipSuccess) return fail(TN_EDEVICE, "hipSetDevice failed");
    if (p->plan.nleaf() == 0) {  // the empty network: one configuration of value 0
        sizes[0] = 0.0f;
        for (int t = 1; t < k; t++) sizes[t] = -INFINITY;
        return TN_OK;
    }
    float top[8];
    // auto: one persistent launch only for small trees.  A persistent launch
    // keeps a job on one chiplet (an eighth of the CUs); an eight-list op
    // costs some twenty 4-byte ops, so larger trees fill the whole chip
    // better through per-node launches.
    const bool small = p->plan.sliced.empty() && p->plan.max_rank <= 14;
    if (executor == 2 || (executor == 0 && small)) {
        if (!p->plan.open.empty()) return fail(TN_EINVAL, "the plan has open vertices");
        std::vector<PassSpec> passes(1);
        passes[0].dsr = DSR_TOPK;
        std::vector<std::array<unsigned char, kAccSlotBytes>> accs;
        tn_status st = run_passes_sync(c, n->net, p->plan, passes, accs);
        if (st != TN_OK) return st;
        std::memcpy(top, accs[0].data(), sizeof top);
    } else {
        tn_solve_opts o;
        tn_solve_opts_default(&o);
        o.semiring = kSemiringTop8;
        o.executor = 1;
        tn_result r;
        std::vector<unsigned char> raw;
        tn_status st = solve_one(c, n->net, p->plan, o, r, nullptr, &raw);
        if (st != TN_OK) return st;
        std::memcpy(top, raw.data(), sizeof top);
    }
    std::memcpy(sizes, top, sizeof(float) * (size_t)k);
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_solve_counting_max_k(tn_ctx* c, const tn_net* n, const tn_plan* p, int32_t k, int32_t executor,
                                  int32_t* top, uint64_t* counts) {
    TN_GUARD_BEGIN
    if (!c || !n || !p || !top || !counts || k < 1 || k > 4)
        return fail(TN_EINVAL, "invalid arguments (k in 1..4, top and counts required)");
    if (executor < 0 || executor > 2) return fail(TN_EINVAL, "executor must be 0, 1 or 2");
    if (executor == 2 && !p->plan.sliced.empty())
        return fail(TN_EINVAL, "the persistent executor runs unsliced plans only");
    if (p->plan.fingerprint != n->net.fingerprint || p->plan.nv != n->net.nv)
        return fail(TN_EINVAL, "plan was built for a different network");
    if (hipSetDevice(c->device) != hipSuccess) return fail(TN_EDEVICE, "hipSetDevice failed");
    if (p->plan.nleaf() == 0) {  // the empty network: one configuration of value 0
        *top = 0;
        counts[0] = 1;
        for (int d = 1; d < k; d++) counts[d] = 0;
        return TN_OK;
    }
    std::vector<unsigned char> raw;
    // auto: one persistent launch for small trees only (as for SizeMax(k))
    const bool small = p->plan.sliced.empty() && p->plan.max_rank <= 14;
    if (executor == 2 || (executor == 0 && small)) {
        if (!p->plan.open.empty()) return fail(TN_EINVAL, "the plan has open vertices");
        if (!n->net.integer_weights) return fail(TN_EINVAL, "CountingMax(k) needs integer weights (|w| <= 65536)");
        std::vector<PassSpec> passes(1);
        passes[0].dsr = DSR_TPOLY;
        std::vector<std::array<unsigned char, kAccSlotBytes>> accs;
        tn_status st = run_passes_sync(c, n->net, p->plan, passes, accs);
        if (st != TN_OK) return st;
        raw.assign(accs[0].begin(), accs[0].end());
    } else {
        tn_solve_opts o;
        tn_solve_opts_default(&o);
        o.semiring = kSemiringTPoly4;
        o.executor = 1;
        tn_result r;
        tn_status st = solve_one(c, n->net, p->plan, o, r, nullptr, &raw);
        if (st != TN_OK) return st;
    }
    int32_t m;
    uint64_t cnt[4];
    std::memcpy(&m, raw.data(), 4);
    std::memcpy(cnt, raw.data() + 8, sizeof cnt);
    const bool none = m <= -(1 << 30);  // no configuration at all
    *top = none ? INT32_MIN : m;
    for (int d = 0; d < k; d++) counts[d] = none ? 0 : cnt[d];
    return TN_OK;
    TN_GUARD_END
}

tn_status tn_solve_single_config_max(tn_ctx* c, const tn_net* n, const tn_plan* p, int32_t* config, float* value) {
    TN_GUARD_BEGIN
    if (!c || !n || !p) return fail(TN_EINVAL, "NULL argument");
    if (hipSetDevice(c->device) != hipSuccess) return fail(TN_EDEVICE, "hipSetDevice failed");
    return single_config_max(c, n->net, p->plan, config, value);
    TN_GUARD_END
}

tn_status tn_solve_polynomial(tn_ctx* c, const tn_net* n, const tn_plan* p, int32_t limbs, uint32_t* coeffs,
                              int32_t* degree) {
    TN_GUARD_BEGIN
    if (!c || !n || !p) return fail(TN_EINVAL, "NULL argument");
    if (p->plan.fingerprint != n->net.fingerprint || p->plan.nv != n->net.nv)
        return fail(TN_EINVAL, "plan was built for a different network");
    if (hipSetDevice(c->device) != hipSuccess) return fail(TN_EDEVICE, "hipSetDevice failed");
    int deg = 0;
    tn_status st = solve_polynomial(c, n->net, p->plan, limbs, coeffs, &deg);
    if (degree) *degree = st == TN_OK ? deg : 0;
    return st;
    TN_GUARD_END
}

}  // extern "C"
