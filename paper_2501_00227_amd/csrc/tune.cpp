// Autotuner of GEMM launch shapes.
//
// A launch shape (kernel family, tile, K step, K splits) is chosen per node
// shape: (device algebra, log2 batch / M / N / K, operand orders).  The
// table below maps such keys to the shape measured fastest on the device;
// keys not in the table use the fixed heuristic (heuristic_gemm_shape).  As
// the key holds nothing but the node's own shape, a job gets the same shapes
// alone and in any batch, so its results do not depend on the mix.
//
// Tuning a key: every candidate shape the kernels accept (the register-tiled
// tiles and K steps, counting-tropical tiles, matrix-core tiles for the real
// algebra, LDS-staged tiles of several output shapes, thin / long-K modes,
// K splits) runs on seeded operands of the node's full size; a candidate
// whose result differs from the heuristic shape's (bit patterns for the exact
// algebras, 1e-4 relative for the real ones: float32 sums of up to 2^12
// positive terms in another order stay well inside it, a wrong result does
// not) is rejected, the others are
// timed with HIP events (best of `reps` launches, split reduction included)
// and the fastest is kept.  Tables are saved to and loaded from a text file
// (TN_TUNE_FILE is loaded at the first context creation).
#include <algorithm>
#include <cerrno>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <tuple>

#include "batch_host.h"
#include "exec.h"

namespace tn {

namespace {

struct TuneKey {
    int dsr, lb, li, lj, lk, a_t, b_t;
    bool operator<(const TuneKey& o) const {
        return std::tie(dsr, lb, li, lj, lk, a_t, b_t) < std::tie(o.dsr, o.lb, o.li, o.lj, o.lk, o.a_t, o.b_t);
    }
};

std::mutex g_mu;
std::map<TuneKey, GemmShape> g_table;
std::vector<tn_tune_record> g_records;
uint64_t g_generation = 1;
bool g_env_done = false;

constexpr size_t kTileLdsCap = 40 * 1024;  // what one persistent-kernel task may stage
constexpr int kMaxLogBlocks = 23;          // grid of at most 2^23 workgroups of 256 threads

int log_blocks(const GemmShape& g) { return (g.lb - g.tb) + (g.li - g.ti) + (g.lj - g.tj) + g.lsplit; }

bool same_shape(const GemmShape& a, const GemmShape& b) {
    return a.mode == b.mode && a.tb == b.tb && a.ti == b.ti && a.tj == b.tj && a.tk == b.tk && a.rm == b.rm &&
           a.rn == b.rn && a.lsplit == b.lsplit && a.mfma == b.mfma;
}

// A table entry (or candidate) the kernels accept for this key.
bool usable(int dsr, const GemmShape& g) {
    return gemm_shape_valid(dsr, g) && gemm_lds_bytes(dsr, g) <= kTileLdsCap && log_blocks(g) <= kMaxLogBlocks;
}

}  // namespace

uint64_t tune_generation() {
    std::lock_guard<std::mutex> l(g_mu);
    return g_generation;
}

GemmShape choose_gemm_shape(int dsr, int lb, int li, int lj, int lk, int a_t, int b_t, bool chiplet) {
    if (chiplet) return heuristic_gemm_shape(dsr, lb, li, lj, lk, a_t, b_t, false);
    {
        std::lock_guard<std::mutex> l(g_mu);
        auto it = g_table.find(TuneKey{dsr, lb, li, lj, lk, a_t, b_t});
        if (it != g_table.end()) return it->second;
    }
    return heuristic_gemm_shape(dsr, lb, li, lj, lk, a_t, b_t);
}

const char* gemm_kernel_name(int dsr, const GemmShape& g, char* buf, size_t cap) {
    if (g.mode == GEMM_THIN) snprintf(buf, cap, "gemm_thin_kernel<%d>", dsr);
    else if (g.mode == GEMM_DOT) snprintf(buf, cap, "gemm_dot_kernel<%d>", dsr);
    else if (g.mfma == 2) snprintf(buf, cap, "gemm_mfma128_kernel<%d>", dsr);
    else if (g.mfma) snprintf(buf, cap, "gemm_mfma_kernel<%d>", dsr);
    else if (g.rm == 8 && dsr == DSR_CTROP)
        snprintf(buf, cap, "gemm_ct_big_kernel<%d, %d, %s>", g.ti, g.tj, ct_ahead_shape(g.ti, g.tj, g.tk) ? "true" : "false");
    else if (g.rm == 8) snprintf(buf, cap, "gemm_big_kernel<%d, %d, %d>", dsr, g.ti, g.tj);
    else snprintf(buf, cap, "gemm_kernel<%d, %d, %d>", dsr, g.rm, g.rn);
    return buf;
}

// Candidate launch shapes of one node shape, the heuristic's first (at most
// kMaxCandidates).  K splits only where the output tiles are too few to
// fill the chip; LDS-staged small tiles only where the heuristic did not
// pick a register-tiled or matrix-core family (those win on large nodes).
constexpr size_t kMaxCandidates = 32;

std::vector<GemmShape> tune_candidates(int dsr, int lb, int li, int lj, int lk, int a_t, int b_t) {
    std::vector<GemmShape> out;
    auto push = [&](GemmShape g) {
        g.lb = lb, g.li = li, g.lj = lj, g.lk = lk, g.a_t = a_t, g.b_t = b_t;
        if (out.size() >= kMaxCandidates || !usable(dsr, g)) return;
        if (!out.empty() && g.lsplit > 0 && (g.lb - g.tb) + (g.li - g.ti) + (g.lj - g.tj) >= 10) return;
        for (const GemmShape& h : out)
            if (same_shape(h, g)) return;
        out.push_back(g);
    };
    const GemmShape h = heuristic_gemm_shape(dsr, lb, li, lj, lk, a_t, b_t);
    push(h);
    if (dsr == DSR_TOPK || dsr == DSR_TPOLY) return out;  // wide entries: one family only
    const int lsplits[] = {0, 1, 2, 3, 4};
    if (h.mode == GEMM_DOT) {
        for (int ls = 0; ls <= 10; ls++) {
            GemmShape g = h;
            g.lsplit = ls;
            push(g);
        }
        return out;
    }
    if (h.mode == GEMM_THIN)
        for (int ti = 10; ti <= 14; ti++) {
            GemmShape g = h;
            g.ti = ti;
            push(g);
        }
    // register-tiled families (8 x 8 / 8 x 4 per thread)
    const int big[][2] = {{7, 7}, {7, 6}, {6, 7}, {8, 6}, {8, 5}, {6, 8}, {5, 8}};
    for (auto& t : big)
        for (int tk = 2; tk <= 5; tk++)
            for (int ls : lsplits) {
                GemmShape g{};
                g.mode = GEMM_TILED;
                g.rm = g.rn = 8;
                g.ti = t[0];
                g.tj = t[1];
                g.tk = tk;
                g.lsplit = ls;
                push(g);
            }
    // matrix cores (real algebra): 128 x 128 tiles, then 64 x 64
    if (dsr == DSR_Z_F32 || dsr == DSR_Z_BF16)
        for (int ls : lsplits) {
            GemmShape g{};
            g.mode = GEMM_TILED;
            g.mfma = 2;
            g.rm = g.rn = 4;
            g.ti = g.tj = 7;
            g.tk = dsr == DSR_Z_BF16 ? 5 : 4;
            g.lsplit = ls;
            push(g);
        }
    if (dsr == DSR_Z_F32 || dsr == DSR_Z_BF16)
        for (int tk = 1; tk <= 5; tk++)
            for (int ls : lsplits) {
                GemmShape g{};
                g.mode = GEMM_TILED;
                g.mfma = 1;
                g.rm = g.rn = 4;
                g.ti = g.tj = 6;
                g.tk = tk;
                g.lsplit = ls;
                push(g);
            }
    // LDS-staged tiles: 256 threads of RM x RN outputs over 2^tb x 2^ti x 2^tj
    if (h.rm == 8 || h.mfma) return out;
    const int rr[][2] = {{1, 1}, {1, 2}, {2, 1}, {2, 2}, {4, 4}};
    for (auto& r : rr) {
        const int lr = (r[0] == 4 ? 2 : r[0] - 1) + (r[1] == 4 ? 2 : r[1] - 1);
        for (int ti = 0; ti <= std::min(li, 7); ti++)
            for (int tj = 0; tj <= std::min(lj, 7); tj++) {
                const int tb = 8 + lr - ti - tj;  // 256 threads when the batch allows
                if (tb < 0 || tb > lb) continue;
                for (int dk = 0; dk < 3; dk++)
                    for (int ls : {0, h.lsplit}) {
                        GemmShape g{};
                        g.mode = GEMM_TILED;
                        g.rm = r[0];
                        g.rn = r[1];
                        g.tb = tb;
                        g.ti = ti;
                        g.tj = tj;
                        g.tk = std::max(0, std::min(lk - ls, 5) - dk);
                        g.lsplit = ls;
                        push(g);
                    }
            }
    }
    return out;
}

namespace {

// Device buffers of one tuning run (allocated through the context).
struct TuneBufs {
    tn_ctx* ctx;
    std::vector<std::pair<void*, size_t>> owned;
    void* get(size_t bytes) {
        void* p = dev_alloc(ctx, bytes);
        if (p) owned.push_back({p, std::max<size_t>(bytes, 256)});
        return p;
    }
    ~TuneBufs() {
        for (auto& o : owned) dev_free(ctx, o.first, o.second);
    }
};

Planes planes_of(TuneBufs& b, int dsr, int64_t n, bool& ok) {
    Planes p;
    const int b0 = plane_bytes(dsr, 0), b1 = plane_bytes(dsr, 1);
    p.p0 = b.get((size_t)n * b0);
    p.p1 = b1 ? b.get((size_t)n * b1) : nullptr;
    ok = ok && p.p0 && (!b1 || p.p1);
    return p;
}

}  // namespace

// Tune one key on the device: returns the winner in *best and a record.
static tn_status tune_key(tn_ctx* ctx, const TuneKey& k, int reps, GemmShape* best, tn_tune_record* rec) {
    const std::vector<GemmShape> cands = tune_candidates(k.dsr, k.lb, k.li, k.lj, k.lk, k.a_t, k.b_t);
    std::memset(rec, 0, sizeof *rec);
    rec->dsr = k.dsr;
    rec->lb = k.lb, rec->li = k.li, rec->lj = k.lj, rec->lk = k.lk, rec->a_t = k.a_t, rec->b_t = k.b_t;
    rec->ncand = (int32_t)cands.size();
    *best = cands[0];
    hipStream_t s = ctx->stream;
    const int64_t na = (int64_t)1 << (k.lb + k.li + k.lk), nb = (int64_t)1 << (k.lb + k.lk + k.lj),
                  nc = (int64_t)1 << (k.lb + k.li + k.lj);
    int64_t npart = 0;
    for (const GemmShape& g : cands)
        if (g.lsplit) npart = std::max(npart, nc << g.lsplit);
    TuneBufs bufs{ctx, {}};
    bool ok = true;
    Planes A = planes_of(bufs, k.dsr, na, ok), B = planes_of(bufs, k.dsr, nb, ok), C = planes_of(bufs, k.dsr, nc, ok),
           R = planes_of(bufs, k.dsr, nc, ok), P = planes_of(bufs, k.dsr, std::max<int64_t>(npart, 1), ok);
    TensorMeta* meta = (TensorMeta*)bufs.get(sizeof(TensorMeta) * 3);
    unsigned long long* bad = (unsigned long long*)bufs.get(sizeof(unsigned long long));
    if (!ok || !meta || !bad) return fail(TN_ENOMEM, "device allocation for tuning failed");
    const AlgebraParams ap = algebra_params(k.dsr, 1073741789u, 0.0);
    hipError_t e = hipSuccess;
    auto chk = [&](hipError_t x) {
        if (x != hipSuccess && e == hipSuccess) e = x;
    };
    chk(launch_fill_tune(k.dsr, A, na, 0x5eed0001ull, ap.p, s));
    chk(launch_fill_tune(k.dsr, B, nb, 0x5eed0002ull, ap.p, s));
    auto run = [&](const GemmShape& g, Planes out) {
        chk(launch_meta_init(meta, 3, s));
        chk(launch_gemm(k.dsr, A, B, out, P, g, ap, meta, 0, 1, 2, s));
        if (g.lsplit > 0) chk(launch_split_reduce(k.dsr, P, out, nc, g.lsplit, ap, meta, 2, s));
    };
    hipEvent_t t0, t1;
    chk(hipEventCreate(&t0));
    chk(hipEventCreate(&t1));
    run(cands[0], R);  // the reference result
    float best_ms = 1e30f;
    for (size_t c = 0; c < cands.size() && e == hipSuccess; c++) {
        const GemmShape& g = cands[c];
        chk(hipMemsetAsync(bad, 0, sizeof *bad, s));
        run(g, C);
        chk(launch_compare_tune(k.dsr, C, R, nc, 1e-4f, bad, s));
        unsigned long long nbad = 0;
        chk(hipMemcpyAsync(&nbad, bad, sizeof nbad, hipMemcpyDeviceToHost, s));
        chk(hipStreamSynchronize(s));
        if (e != hipSuccess) break;
        if (nbad) {
            rec->nrejected++;
            continue;
        }
        float ms = 1e30f;
        for (int r = 0; r < std::max(1, reps); r++) {
            chk(hipEventRecord(t0, s));
            run(g, C);
            chk(hipEventRecord(t1, s));
            chk(hipEventSynchronize(t1));
            float x = 0;
            chk(hipEventElapsedTime(&x, t0, t1));
            ms = std::min(ms, x);
        }
        if (c == 0) rec->heuristic_ms = ms;
        if (ms < best_ms) {
            best_ms = ms;
            *best = g;
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    if (e != hipSuccess) return fail(TN_EDEVICE, std::string("tuning launch failed: ") + hipGetErrorString(e));
    rec->best_ms = best_ms;
    const GemmShape& b = *best;
    const int32_t shape[10] = {b.mode, b.tb, b.ti, b.tj, b.tk, b.rm, b.rn, b.lsplit, b.mfma, 0};
    std::memcpy(rec->shape, shape, sizeof shape);
    return TN_OK;
}

tn_status tune_plan(tn_ctx* ctx, const Plan& plan, const std::vector<int>& dsrs, double min_log2_ops, int reps,
                    int32_t* ntuned) {
    std::vector<TuneKey> keys;
    for (int dsr : dsrs)
        for (const NodeProg& np : plan.prog) {
            if (np.lb + np.li + np.lj + np.lk < min_log2_ops) continue;
            TuneKey k{dsr, np.lb, np.li, np.lj, np.lk, np.a_t ? 1 : 0, np.b_t ? 1 : 0};
            bool seen = false;
            {
                std::lock_guard<std::mutex> l(g_mu);
                seen = g_table.count(k) > 0;
            }
            for (const TuneKey& q : keys) seen = seen || (!(q < k) && !(k < q));
            if (!seen) keys.push_back(k);
        }
    int32_t n = 0;
    for (const TuneKey& k : keys) {
        GemmShape best;
        tn_tune_record rec;
        tn_status st = tune_key(ctx, k, reps, &best, &rec);
        if (st != TN_OK) return st;
        std::lock_guard<std::mutex> l(g_mu);
        g_table[k] = best;
        g_records.push_back(rec);
        g_generation++;
        n++;
    }
    if (ntuned) *ntuned = n;
    batch_cache_drop(ctx);  // its task table holds the shapes it was built with
    return TN_OK;
}

// ----------------------------------------------------------- table file --
static const char* kHeader = "# tn GEMM launch-shape table v1: dsr lb li lj lk a_t b_t : mode tb ti tj tk rm rn lsplit mfma";

tn_status tune_save(const char* path, int32_t* nentries) {
    FILE* f = fopen(path, "w");
    if (!f) return fail(TN_EINVAL, std::string("cannot write ") + path + ": " + strerror(errno));
    std::lock_guard<std::mutex> l(g_mu);
    fprintf(f, "%s\n", kHeader);
    for (auto& kv : g_table) {
        const TuneKey& k = kv.first;
        const GemmShape& g = kv.second;
        fprintf(f, "%d %d %d %d %d %d %d : %d %d %d %d %d %d %d %d %d\n", k.dsr, k.lb, k.li, k.lj, k.lk, k.a_t, k.b_t,
                g.mode, g.tb, g.ti, g.tj, g.tk, g.rm, g.rn, g.lsplit, g.mfma);
    }
    const bool bad = ferror(f) != 0;
    fclose(f);
    if (bad) return fail(TN_EINVAL, std::string("write error on ") + path);
    if (nentries) *nentries = (int32_t)g_table.size();
    return TN_OK;
}

tn_status tune_load(const char* path, int32_t* nentries) {
    FILE* f = fopen(path, "r");
    if (!f) return fail(TN_EINVAL, std::string("cannot read ") + path + ": " + strerror(errno));
    std::map<TuneKey, GemmShape> add;
    char line[512];
    int lineno = 0;
    tn_status st = TN_OK;
    while (fgets(line, sizeof line, f)) {
        lineno++;
        if (line[0] == '#' || line[0] == '\n') continue;
        TuneKey k;
        GemmShape g{};
        const int got = sscanf(line, "%d %d %d %d %d %d %d : %d %d %d %d %d %d %d %d %d", &k.dsr, &k.lb, &k.li, &k.lj,
                               &k.lk, &k.a_t, &k.b_t, &g.mode, &g.tb, &g.ti, &g.tj, &g.tk, &g.rm, &g.rn, &g.lsplit,
                               &g.mfma);
        g.lb = k.lb, g.li = k.li, g.lj = k.lj, g.lk = k.lk, g.a_t = k.a_t, g.b_t = k.b_t;
        if (got != 16 || k.dsr < 0 || k.dsr >= DSR_COUNT_ || !usable(k.dsr, g)) {
            st = fail(TN_EINVAL, std::string(path) + ":" + std::to_string(lineno) + ": not a usable table entry");
            break;
        }
        add[k] = g;
    }
    fclose(f);
    if (st != TN_OK) return st;  // nothing of a bad file is taken
    std::lock_guard<std::mutex> l(g_mu);
    for (auto& kv : add) g_table[kv.first] = kv.second;
    g_generation++;
    if (nentries) *nentries = (int32_t)g_table.size();
    return TN_OK;
}

void tune_clear() {
    std::lock_guard<std::mutex> l(g_mu);
    g_table.clear();
    g_records.clear();
    g_generation++;
}

int32_t tune_records(tn_tune_record* recs, int32_t cap) {
    std::lock_guard<std::mutex> l(g_mu);
    const int32_t n = (int32_t)g_records.size();
    for (int32_t i = 0; i < std::min(n, cap); i++) recs[i] = g_records[i];
    return n;
}

tn_status tune_env_load() {
    {
        std::lock_guard<std::mutex> l(g_mu);
        if (g_env_done) return TN_OK;
        g_env_done = true;
    }
    const char* p = getenv("TN_TUNE_FILE");
    if (!p || !*p) return TN_OK;
    return tune_load(p, nullptr);
}

}  // namespace tn
