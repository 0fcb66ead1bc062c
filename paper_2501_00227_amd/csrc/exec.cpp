// Single-network executor: leaf initialisation, per-node permute + batched
// semiring GEMM in execution order, slicing loop with root accumulation, and
// root decoding (CRT for exact counts, mantissa/exponent for Z).
#include "exec.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <thread>
#include <unordered_set>

namespace tn {

// ---------------------------------------------------------------- memory --
void* dev_alloc(tn_ctx* ctx, size_t bytes) {
    bytes = std::max<size_t>(bytes, 256);
    if (ctx->has_alloc) return ctx->alloc.alloc(bytes, ctx->alloc.user, (void*)ctx->stream);
    void* p = nullptr;
    if (hipMallocAsync(&p, bytes, ctx->stream) != hipSuccess) return nullptr;
    return p;
}

void dev_free(tn_ctx* ctx, void* p, size_t bytes) {
    if (!p) return;
    bytes = std::max<size_t>(bytes, 256);
    if (ctx->has_alloc)
        ctx->alloc.free(p, bytes, ctx->alloc.user, (void*)ctx->stream);
    else
        (void)hipFreeAsync(p, ctx->stream);
}

tn_status ensure_pinned(tn_ctx* ctx, size_t bytes) {
    if (ctx->pinned_bytes >= bytes) return TN_OK;
    const size_t had = ctx->pinned_bytes;
    if (ctx->pinned) {
        (void)hipStreamSynchronize(ctx->stream);
        (void)hipHostFree(ctx->pinned);
        ctx->pinned = nullptr;
        ctx->pinned_bytes = 0;
    }
    // grow geometrically: a stream of slightly larger requests reallocates
    // (a slow pinned allocation) only a logarithmic number of times
    size_t n = std::max<size_t>(std::max<size_t>(bytes, 1 << 16), 2 * had);
    if (hipHostMalloc(&ctx->pinned, n, hipHostMallocDefault) != hipSuccess)
        return fail(TN_ENOMEM, "hipHostMalloc of the staging buffer failed");
    ctx->pinned_bytes = n;
    return TN_OK;
}

static size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

void* pinned_acquire(tn_ctx* ctx, size_t bytes) {
    std::lock_guard<std::mutex> g(ctx->pinned_mu);
    tn_ctx::PinnedBuf* best = nullptr;
    for (auto& b : ctx->pinned_pool)
        if (!b.busy && b.bytes >= bytes && (!best || b.bytes < best->bytes)) best = &b;
    if (best) {
        best->busy = true;
        return best->p;
    }
    // a new buffer rounds up to a power of two, so later launches of a similar
    // size find it free instead of allocating again
    void* p = nullptr;
    size_t n = 1 << 16;
    while (n < bytes) n <<= 1;
    if (hipHostMalloc(&p, n, hipHostMallocDefault) != hipSuccess) return nullptr;
    ctx->pinned_pool.push_back({p, n, true});
    return p;
}

void pinned_release(tn_ctx* ctx, void* p) {
    std::lock_guard<std::mutex> g(ctx->pinned_mu);
    for (auto& b : ctx->pinned_pool)
        if (b.p == p) b.busy = false;
}

// ------------------------------------------------------------- profiling --
ProfScope::ProfScope(tn_ctx* c, int kind, int node, int sr, const int shape[4], double bytes, double ops,
                     const char* kernel, bool enable)
    : ctx(c), on(c->profiling && enable) {
    if (!on) return;
    auto get = [&]() {
        hipEvent_t e;
        if (!ctx->event_pool.empty()) {
            e = ctx->event_pool.back();
            ctx->event_pool.pop_back();
        } else {
            (void)hipEventCreate(&e);
        }
        return e;
    };
    pr.start = get();
    pr.stop = get();
    pr.rec.kind = kind;
    pr.rec.node = node;
    pr.rec.semiring = sr;
    for (int k = 0; k < 4; k++) pr.rec.shape[k] = shape ? shape[k] : 0;
    pr.rec.ms = 0;
    pr.rec.alg_bytes = bytes;
    pr.rec.ops = ops;
    std::memset(pr.rec.kernel, 0, sizeof pr.rec.kernel);
    std::strncpy(pr.rec.kernel, kernel ? kernel : "", sizeof pr.rec.kernel - 1);
    (void)hipEventRecord(pr.start, ctx->stream);
}

ProfScope::~ProfScope() {
    if (!on) return;
    (void)hipEventRecord(pr.stop, ctx->stream);
    ctx->pending.push_back(pr);
}

// -------------------------------------------------------- device program --
namespace {

// Host side of one program: leaf records, compact permutes, slice positions.
struct ProgramHost {
    const Plan* plan;
    DevProgram dp;
    std::vector<LeafDev> leaves;
    std::vector<PermParams> perms;
    std::vector<int> spos;
    size_t o_leaf = 0, o_spos = 0, perm_first = 0;
};

void build_program_host(const Plan& p, ProgramHost& h) {
    h.plan = &p;
    const int nleaf = p.nleaf();
    h.leaves.resize(nleaf);
    for (int l = 0; l < nleaf; l++) {
        const LeafProg& lp = p.leaf_prog[l];
        LeafDev& d = h.leaves[l];
        d.u = lp.u;
        d.v = lp.has_edge ? lp.v : -1;
        d.flags = (lp.has_edge ? 1 : 0) | (lp.wu ? 2 : 0) | (lp.wv ? 4 : 0) | (p.kind == 1 ? 8 : 0);
        d.jidx = (p.kind == 1 && lp.has_edge) ? p.nv + lp.edge : -1;
        d.pad = 0;
        d.rank = lp.rank;
        d.var0 = lp.var[0];
        d.var1 = lp.var[1];
        d.off = lp.off;
    }
    h.dp.perm_slot_a.assign(p.prog.size(), -1);
    h.dp.perm_slot_b.assign(p.prog.size(), -1);
    auto add_perm = [&](const std::vector<int>& src) {
        PermParams pp;
        build_perm_params((int)src.size(), src.data(), pp);
        h.perms.push_back(pp);
        return (int)h.perms.size() - 1;
    };
    for (size_t t = 0; t < p.prog.size(); t++) {
        const NodeProg& np = p.prog[t];
        if (np.perm_a) h.dp.perm_slot_a[t] = add_perm(np.perm_a_src);
        if (np.perm_b) h.dp.perm_slot_b[t] = add_perm(np.perm_b_src);
    }
    h.spos.assign(std::max(p.nv, 1), -1);
    for (size_t k = 0; k < p.sliced.size(); k++) h.spos[p.sliced[k]] = (int)k;
}

}  // namespace

// Programs for every plan not yet on the device, in one buffer: each plan's
// leaves and slice positions, then all compact permutes (uploaded in one
// copy), then all permute tables, expanded on the device by one launch.
tn_status get_programs(tn_ctx* ctx, const std::vector<const Plan*>& plans) {
    std::vector<const Plan*> fresh;
    std::unordered_set<uint64_t> seen;
    for (const Plan* p : plans)
        if (p && p->nleaf() > 0 && !ctx->progs.count(p->uid) && seen.insert(p->uid).second) fresh.push_back(p);
    if (fresh.empty()) return TN_OK;
    // host tables of each plan (independent: several threads for many plans)
    std::vector<ProgramHost> todo(fresh.size());
    const size_t nthreads =
        fresh.size() >= 32 ? std::min<size_t>(8, std::max(1u, std::thread::hardware_concurrency())) : 1;
    if (nthreads > 1) {
        std::atomic<size_t> next{0};
        std::vector<std::thread> pool;
        for (size_t w = 0; w < nthreads; w++)
            pool.emplace_back([&] {
                for (size_t u = next++; u < fresh.size(); u = next++) build_program_host(*fresh[u], todo[u]);
            });
        for (auto& th : pool) th.join();
    } else {
        for (size_t u = 0; u < fresh.size(); u++) build_program_host(*fresh[u], todo[u]);
    }
    size_t off = 0, nperm = 0;
    for (ProgramHost& h : todo) {
        h.o_leaf = off;
        off = align256(off + sizeof(LeafDev) * h.leaves.size());
        h.o_spos = off;
        off = align256(off + sizeof(int) * h.spos.size());
        h.perm_first = nperm;
        nperm += h.perms.size();
    }
    const size_t o_perm = off;
    const size_t o_tab = align256(o_perm + sizeof(PermParams) * nperm);
    const size_t total = align256(o_tab + sizeof(PermTables) * nperm);
    unsigned char* d = (unsigned char*)dev_alloc(ctx, total);
    if (!d) return fail(TN_ENOMEM, "device allocation of the plan programs failed");
    tn_status st = ensure_pinned(ctx, o_tab);
    if (st != TN_OK) {
        dev_free(ctx, d, total);
        return st;
    }
    (void)hipStreamSynchronize(ctx->stream);  // the staging buffer may still be in use
    unsigned char* hb = (unsigned char*)ctx->pinned;
    for (const ProgramHost& h : todo) {
        std::memcpy(hb + h.o_leaf, h.leaves.data(), sizeof(LeafDev) * h.leaves.size());
        std::memcpy(hb + h.o_spos, h.spos.data(), sizeof(int) * h.spos.size());
        if (!h.perms.empty())
            std::memcpy(hb + o_perm + sizeof(PermParams) * h.perm_first, h.perms.data(),
                        sizeof(PermParams) * h.perms.size());
    }
    if (hipMemcpyAsync(d, hb, o_tab, hipMemcpyHostToDevice, ctx->stream) != hipSuccess ||
        launch_expand_perms((const PermParams*)(d + o_perm), (PermTables*)(d + o_tab), (int)nperm, ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        dev_free(ctx, d, total);
        return fail(TN_EDEVICE, "upload of the plan programs failed");
    }
    ctx->prog_bufs.push_back({d, total});
    PermTables* tabs = (PermTables*)(d + o_tab);
    for (ProgramHost& h : todo) {
        DevProgram& dp = h.dp;
        dp.leaves = (LeafDev*)(d + h.o_leaf);
        dp.slice_pos = (int*)(d + h.o_spos);
        dp.perms = tabs + h.perm_first;
        dp.nperms = (int)h.perms.size();
        ctx->progs.emplace(h.plan->uid, std::move(dp));
    }
    return TN_OK;
}

// Offsets of one program's pieces in its device region.
struct ProgramOffsets {
    size_t o_leaf, o_spos, o_perm, o_tab, total;
};

static ProgramOffsets program_offsets(const ProgramHost& h) {
    ProgramOffsets q;
    q.o_leaf = 0;
    q.o_spos = align256(sizeof(LeafDev) * h.leaves.size());
    q.o_perm = align256(q.o_spos + sizeof(int) * h.spos.size());
    q.o_tab = align256(q.o_perm + sizeof(PermParams) * h.perms.size());
    q.total = align256(q.o_tab + sizeof(PermTables) * h.perms.size());
    return q;
}

size_t program_bytes(const Plan& p) {
    if (p.nleaf() == 0) return 0;
    ProgramHost h;
    build_program_host(p, h);
    return program_offsets(h).total;
}

tn_status program_into(tn_ctx* ctx, const Plan& p, unsigned char* dev, DevProgram& dp) {
    ProgramHost h;
    build_program_host(p, h);
    const ProgramOffsets q = program_offsets(h);
    std::vector<unsigned char> img(q.o_tab, 0);  // pageable: the copy below waits for it
    std::memcpy(img.data() + q.o_leaf, h.leaves.data(), sizeof(LeafDev) * h.leaves.size());
    std::memcpy(img.data() + q.o_spos, h.spos.data(), sizeof(int) * h.spos.size());
    if (!h.perms.empty()) std::memcpy(img.data() + q.o_perm, h.perms.data(), sizeof(PermParams) * h.perms.size());
    hipStream_t s = ctx->stream;
    if (hipMemcpyAsync(dev, img.data(), q.o_tab, hipMemcpyHostToDevice, s) != hipSuccess ||
        (!h.perms.empty() && launch_expand_perms((const PermParams*)(dev + q.o_perm), (PermTables*)(dev + q.o_tab),
                                                 (int)h.perms.size(), s) != hipSuccess) ||
        hipStreamSynchronize(s) != hipSuccess)
        return fail(TN_EDEVICE, "upload of the plan program failed");
    dp = std::move(h.dp);
    dp.leaves = (LeafDev*)(dev + q.o_leaf);
    dp.slice_pos = (int*)(dev + q.o_spos);
    dp.perms = (PermTables*)(dev + q.o_tab);
    dp.nperms = (int)h.perms.size();
    return TN_OK;
}

tn_status get_program(tn_ctx* ctx, const Plan& p, DevProgram*& out) {
    auto it = ctx->progs.find(p.uid);
    if (it == ctx->progs.end()) {
        tn_status st = get_programs(ctx, {&p});
        if (st != TN_OK) return st;
        it = ctx->progs.find(p.uid);
        if (it == ctx->progs.end()) return fail(TN_EINVAL, "a plan without leaves has no program");
    }
    out = &it->second;
    return TN_OK;
}

tn_status ensure_wide_perms(tn_ctx* ctx, const Plan& p, DevProgram& dp) {
    if (dp.perms_wide || dp.nperms == 0) return TN_OK;
    std::vector<PermParams> wide(dp.nperms);
    auto build = [&](const std::vector<int>& src, int slot) {
        std::vector<int> w{0, 1, 2};  // 32-byte entries: eight 4-byte words each
        for (int x : src) w.push_back(x + 3);
        build_perm_params((int)w.size(), w.data(), wide[slot]);
    };
    for (size_t t = 0; t < p.prog.size(); t++) {
        if (dp.perm_slot_a[t] >= 0) build(p.prog[t].perm_a_src, dp.perm_slot_a[t]);
        if (dp.perm_slot_b[t] >= 0) build(p.prog[t].perm_b_src, dp.perm_slot_b[t]);
    }
    // compact permutes (uploaded), then their expanded tables
    const size_t o_tab = align256(sizeof(PermParams) * wide.size());
    const size_t bytes = o_tab + sizeof(PermTables) * wide.size();
    void* buf = dev_alloc(ctx, bytes);
    if (!buf) return fail(TN_ENOMEM, "device allocation of the widened permute tables failed");
    tn_status st = ensure_pinned(ctx, o_tab);
    if (st != TN_OK) {
        dev_free(ctx, buf, bytes);
        return st;
    }
    (void)hipStreamSynchronize(ctx->stream);  // the staging buffer may still be in use
    std::memcpy(ctx->pinned, wide.data(), sizeof(PermParams) * wide.size());
    unsigned char* d = (unsigned char*)buf;
    if (hipMemcpyAsync(buf, ctx->pinned, sizeof(PermParams) * wide.size(), hipMemcpyHostToDevice, ctx->stream) !=
            hipSuccess ||
        launch_expand_perms((const PermParams*)d, (PermTables*)(d + o_tab), (int)wide.size(), ctx->stream) !=
            hipSuccess ||
        hipStreamSynchronize(ctx->stream) != hipSuccess) {
        dev_free(ctx, buf, bytes);
        return fail(TN_EDEVICE, "upload of the widened permute tables failed");
    }
    dp.wide_buf = buf;
    dp.wide_bytes = bytes;
    dp.perms_wide = (PermTables*)(d + o_tab);
    return TN_OK;
}

const LaunchSet& node_launches(DevProgram& dp, const Plan& p, int dsr, bool chiplet) {
    const int64_t key = chiplet ? -1 - (int64_t)dsr : (int64_t)(tune_generation() << 8) | dsr;
    auto it = dp.launch_sets.find(key);
    if (it != dp.launch_sets.end()) return it->second;
    LaunchSet ls;
    ls.nodes.resize(p.prog.size());
    ls.part_off_dag.assign(p.prog.size(), 0);
    for (size_t t = 0; t < p.prog.size(); t++) {
        const NodeProg& np = p.prog[t];
        NodeLaunch& v = ls.nodes[t];
        v.shape = choose_gemm_shape(dsr, np.lb, np.li, np.lj, np.lk, np.a_t, np.b_t, chiplet);
        if (v.shape.lsplit > 0) v.part_entries = (int64_t)1 << (v.shape.lsplit + np.lb + np.li + np.lj);
        ls.part_entries = std::max(ls.part_entries, v.part_entries);
        // concurrent nodes of the dependency-graph executor need separate partials
        ls.part_off_dag[t] = ls.part_entries_dag;
        ls.part_entries_dag += (v.part_entries + 63) & ~(int64_t)63;
    }
    return dp.launch_sets.emplace(key, std::move(ls)).first->second;
}

// --------------------------------------------------------------- algebra --
static uint32_t powmod(uint64_t b, uint64_t e, uint32_t m) {
    uint64_t r = 1 % m;
    b %= m;
    while (e) {
        if (e & 1) r = r * b % m;
        b = b * b % m;
        e >>= 1;
    }
    return (uint32_t)r;
}

AlgebraParams algebra_params(int dsr, uint32_t prime, double beta, uint32_t xval) {
    AlgebraParams ap;
    ap.beta = beta;
    if (dsr == DSR_MODP) {
        uint32_t inv = prime;  // Newton iteration for p^{-1} mod 2^32 (p odd)
        for (int k = 0; k < 5; k++) inv *= 2u - prime * inv;
        ap.p = prime;
        ap.pinv = (uint32_t)(0u - inv);
        ap.r1 = (uint32_t)((1ull << 32) % prime);
        ap.xv = (uint32_t)(((uint64_t)(xval % prime) << 32) % prime);
    }
    return ap;
}

// the largest primes below 2^30 (residues then admit one Montgomery
// reduction per four products: 4 p^2 < p 2^32)
static const uint32_t kDefaultPrimes[kMaxPrimes] = {
    1073741789u, 1073741783u, 1073741741u, 1073741723u, 1073741719u, 1073741717u, 1073741689u, 1073741671u,
    1073741663u, 1073741651u, 1073741621u, 1073741567u, 1073741561u, 1073741527u, 1073741503u, 1073741477u};

static bool is_prime(uint32_t p) {
    if (p < 2) return false;
    for (uint64_t d = 2; d * d <= p; d++)
        if (p % d == 0) return false;
    return true;
}

// log2 of an upper bound on the number of configurations the exact count can
// reach: 2^n for a spin glass; for independent sets the bound of Sah,
// Sawhney, Stoner and Zhao (the number of independent sets is at most the
// product over edges uv of i(K_{d_u, d_v})^(1 / (d_u d_v)), with
// i(K_{a,b}) = 2^a + 2^b - 1), times 2 per isolated vertex.
double count_bound_bits(const Net& net) {
    if (net.kind != 0) return (double)net.nv;
    std::vector<int> deg(net.nv, 0);
    for (auto& e : net.edges) {
        deg[e[0]]++;
        deg[e[1]]++;
    }
    double b = 0;
    for (int v = 0; v < net.nv; v++)
        if (deg[v] == 0) b += 1.0;
    for (auto& e : net.edges) {
        const double du = deg[e[0]], dv = deg[e[1]], m = std::max(du, dv);
        const double l = m + std::log2(std::exp2(du - m) + std::exp2(dv - m) - std::exp2(-m));
        b += l / (du * dv);
    }
    return b;
}

tn_status make_passes(const Net& net, const tn_solve_opts& o, std::vector<PassSpec>& passes) {
    passes.clear();
    switch (o.semiring) {
    case TN_TROPICAL_I32:
        if (!net.integer_weights) return fail(TN_EINVAL, "TN_TROPICAL_I32 needs integer weights (|w| <= 65536)");
        passes.push_back({DSR_TROP_I32, 0});
        break;
    case TN_TROPICAL_F32: passes.push_back({DSR_TROP_F32, 0}); break;
    case TN_COUNTING_TROPICAL:
        if (!net.integer_weights) return fail(TN_EINVAL, "TN_COUNTING_TROPICAL needs integer weights");
        passes.push_back({DSR_CTROP, 0});
        break;
    case TN_COUNT_EXACT: {
        // default: enough CRT primes (each above 2^29.99) for the bound on the
        // count, plus one check prime
        int np = o.nprimes;
        if (np <= 0)
            np = std::min(kMaxPrimes, std::max(2, (int)std::ceil((count_bound_bits(net) + 2.0) / 29.0) + 1));
        if (np < 2 || np > kMaxPrimes)
            return fail(TN_EINVAL, "nprimes must be in [2, 16] (CRT primes + one check prime)");
        for (int k = 0; k < np; k++) {
            uint32_t p = o.primes ? o.primes[k] : kDefaultPrimes[k];
            if (p >= (1u << 30) || p < 3 || !is_prime(p)) return fail(TN_EINVAL, "residue moduli must be odd primes below 2^30");
            for (auto& q : passes)
                if (q.prime == p) return fail(TN_EINVAL, "residue primes must be distinct");
            passes.push_back({DSR_MODP, p});
        }
        break;
    }
    case TN_PARTITION_F32: passes.push_back({DSR_Z_F32, 0}); break;
    case TN_PARTITION_BF16: passes.push_back({DSR_Z_BF16, 0}); break;
    case kSemiringTop8: passes.push_back({DSR_TOPK, 0}); break;
    case kSemiringTPoly4:
        if (!net.integer_weights) return fail(TN_EINVAL, "CountingMax(k) needs integer weights (|w| <= 65536)");
        passes.push_back({DSR_TPOLY, 0});
        break;
    default: return fail(TN_EINVAL, "unknown semiring");
    }
    if ((o.semiring == TN_PARTITION_F32 || o.semiring == TN_PARTITION_BF16) && !std::isfinite(o.beta))
        return fail(TN_EINVAL, "beta must be finite");
    return TN_OK;
}

// little-endian 32-bit limb helpers for the CRT value
struct BigU {
    std::vector<uint32_t> d;
    void mul_small(uint32_t m) {
        uint64_t carry = 0;
        for (auto& x : d) {
            uint64_t t = (uint64_t)x * m + carry;
            x = (uint32_t)t;
            carry = t >> 32;
        }
        if (carry) d.push_back((uint32_t)carry);
    }
    void add(const BigU& o) {
        if (o.d.size() > d.size()) d.resize(o.d.size(), 0);
        uint64_t carry = 0;
        for (size_t k = 0; k < d.size(); k++) {
            uint64_t t = (uint64_t)d[k] + (k < o.d.size() ? o.d[k] : 0) + carry;
            d[k] = (uint32_t)t;
            carry = t >> 32;
        }
        if (carry) d.push_back((uint32_t)carry);
    }
    uint32_t mod_small(uint32_t m) const {
        uint64_t r = 0;
        for (size_t k = d.size(); k-- > 0;) r = ((r << 32) | d[k]) % m;
        return (uint32_t)r;
    }
    void trim() {
        while (!d.empty() && d.back() == 0) d.pop_back();
    }
};

// The exact count from res.residues / res.primes (nresidues of them): Garner
// over all primes but the last, which checks the value.
static tn_status crt_decode(tn_result& res) {
    const int np = res.nresidues;
    BigU x, M;
    x.d = {res.residues[0]};
    M.d = {res.primes[0]};
    for (int k = 1; k < np - 1; k++) {
        uint32_t p = res.primes[k];
        uint32_t xm = x.mod_small(p), mm = M.mod_small(p);
        uint32_t t = (uint32_t)((uint64_t)((res.residues[k] + (uint64_t)p - xm) % p) * powmod(mm, p - 2, p) % p);
        BigU add = M;
        add.mul_small(t);
        x.add(add);
        M.mul_small(p);
    }
    x.trim();
    if (x.d.size() > 16) return fail(TN_EOVERFLOW, "exact count needs more than 512 bits");
    res.count_nlimbs = (int)x.d.size();
    for (size_t k = 0; k < 16; k++) res.count_limbs[k] = k < x.d.size() ? x.d[k] : 0;
    res.count_mod_2_64 = (x.d.size() > 0 ? (uint64_t)x.d[0] : 0) | (x.d.size() > 1 ? (uint64_t)x.d[1] << 32 : 0);
    uint32_t pc = res.primes[np - 1];
    if (x.mod_small(pc) != res.residues[np - 1])
        return fail(TN_EOVERFLOW, "exact count exceeds the CRT range: the check prime disagrees");
    return TN_OK;
}

tn_status combine_results(const tn_result& a, const tn_result& b, tn_result& out) {
    if (a.semiring != b.semiring) return fail(TN_EINVAL, "results of different semirings");
    tn_result r = a;
    r.seconds = a.seconds + b.seconds;
    switch (a.semiring) {
    case TN_TROPICAL_I32:
    case TN_COUNTING_TROPICAL: {
        const bool ca = !a.size_is_neg_inf, cb = !b.size_is_neg_inf;
        if (!ca || (cb && b.size_i32 > a.size_i32)) {
            r.size_i32 = b.size_i32;
            r.size_f32 = b.size_f32;
            r.size_is_neg_inf = b.size_is_neg_inf;
            r.count_mod_2_64 = b.count_mod_2_64;
        } else if (ca && cb && b.size_i32 == a.size_i32) {
            r.count_mod_2_64 = a.count_mod_2_64 + b.count_mod_2_64;  // mod 2^64
        }
        if (a.semiring == TN_TROPICAL_I32) r.count_mod_2_64 = 0;
        break;
    }
    case TN_TROPICAL_F32:
        if (b.size_f32 > a.size_f32 || a.size_is_neg_inf) {
            r.size_f32 = b.size_f32;
            r.size_i32 = b.size_i32;
            r.size_is_neg_inf = b.size_is_neg_inf;
        }
        break;
    case TN_COUNT_EXACT: {
        if (a.nresidues != b.nresidues || a.nresidues < 2 || a.nresidues > 16)
            return fail(TN_EINVAL, "exact counts with different prime sets");
        for (int k = 0; k < a.nresidues; k++) {
            if (a.primes[k] != b.primes[k] || a.primes[k] < 2) return fail(TN_EINVAL, "exact counts with different primes");
            r.residues[k] = (uint32_t)(((uint64_t)a.residues[k] + b.residues[k]) % a.primes[k]);
        }
        tn_status st = crt_decode(r);
        if (st != TN_OK) return st;
        break;
    }
    case TN_PARTITION_F32:
    case TN_PARTITION_BF16: {
        // z = mant * 2^exp with mant in [1, 2) or 0
        const bool za = a.z_mant == 0.0, zb = b.z_mant == 0.0;
        if (za) {
            r = b;
            r.seconds = a.seconds + b.seconds;
        } else if (!zb) {
            const int64_t e = std::max(a.z_exp2, b.z_exp2);
            const int64_t da = std::max<int64_t>(a.z_exp2 - e, -2000), db = std::max<int64_t>(b.z_exp2 - e, -2000);
            int k = 0;
            const double f = std::frexp(std::ldexp(a.z_mant, (int)da) + std::ldexp(b.z_mant, (int)db), &k);
            r.z_mant = 2.0 * f;
            r.z_exp2 = e + k - 1;
            r.log_z = std::log(r.z_mant) + (double)r.z_exp2 * std::log(2.0);
            r.z = r.z_exp2 > 1100 ? INFINITY : std::ldexp(r.z_mant, (int)std::max<int64_t>(r.z_exp2, -2000));
        }
        r.z_range_log2 = std::max(a.z_range_log2, b.z_range_log2);
        break;
    }
    default: return fail(TN_EINVAL, "no combination for this semiring");
    }
    out = r;
    return TN_OK;
}

tn_status decode_result(const tn_solve_opts& o, const std::vector<PassSpec>& passes,
                        const std::vector<std::vector<unsigned char>>& acc, tn_result& res) {
    std::memset(&res, 0, sizeof res);
    res.semiring = o.semiring;
    const unsigned char* a0 = acc[0].data();
    switch (o.semiring) {
    case TN_TROPICAL_I32: {
        int v;
        std::memcpy(&v, a0, 4);
        res.size_i32 = v;
        res.size_f32 = (float)v;
        res.size_is_neg_inf = v <= -(1 << 30);
        break;
    }
    case TN_TROPICAL_F32: {
        float v;
        std::memcpy(&v, a0, 4);
        res.size_f32 = v;
        res.size_i32 = std::isfinite(v) ? (int32_t)v : INT32_MIN;
        res.size_is_neg_inf = std::isinf(v) && v < 0;
        break;
    }
    case TN_COUNTING_TROPICAL: {
        int n;
        uint64_t c;
        std::memcpy(&n, a0, 4);
        std::memcpy(&c, a0 + 8, 8);
        res.size_i32 = n;
        res.size_f32 = (float)n;
        res.size_is_neg_inf = n <= -(1 << 30);
        res.count_mod_2_64 = res.size_is_neg_inf ? 0 : c;
        break;
    }
    case TN_COUNT_EXACT: {
        const int np = (int)passes.size();
        res.nresidues = np;
        for (int k = 0; k < np; k++) {
            uint32_t p = passes[k].prime, xm;
            std::memcpy(&xm, acc[k].data(), 4);
            uint32_t rinv = powmod((1ull << 32) % p, p - 2, p);  // R^{-1} mod p
            res.residues[k] = (uint32_t)((uint64_t)xm * rinv % p);
            res.primes[k] = p;
        }
        tn_status st = crt_decode(res);
        if (st != TN_OK) return st;
        break;
    }
    case TN_PARTITION_F32:
    case TN_PARTITION_BF16: {
        double m;
        int64_t e;
        std::memcpy(&m, a0, 8);
        std::memcpy(&e, a0 + 8, 8);
        res.z_mant = m;
        res.z_exp2 = m == 0.0 ? 0 : e;
        res.log_z = m == 0.0 ? -INFINITY : std::log(m) + (double)e * std::log(2.0);
        res.z = m == 0.0 ? 0.0 : (e > 1100 ? INFINITY : std::ldexp(m, (int)std::max<int64_t>(e, -2000)));
        if (acc[0].size() >= (size_t)kZRangeOffset + 4) {
            float r;
            std::memcpy(&r, a0 + kZRangeOffset, 4);
            res.z_range_log2 = r;
        }
        break;
    }
    case kSemiringTop8:
    case kSemiringTPoly4: break;  // the caller reads the raw accumulator
    default: return fail(TN_EINVAL, "unknown semiring");
    }
    return TN_OK;
}

// ------------------------------------------------------------------ solve --
static int64_t node_entries(const Plan& p, int node) { return (int64_t)1 << p.order[node].size(); }

// Check the plan against the network and the slice range against the plan.
tn_status check_solve(const Net& net, const Plan& plan, const tn_solve_opts& o, int64_t& sb, int64_t& se) {
    if (plan.fingerprint != net.fingerprint || plan.nv != net.nv)
        return fail(TN_EINVAL, "plan was built for a different network");
    const int ns = (int)plan.sliced.size();
    if (ns > 62) return fail(TN_EINVAL, "too many sliced indices");
    const int64_t nslices = (int64_t)1 << ns;
    sb = o.slice_begin;
    se = o.slice_end;
    if (sb == 0 && se == 0) se = nslices;
    if (sb < 0 || se > nslices || sb >= se) return fail(TN_EINVAL, "slice range out of bounds");
    return TN_OK;
}

// Offsets (bytes from the solve buffer's base) of the arena planes, split
// partials, Z bookkeeping, weights and root accumulators of one solve.
SolveLayout solve_layout(const Net& net, const Plan& plan, const std::vector<PassSpec>& passes, DevProgram* dp,
                         bool tensor_root) {
    SolveLayout L;
    const int nn = (int)plan.nodes.size();
    const int64_t E = std::max<int64_t>(plan.arena_entries, 64);
    int64_t Pe = 0;
    for (auto& ps : passes)
        if (dp) Pe = std::max(Pe, node_launches(*dp, plan, ps.dsr, false).part_entries);
    for (auto& ps : passes) {
        L.pb0 = std::max(L.pb0, plane_bytes(ps.dsr, 0));
        L.pb1 = std::max(L.pb1, plane_bytes(ps.dsr, 1));
    }
    L.o_a0 = 0;
    L.o_a1 = align256(L.o_a0 + (size_t)E * L.pb0);
    L.o_p0 = align256(L.o_a1 + (size_t)E * L.pb1);
    L.o_p1 = align256(L.o_p0 + (size_t)Pe * L.pb0);
    L.o_meta = align256(L.o_p1 + (size_t)Pe * L.pb1);
    L.o_w = align256(L.o_meta + sizeof(TensorMeta) * (size_t)std::max(nn, 1));
    // root entries: 2^|open| for plans with open vertices, else one
    L.nent = (plan.nleaf() > 0 && tensor_root) ? (int64_t)1 << plan.order[nn - 1].size() : 1;
    L.acc_bytes = kAccSlotBytes * (size_t)L.nent * passes.size();
    L.o_acc = align256(L.o_w + sizeof(float) * std::max<size_t>(net.wdev.size(), 1));
    L.need = align256(L.o_acc + L.acc_bytes);
    return L;
}

// Every pass over slices [sb, se) on the context stream, in the solve buffer
// at base (laid out by L); stage: host memory of at least
// max(L.acc_bytes, weight bytes) for the weight upload and the result copy.
// all receives the accumulators of every pass.
tn_status run_solve(tn_ctx* ctx, const Net& net, const Plan& plan, const tn_solve_opts& o,
                    const std::vector<PassSpec>& passes, DevProgram* dp, unsigned char* base, const SolveLayout& L,
                    int64_t sb, int64_t se, void* stage, std::vector<unsigned char>& all) {
    return run_solve_on(ctx, ctx->stream, false, net, plan, o, passes, dp, base, L, sb, se, stage, &all);
}

tn_status run_solve_on(tn_ctx* ctx, hipStream_t s, bool async, const Net& net, const Plan& plan,
                       const tn_solve_opts& o, const std::vector<PassSpec>& passes, DevProgram* dp,
                       unsigned char* base, const SolveLayout& L, int64_t sb, int64_t se, void* stage,
                       std::vector<unsigned char>* all) {
    const bool prof = !async;  // launches of another thread's stream are not profiled
    const int nleaf = plan.nleaf();
    const int nn = (int)plan.nodes.size();
    const int pb1 = L.pb1;
    Planes arena{base + L.o_a0, pb1 ? base + L.o_a1 : nullptr};
    Planes part{base + L.o_p0, pb1 ? base + L.o_p1 : nullptr};
    TensorMeta* meta = (TensorMeta*)(base + L.o_meta);
    float* wdev = net.wdev.empty() ? nullptr : (float*)(base + L.o_w);
    const int64_t nent = L.nent;
    hipError_t herr = hipSuccess;
    const char* herr_at = "";
    auto chk = [&](hipError_t e, const char* at) {
        if (e != hipSuccess && herr == hipSuccess) {
            herr = e;
            herr_at = at;
        }
    };
    if (wdev) {
        if (!async) chk(hipStreamSynchronize(s), "sync before weights");
        std::memcpy(stage, net.wdev.data(), sizeof(float) * net.wdev.size());
        chk(hipMemcpyAsync(wdev, stage, sizeof(float) * net.wdev.size(), hipMemcpyHostToDevice, s), "weights upload");
        // the staging is reused for the results: in order on the stream
        if (!async) chk(hipStreamSynchronize(s), "weights sync");
    }
    auto plane_at = [&](Planes pl, int dsr, int64_t off) {
        Planes r;
        r.p0 = (unsigned char*)pl.p0 + off * plane_bytes(dsr, 0);
        r.p1 = plane_bytes(dsr, 1) ? (unsigned char*)pl.p1 + off * plane_bytes(dsr, 1) : nullptr;
        return r;
    };
    for (size_t pi = 0; pi < passes.size() && herr == hipSuccess; pi++) {
        const int dsr = passes[pi].dsr;
        AlgebraParams ap = algebra_params(dsr, passes[pi].prime, o.beta, passes[pi].xval);
        ap.fix_off = net.fix_off;
        void* acc = base + L.o_acc + kAccSlotBytes * (size_t)nent * pi;
        const int eb = plane_bytes(dsr, 0) + plane_bytes(dsr, 1);
        const bool is_z = dsr == DSR_Z_F32 || dsr == DSR_Z_BF16;
        if (nleaf == 0) {
            chk(launch_set_one(dsr, acc, ap, s), "set one");
            continue;
        }
        const auto& launches = node_launches(*dp, plan, dsr, false).nodes;
        for (int64_t sl = sb; sl < se && herr == hipSuccess; sl++) {
            if (is_z) chk(launch_meta_init(meta, nn, s), "meta init");
            {
                char kn[64];
                snprintf(kn, sizeof kn, "leaf_kernel<%d>", dsr);
                ProfScope ps(ctx, TN_K_LEAF, -1, o.semiring, nullptr, (double)plan.leaf_entries * eb, 0, kn, prof);
                chk(launch_leaves(dsr, dp->leaves, nleaf, wdev, dp->slice_pos, (unsigned long long)sl, arena, ap,
                                  meta, s),
                    "leaves");
            }
            for (size_t t = 0; t < plan.prog.size() && herr == hipSuccess; t++) {
                const NodeProg& np = plan.prog[t];
                const NodeLaunch& nl = launches[t];
                Planes Ap = plane_at(arena, dsr, plan.node_off[np.a]);
                Planes Bp = plane_at(arena, dsr, plan.node_off[np.b]);
                for (int side = 0; side < 2; side++) {
                    bool perm = side ? np.perm_b : np.perm_a;
                    if (!perm) continue;
                    int slot = side ? dp->perm_slot_b[t] : dp->perm_slot_a[t];
                    int src_node = side ? np.b : np.a;
                    int rank = (int)plan.order[src_node].size();
                    Planes src = side ? Bp : Ap;
                    Planes dst = plane_at(arena, dsr, side ? np.b_tmp_off : np.a_tmp_off);
                    int tb = perm_tile_bits(rank);
                    int shp[4] = {rank, 0, 0, 0};
                    for (int pl = 0; pl < 2; pl++) {
                        int pbytes = plane_bytes(dsr, pl);
                        if (!pbytes) continue;
                        ProfScope ps(ctx, TN_K_PERMUTE, np.node, o.semiring, shp,
                                     2.0 * (double)node_entries(plan, src_node) * pbytes, 0,
                                     pbytes == 8 ? "permute_kernel<unsigned long long>" : "permute_kernel<unsigned int>",
                                     prof);
                        if (pbytes == 32)  // 32-byte entries: 4-byte words, the three lowest bits in place
                            chk(launch_permute(4, pl ? src.p1 : src.p0, pl ? dst.p1 : dst.p0, dp->perms_wide + slot,
                                               rank + 3, perm_tile_bits(rank + 3), s),
                                "permute");
                        else
                            chk(launch_permute(pbytes, pl ? src.p1 : src.p0, pl ? dst.p1 : dst.p0, dp->perms + slot,
                                               rank, tb, s),
                                "permute");
                    }
                    if (side)
                        Bp = dst;
                    else
                        Ap = dst;
                }
                Planes Cp = plane_at(arena, dsr, np.c_off);
                const GemmShape& g = nl.shape;
                double ent = std::exp2((double)(g.lb + g.li + g.lk)) + std::exp2((double)(g.lb + g.lk + g.lj)) +
                             std::exp2((double)(g.lb + g.li + g.lj));
                int shp[4] = {g.lb, g.li, g.lj, g.lk};
                {
                    const int kind = g.mode == GEMM_THIN  ? TN_K_GEMM_THIN
                                     : g.mode == GEMM_DOT ? TN_K_GEMM_DOT
                                     : g.mfma             ? TN_K_GEMM_MFMA
                                     : g.rm == 8          ? TN_K_GEMM_BIG
                                                          : TN_K_GEMM;
                    char kn[64];
                    ProfScope ps(ctx, kind, np.node, o.semiring, shp, ent * eb,
                                 std::exp2((double)(g.lb + g.li + g.lj + g.lk)), gemm_kernel_name(dsr, g, kn, sizeof kn),
                                 prof);
                    chk(launch_gemm(dsr, Ap, Bp, Cp, part, g, ap, meta, np.a, np.b, np.node, s), "gemm");
                }
                if (g.lsplit > 0) {
                    int64_t nout = (int64_t)1 << (g.lb + g.li + g.lj);
                    char kn[64];
                    snprintf(kn, sizeof kn, "split_reduce_kernel<%d>", dsr);
                    ProfScope ps(ctx, TN_K_ACCUM, np.node, o.semiring, shp,
                                 (double)(nout << g.lsplit) * eb + (double)nout * eb, 0, kn, prof);
                    chk(launch_split_reduce(dsr, part, Cp, nout, g.lsplit, ap, meta, np.node, s), "split reduce");
                }
            }
            int root = nn - 1;
            chk(launch_accumulate(dsr, plane_at(arena, dsr, plan.node_off[root]), root, meta, acc, sl == sb ? 1 : 0,
                                  ap, s, nent),
                "root accumulate");
            if (is_z) chk(launch_z_range(meta, nn, acc, sl == sb ? 1 : 0, s), "z range");
        }
    }
    if (herr == hipSuccess) chk(hipMemcpyAsync(stage, base + L.o_acc, L.acc_bytes, hipMemcpyDeviceToHost, s), "result copy");
    if (!async) {
        all->assign(L.acc_bytes, 0);
        if (herr == hipSuccess) {
            chk(hipStreamSynchronize(s), "result sync");
            std::memcpy(all->data(), stage, L.acc_bytes);
        }
    }
    if (herr != hipSuccess) return fail(TN_EDEVICE, std::string("HIP error at ") + herr_at + ": " + hipGetErrorString(herr));
    return TN_OK;
}

tn_status decode_root(const tn_solve_opts& o, const std::vector<PassSpec>& passes, const std::vector<unsigned char>& all,
                      int64_t nent, int64_t addr, tn_result& r) {
    std::vector<std::vector<unsigned char>> accs(passes.size(), std::vector<unsigned char>(kAccSlotBytes));
    for (size_t k = 0; k < passes.size(); k++) {
        std::memcpy(accs[k].data(), all.data() + kAccSlotBytes * ((size_t)nent * k + (size_t)addr), kAccSlotBytes);
        // the Z dynamic range belongs to the whole contraction: entry 0's slot
        std::memcpy(accs[k].data() + kZRangeOffset, all.data() + kAccSlotBytes * ((size_t)nent * k) + kZRangeOffset, 4);
    }
    return decode_result(o, passes, accs, r);
}

tn_status solve_one(tn_ctx* ctx, const Net& net, const Plan& plan, const tn_solve_opts& o, tn_result& res,
                    std::vector<tn_result>* tensor, std::vector<unsigned char>* raw) {
    auto t0 = std::chrono::steady_clock::now();
    int64_t sb = 0, se = 0;
    tn_status st = check_solve(net, plan, o, sb, se);
    if (st != TN_OK) return st;
    if (!plan.open.empty() && !tensor) return fail(TN_EINVAL, "the plan has open vertices: use tn_solve_open");
    std::vector<PassSpec> passes;
    st = make_passes(net, o, passes);
    if (st != TN_OK) return st;
    const int nleaf = plan.nleaf();
    const int nn = (int)plan.nodes.size();

    DevProgram* dp = nullptr;
    if (nleaf > 0) {
        st = get_program(ctx, plan, dp);
        if (st != TN_OK) return st;
        for (auto& ps : passes)
            if (plane_bytes(ps.dsr, 0) == 32 || plane_bytes(ps.dsr, 1) == 32) {
                st = ensure_wide_perms(ctx, plan, *dp);
                if (st != TN_OK) return st;
            }
    }
    // one allocation: arena planes, split partials, meta, weights, accumulator
    const SolveLayout L = solve_layout(net, plan, passes, dp, tensor != nullptr);
    unsigned char* base = (unsigned char*)dev_alloc(ctx, L.need);
    if (!base) return fail(TN_ENOMEM, "device allocation of " + std::to_string(L.need) + " bytes failed");
    st = ensure_pinned(ctx, std::max<size_t>(L.acc_bytes, sizeof(float) * net.wdev.size()) + 64);
    if (st != TN_OK) {
        dev_free(ctx, base, L.need);
        return st;
    }
    std::vector<unsigned char> all;
    st = run_solve(ctx, net, plan, o, passes, dp, base, L, sb, se, ctx->pinned, all);
    dev_free(ctx, base, L.need);
    if (st != TN_OK) return st;
    if (raw) raw->assign(all.begin(), all.begin() + kAccSlotBytes);
    const int64_t nent = L.nent;
    const double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (tensor) {
        // result entry bit q = open vertex plan.open[q]; find its bit in the root
        const int k = (int)plan.open.size();
        std::vector<int> pos(k, 0);
        if (nleaf > 0)
            for (int q = 0; q < k; q++) {
                const auto& ord = plan.order[nn - 1];
                pos[q] = (int)(std::find(ord.begin(), ord.end(), plan.open[q]) - ord.begin());
            }
        tensor->assign((size_t)1 << k, tn_result{});
        for (int64_t e = 0; e < ((int64_t)1 << k); e++) {
            int64_t addr = 0;
            for (int q = 0; q < k; q++) addr |= ((e >> q) & 1) << pos[q];
            tn_status s2 = decode_root(o, passes, all, nent, addr, (*tensor)[e]);
            if (s2 != TN_OK) return s2;
            (*tensor)[e].seconds = sec;
        }
        res = (*tensor)[0];
        return TN_OK;
    }
    st = decode_root(o, passes, all, nent, 0, res);
    res.seconds = sec;
    return st;
}

}  // namespace tn
