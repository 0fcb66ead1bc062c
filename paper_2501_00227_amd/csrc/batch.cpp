// Host side of the persistent batched executor: builds the task table of a
// set of contraction passes, uploads it with one copy, launches one
// persistent kernel, and decodes the roots.
#include "batch_host.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <queue>
#include <thread>

namespace tn {

namespace {

struct Counter {
    int id = -1;
    int need = 0;
    int level = 0;
};

size_t a256(size_t x) { return (x + 255) & ~(size_t)255; }

// tensors of at most 2^small_rank() entries are contracted inside one task;
// Fusing trades parallelism inside one job for fewer synchronisations: it
// pays when a launch holds enough jobs to keep every chiplet busy.
int small_rank(size_t njobs, int nworkgroups) {
    static int env = -2;
    if (env == -2) {
        const char* e = std::getenv("TN_FUSE_RANK");
        env = e ? std::atoi(e) : -1;
    }
    if (env >= 0) return env;
    return (int)njobs >= nworkgroups / 4 ? 12 : 0;
}
// a large node is cut into at most this many tasks (each loops over tiles);
// the wide-entry algebras' GEMM tiles (eight-lists, truncated polynomials)
// cost some twenty times a 4-byte tile, so their GEMMs get one task per
// resident workgroup (two per CU)
constexpr int64_t kMaxTasksPerNode = 64;
constexpr int64_t kMaxTasksPerNodeTop8 = 512;

int64_t chunk(int64_t ntiles, int64_t max_tasks = kMaxTasksPerNode) {  // tiles per task (powers of two divide exactly)
    int64_t per = 1;
    while (ntiles / per > max_tasks) per *= 2;
    return per;
}

// Estimated microseconds one workgroup spends on a task (a rough model: a
// fixed cost per task, permutes at ~20 GB/s and GEMMs at ~50 G semiring ops/s
// per workgroup); only the relative order matters.
double task_cost(const BTask& t, const std::vector<BNode>& bn, const std::vector<int>& subtree) {
    auto gemm_ops = [&](const BNode& N, double tiles) {
        return tiles * std::exp2((double)(N.g.tb + N.g.ti + N.g.tj + N.g.lk - N.g.lsplit));
    };
    switch (t.kind) {
    case BT_PERM: {
        const BNode& N = bn[t.node];
        const double bytes = (double)t.count * std::exp2((double)N.ptile_bits[t.aux >> 1]) * 8.0;
        return 3.0 + bytes / 2.0e4;
    }
    case BT_GEMM: return 3.0 + gemm_ops(bn[t.node], (double)t.count) / 5.0e4;
    case BT_REDUCE: return 3.0 + (double)t.count * 0.5;
    case BT_SUBTREE: {
        double c = 3.0;
        for (int k = 0; k < t.aux; k++) {
            const BNode& N = bn[subtree[t.node + k]];
            c += 1.0 + gemm_ops(N, std::exp2((double)((N.g.lb - N.g.tb) + (N.g.li - N.g.ti) + (N.g.lj - N.g.tj) +
                                                      N.g.lsplit))) / 5.0e4;
        }
        return c;
    }
    default: return 2.0;
    }
}

// Rank of every task in an earliest-start-first order: a simulation of
// `workers` workgroups that each take the next ticket when free, as the
// device does.  A task enters the candidates once all its producers hold
// tickets (so producers always precede consumers), with an estimated ready
// time (its counters' last producer end plus a signalling latency); the free
// workgroup takes, among the candidates ready by then, the one with the
// largest bottom level, else the one ready first.  Unlike a plain
// critical-path order, a task whose inputs are still far off does not hold a
// workgroup (and the tickets behind it) while work that could run waits.
std::vector<int> earliest_start_order(const std::vector<BTask>& bt, const std::vector<BNode>& bn,
                                      const std::vector<int>& subtree, int ncounters, int workers) {
    constexpr double kSignalLatency = 2.0;  // microseconds from a producer's end to a waiter's start
    const int n = (int)bt.size();
    std::vector<double> cost(n), blevel(n, 0.0), cblevel(ncounters, 0.0);
    for (int k = n - 1; k >= 0; k--) {
        const BTask& t = bt[k];
        cost[k] = task_cost(t, bn, subtree);
        blevel[k] = cost[k] + (t.signal >= 0 ? cblevel[t.signal] : 0.0);
        for (int d : {t.dep0, t.dep1})
            if (d >= 0) cblevel[d] = std::max(cblevel[d], blevel[k]);
    }
    std::vector<int> producers_left(ncounters, 0), waiting(n, 0);
    std::vector<std::vector<int>> waiters(ncounters);
    for (int k = 0; k < n; k++) {
        const BTask& t = bt[k];
        if (t.signal >= 0) producers_left[t.signal]++;
        for (int d : {t.dep0, t.dep1})
            if (d >= 0) {
                waiters[d].push_back(k);
                waiting[k]++;
            }
    }
    std::vector<double> cdone(ncounters, 0.0);
    using RK = std::pair<double, int>;
    std::priority_queue<RK, std::vector<RK>, std::greater<RK>> pending;  // (estimated ready, task)
    std::priority_queue<RK> avail;                                        // (bottom level, -task)
    std::priority_queue<double, std::vector<double>, std::greater<double>> free_at;
    for (int w = 0; w < std::max(workers, 1); w++) free_at.push(0.0);
    for (int k = 0; k < n; k++)
        if (!waiting[k]) pending.push({0.0, k});
    std::vector<int> rank(n, 0);
    int next = 0;
    while (!pending.empty() || !avail.empty()) {
        double start = free_at.top();
        if (avail.empty() && pending.top().first > start) start = pending.top().first;
        while (!pending.empty() && pending.top().first <= start) {
            avail.push({blevel[pending.top().second], -pending.top().second});
            pending.pop();
        }
        const int k = -avail.top().second;
        avail.pop();
        free_at.pop();
        const double end = start + cost[k];
        free_at.push(end);
        rank[k] = next++;
        const int c = bt[k].signal;
        if (c < 0) continue;
        cdone[c] = std::max(cdone[c], end);
        if (--producers_left[c] == 0)
            for (int w : waiters[c])
                if (--waiting[w] == 0) {
                    double r = 0.0;
                    for (int d : {bt[w].dep0, bt[w].dep1})
                        if (d >= 0) r = std::max(r, cdone[d] + kSignalLatency);
                    pending.push({r, w});
                }
    }
    for (int k = 0; k < n; k++)  // unreachable with a well-formed table; keep every task in a valid place
        if (waiting[k]) rank[k] = next++;
    return rank;
}

struct JobPlan {
    int item, pass;
    const Plan* plan;
    int dsr;
    uint32_t prime, xval;
    DevProgram* dp;
    const LaunchSet* ls;
    int64_t E, Pe;
    size_t o_arena0, o_arena1, o_part0, o_part1, o_meta, o_acc;
};

// The tasks, nodes and fused-subtree lists of one job, built once per (plan,
// algebra) in a launch and copied for every job that shares them (many
// passes of one network differ only in their prime or evaluation point):
// node ids, subtree offsets and counter ids are relative to the job's own
// first entries, the job index is 0.
struct JobTemplate {
    std::vector<BNode> bn;
    std::vector<BTask> bt;
    std::vector<int> subtree;
    int ncounters = 0;
    double ops = 0, bytes = 0, work = 0;
    std::vector<int> order;  // task indices in earliest-start-first order
    int bn0 = -1, sub0 = 0;  // where the launch holds its nodes and subtree lists (shared by its jobs)
};

void build_template(const JobPlan& jp, int fuse_rank, JobTemplate& T) {
    const Plan& p = *jp.plan;
    auto add = [&](int kind, int node, int aux, int64_t tile, Counter d0, Counter d1, int signal, int lvl,
                   int count = 1) {
        BTask t;
        t.kind = kind;
        t.job = 0;
        t.node = node;
        t.aux = aux;
        t.tile = tile;
        t.dep0 = d0.id;
        t.need0 = d0.need;
        t.dep1 = d1.id;
        t.need1 = d1.need;
        t.signal = signal;
        t.count = count;
        T.bt.push_back(t);
        (void)lvl;
    };
    if (p.nleaf() == 0) {
        add(BT_ONE, -1, 0, 0, Counter(), Counter(), -1, 0);
        return;
    }
    const int nleaf = p.nleaf();
    Counter leaves_done{T.ncounters++, 1, 0};
    add(BT_LEAVES, -1, 0, 0, Counter(), Counter(), leaves_done.id, 0);
    std::vector<Counter> final_of(p.nodes.size());
    for (int l = 0; l < nleaf; l++) final_of[l] = leaves_done;
    const int npl = plane_bytes(jp.dsr, 1) ? 2 : 1;
    // small subtrees (every tensor <= 2^fuse_rank entries) run as one
    // task each: one workgroup contracts the whole subtree in order
    const int ninner = (int)p.prog.size();
    std::vector<char> small(ninner, 0);
    std::vector<int> parent_t(p.nodes.size(), -1);
    for (int t = 0; t < ninner; t++) {
        const NodeProg& np = p.prog[t];
        parent_t[np.a] = parent_t[np.b] = t;
        int r = std::max({(int)p.order[np.a].size(), (int)p.order[np.b].size(), (int)p.order[np.node].size()});
        bool ok = r <= fuse_rank;
        for (int ch : {np.a, np.b})
            if (ch >= nleaf && !small[ch - nleaf]) ok = false;
        small[t] = ok;
    }
    const int bn0 = 0;
    for (int t = 0; t < ninner; t++) {
        const NodeProg& np = p.prog[t];
        const NodeLaunch& nl = jp.ls->nodes[t];
        BNode N{};
        N.g = nl.shape;  // chiplet-scope shape: never the 128 x 128 matrix-core tiles
        N.ma = np.a;
        N.mb = np.b;
        N.mc = np.node;
        N.a_off = np.perm_a ? np.dag_a_tmp : p.node_off_dag[np.a];
        N.b_off = np.perm_b ? np.dag_b_tmp : p.node_off_dag[np.b];
        N.c_off = np.dag_c_off;
        N.nout = (int64_t)1 << (N.g.lb + N.g.li + N.g.lj);
        N.reduce_per_block = N.nout < 1024 ? 1 : 0;
        N.part_off = jp.ls->part_off_dag[t];
        for (int side = 0; side < 2; side++) {
            int child = side ? np.b : np.a;
            bool perm = side ? np.perm_b : np.perm_a;
            N.pp[side] = nullptr;
            if (!perm) continue;
            int slot = side ? jp.dp->perm_slot_b[t] : jp.dp->perm_slot_a[t];
            int rank = (int)p.order[child].size();
            // 32-byte entries move as eight 4-byte words: three more bits, kept lowest
            const int wide = jp.dsr == DSR_TOPK ? 3 : 0;
            N.pp[side] = (wide ? jp.dp->perms_wide : jp.dp->perms) + slot;
            N.pp1[side] = jp.dsr == DSR_TPOLY ? jp.dp->perms_wide + slot : nullptr;
            N.psrc[side] = p.node_off_dag[child];
            N.pdst[side] = side ? np.dag_b_tmp : np.dag_a_tmp;
            N.prank[side] = rank + wide;
            N.ptile_bits[side] = perm_tile_bits(rank + wide);
        }
        T.ops += std::exp2((double)(N.g.lb + N.g.li + N.g.lj + N.g.lk));
        T.bytes += (std::exp2((double)(N.g.lb + N.g.li + N.g.lk)) + std::exp2((double)(N.g.lb + N.g.lk + N.g.lj)) +
                          std::exp2((double)(N.g.lb + N.g.li + N.g.lj))) *
                         (plane_bytes(jp.dsr, 0) + plane_bytes(jp.dsr, 1));
        T.bn.push_back(N);
        if (small[t]) {
            bool sub_root = parent_t[np.node] < 0 || !small[parent_t[np.node]];
            if (!sub_root) continue;
            // collect the subtree's inner nodes in execution order
            std::vector<int> stack{t}, members;
            while (!stack.empty()) {
                int u = stack.back();
                stack.pop_back();
                members.push_back(u);
                for (int ch : {p.prog[u].a, p.prog[u].b})
                    if (ch >= nleaf) stack.push_back(ch - nleaf);
            }
            std::sort(members.begin(), members.end());
            int off = (int)T.subtree.size();
            for (int u : members) T.subtree.push_back(bn0 + u);
            Counter done{T.ncounters++, 1, leaves_done.level + 1};
            add(BT_SUBTREE, off, (int)members.size(), 0, leaves_done, Counter(), done.id, done.level);
            final_of[np.node] = done;
            continue;
        }
        const int nidx = bn0 + t;
        Counter ready[2];
        for (int side = 0; side < 2; side++) {
            int child = side ? np.b : np.a;
            if (!N.pp[side]) {
                ready[side] = final_of[child];
                continue;
            }
            // tiles per plane (the truncated polynomial's count plane moves as
            // 4-byte words of rank + 3)
            int64_t per_pl[2], ntask_pl[2], ntask_all = 0;
            for (int pl = 0; pl < npl; pl++) {
                const int r = (jp.dsr == DSR_TPOLY && pl == 1) ? N.prank[side] + 3 : N.prank[side];
                const int64_t ntiles = (int64_t)1 << (r - perm_tile_bits(r));
                per_pl[pl] = chunk(ntiles);
                ntask_pl[pl] = ntiles / per_pl[pl];
                ntask_all += ntask_pl[pl];
            }
            Counter c{T.ncounters++, (int)ntask_all, final_of[child].level + 1};
            for (int pl = 0; pl < npl; pl++)
                for (int64_t k = 0; k < ntask_pl[pl]; k++)
                    add(BT_PERM, nidx, side * 2 + pl, k * per_pl[pl], final_of[child], Counter(), c.id, c.level,
                        (int)per_pl[pl]);
            ready[side] = c;
        }
        int64_t nblocks = (int64_t)1 << ((N.g.lb - N.g.tb) + (N.g.li - N.g.ti) + (N.g.lj - N.g.tj) + N.g.lsplit);
        const bool wide_entry = jp.dsr == DSR_TOPK || jp.dsr == DSR_TPOLY;
        int64_t per = chunk(nblocks, wide_entry ? kMaxTasksPerNodeTop8 : kMaxTasksPerNode);
        Counter gdone{T.ncounters++, (int)(nblocks / per), std::max(ready[0].level, ready[1].level) + 1};
        for (int64_t k = 0; k < nblocks / per; k++)
            add(BT_GEMM, nidx, 0, k * per, ready[0], ready[1], gdone.id, gdone.level, (int)per);
        Counter fin = gdone;
        if (N.g.lsplit > 0) {
            int64_t nred = N.reduce_per_block ? N.nout : (N.nout + 255) / 256;
            int64_t rper = 1;
            while (nred / rper > kMaxTasksPerNode) rper *= 2;
            int64_t nrt = (nred + rper - 1) / rper;
            Counter rdone{T.ncounters++, (int)nrt, gdone.level + 1};
            for (int64_t k = 0; k < nrt; k++)
                add(BT_REDUCE, nidx, 0, k * rper, gdone, Counter(), rdone.id, rdone.level,
                    (int)std::min<int64_t>(rper, nred - k * rper));
            fin = rdone;
        }
        final_of[np.node] = fin;
    }
    int root = (int)p.nodes.size() - 1;
    add(BT_ACCUM, -1, 0, p.node_off_dag[root], final_of[root], Counter(), -1, final_of[root].level + 1);
}

}  // namespace

int device_cu_count(tn_ctx* ctx) {
    if (ctx->cu_count > 0) return ctx->cu_count;
    int n = 0;
    if (hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, ctx->device) != hipSuccess || n <= 0) n = 256;
    ctx->cu_count = n;
    return n;
}

// Host-side phase timing of batch_prepare on stderr when TN_HOST_TIMING is
// set (diagnostics only).
namespace {
struct PhaseClock {
    bool on;
    std::chrono::steady_clock::time_point t;
    PhaseClock() : on(std::getenv("TN_HOST_TIMING") != nullptr), t(std::chrono::steady_clock::now()) {}
    void mark(const char* what, size_t njobs) {
        if (!on) return;
        const auto now = std::chrono::steady_clock::now();
        std::fprintf(stderr, "[tn host] %-10s %8.3f ms (%zu jobs)\n", what,
                     std::chrono::duration<double, std::milli>(now - t).count(), njobs);
        t = now;
    }
};
}  // namespace

tn_status batch_prepare(tn_ctx* ctx, std::vector<BatchItem>& items, BatchLaunch& L, const DevAllocFn& alloc) {
    PhaseClock clk;
    L = BatchLaunch();
    L.items.resize(items.size());
    std::vector<JobPlan> jobs;
    std::vector<size_t> item_w_off(items.size(), 0);
    size_t data = 0;
    // weights of every item first, so one contiguous copy uploads them
    for (size_t i = 0; i < items.size(); i++) {
        if (!items[i].net->wdev.empty()) {
            item_w_off[i] = data;
            data = a256(data + sizeof(float) * items[i].net->wdev.size());
        }
    }
    const size_t weights_end = data;
    // programs of every plan new to the device, with one upload (a failure
    // here is reported per item by get_program below)
    {
        std::vector<const Plan*> plans;
        plans.reserve(items.size());
        for (const BatchItem& it : items)
            if (it.plan && it.plan->fingerprint == it.net->fingerprint) plans.push_back(it.plan);
        (void)get_programs(ctx, plans);
    }
    clk.mark("programs", items.size());
    // ---- per item: passes and device programs; lay out device memory
    for (size_t i = 0; i < items.size(); i++) {
        BatchItem& it = items[i];
        ItemState& st = L.items[i];
        st.opts = it.opts;
        st.status = TN_OK;
        if (it.plan->fingerprint != it.net->fingerprint || it.plan->nv != it.net->nv) {
            st.status = fail(TN_EINVAL, "plan was built for a different network");
            continue;
        }
        if (!it.plan->sliced.empty()) {
            st.status = fail(TN_EINVAL, "batched jobs must not be sliced; use tn_solve for sliced plans");
            continue;
        }
        if (!it.plan->open.empty()) {
            st.status = fail(TN_EINVAL, "the plan has open vertices: use tn_solve_open");
            continue;
        }
        tn_status s = TN_OK;
        st.raw = it.passes != nullptr;
        if (it.passes)
            st.passes = *it.passes;
        else
            s = make_passes(*it.net, it.opts, st.passes);
        if (s != TN_OK) {
            st.status = s;
            continue;
        }
        DevProgram* dp = nullptr;
        if (it.plan->nleaf() > 0) {
            s = get_program(ctx, *it.plan, dp);
            for (const PassSpec& ps : st.passes)
                if (s == TN_OK && (ps.dsr == DSR_TOPK || ps.dsr == DSR_TPOLY)) s = ensure_wide_perms(ctx, *it.plan, *dp);
            if (s != TN_OK) {
                st.status = s;
                continue;
            }
        }
        for (size_t p = 0; p < st.passes.size(); p++) {
            JobPlan jp{};
            jp.item = (int)i;
            jp.pass = (int)p;
            jp.plan = it.plan;
            jp.dsr = st.passes[p].dsr;
            jp.prime = st.passes[p].prime;
            jp.xval = st.passes[p].xval;
            jp.dp = dp;
            jp.ls = dp ? &node_launches(*dp, *it.plan, jp.dsr, true) : nullptr;
            jp.E = std::max<int64_t>(it.plan->arena_entries_dag, 64);
            jp.Pe = dp ? jp.ls->part_entries_dag : 0;
            int pb0 = plane_bytes(jp.dsr, 0), pb1 = plane_bytes(jp.dsr, 1);
            jp.o_arena0 = data;
            data = a256(data + (size_t)jp.E * pb0);
            jp.o_arena1 = data;
            data = a256(data + (size_t)jp.E * pb1);
            jp.o_part0 = data;
            data = a256(data + (size_t)jp.Pe * pb0);
            jp.o_part1 = data;
            data = a256(data + (size_t)jp.Pe * pb1);
            jp.o_meta = data;
            data = a256(data + sizeof(TensorMeta) * (size_t)std::max<size_t>(it.plan->nodes.size(), 1));
            st.job_ids.push_back((int)jobs.size());
            jobs.push_back(jp);
        }
    }
    L.njobs = (int)jobs.size();
    if (jobs.empty()) return TN_OK;
    {  // one kernel instance serves the wide-entry algebras, another the rest
        int nwide = 0;
        for (const JobPlan& jp : jobs) nwide += (jp.dsr == DSR_TOPK || jp.dsr == DSR_TPOLY) ? 1 : 0;
        if (nwide > 0 && nwide < (int)jobs.size())
            return fail(TN_EINVAL, "a persistent launch cannot mix the wide-entry algebras with the others");
        L.wide = nwide > 0 ? 1 : 0;
    }
    // every job's root accumulator slot, side by side: one read-back
    const size_t o_accs = data;
    for (size_t ji = 0; ji < jobs.size(); ji++) jobs[ji].o_acc = o_accs + kAccSlotBytes * ji;
    data = a256(data + kAccSlotBytes * jobs.size());
    L.data_bytes = std::max<size_t>(data, 256);
    L.data = alloc.alloc(L.data_bytes);
    if (!L.data) return fail(TN_ENOMEM, "device allocation of " + std::to_string(L.data_bytes) + " bytes failed");
    L.free_fn = alloc.free;
    unsigned char* dbase = (unsigned char*)L.data;

    // ---- task table
    std::vector<BJob> bj(jobs.size());
    std::vector<BNode> bn;
    std::vector<BTask> bt;
    int ncounters = 0;
    const int fuse_rank = small_rank(jobs.size(), device_cu_count(ctx) * 2);
    // workgroups one job template's tasks share in the schedule simulation:
    // one chiplet's, divided among the jobs its queue holds
    const int nq_sched = std::max(1, std::min(16, device_cu_count(ctx) / 32));
    const int jobs_per_q = (int)((jobs.size() + (size_t)nq_sched - 1) / (size_t)nq_sched);
    const int order_workers = std::max(1, device_cu_count(ctx) * 2 / nq_sched / std::max(1, jobs_per_q));
    // one template per (plan, algebra); the templates are independent of each
    // other, so a large launch builds them on several host threads
    std::map<std::pair<const Plan*, int>, JobTemplate> templates;
    {
        std::vector<std::pair<JobTemplate*, size_t>> todo;  // template, its first job
        for (size_t ji = 0; ji < jobs.size(); ji++) {
            auto ins = templates.emplace(std::make_pair(jobs[ji].plan, jobs[ji].dsr), JobTemplate());
            if (ins.second) todo.push_back({&ins.first->second, ji});
        }
        auto build = [&](size_t u) {
            JobTemplate& T = *todo[u].first;
            build_template(jobs[todo[u].second], fuse_rank, T);
            const std::vector<int> rank = earliest_start_order(T.bt, T.bn, T.subtree, T.ncounters, order_workers);
            T.order.assign(T.bt.size(), 0);
            for (size_t k = 0; k < rank.size(); k++) T.order[(size_t)rank[k]] = (int)k;
            T.work = 2.0e4 * (double)T.bt.size();
            for (auto& N : T.bn)
                T.work += std::exp2((double)(N.g.lb + N.g.li + N.g.lj + N.g.lk)) * (N.g.rm == 4 ? 0.5 : 1.0);
        };
        const size_t nthreads =
            todo.size() >= 32 ? std::min<size_t>(8, std::max(1u, std::thread::hardware_concurrency())) : 1;
        if (nthreads > 1) {
            std::atomic<size_t> next{0};
            std::vector<std::thread> pool;
            for (size_t w = 0; w < nthreads; w++)
                pool.emplace_back([&] {
                    for (size_t u = next++; u < todo.size(); u = next++) build(u);
                });
            for (auto& th : pool) th.join();
        } else {
            for (size_t u = 0; u < todo.size(); u++) build(u);
        }
    }
    std::vector<const JobTemplate*> job_tmpl(jobs.size(), nullptr);
    std::vector<int> job_task0(jobs.size(), 0);
    for (size_t ji = 0; ji < jobs.size(); ji++) {
        JobPlan& jp = jobs[ji];
        const Plan& p = *jp.plan;
        BJob& J = bj[ji];
        J.dsr = jp.dsr;
        J.nleaf = p.nleaf();
        J.nnode = (int)p.nodes.size();
        J.root = J.nnode - 1;
        J.ap = algebra_params(jp.dsr, jp.prime, items[jp.item].opts.beta, jp.xval);
        J.ap.fix_off = items[jp.item].net->fix_off;
        J.arena.p0 = dbase + jp.o_arena0;
        L.job_arena0.push_back(J.arena.p0);
        J.arena.p1 = plane_bytes(jp.dsr, 1) ? dbase + jp.o_arena1 : nullptr;
        J.part.p0 = dbase + jp.o_part0;
        J.part.p1 = plane_bytes(jp.dsr, 1) ? dbase + jp.o_part1 : nullptr;
        const bool isz = jp.dsr == DSR_Z_F32 || jp.dsr == DSR_Z_BF16;
        J.meta = isz ? (TensorMeta*)(dbase + jp.o_meta) : nullptr;
        J.acc = dbase + jp.o_acc;
        J.leaves = jp.dp ? jp.dp->leaves : nullptr;
        J.spos = jp.dp ? jp.dp->slice_pos : nullptr;
        J.w = items[jp.item].net->wdev.empty() ? nullptr : (const float*)(dbase + item_w_off[jp.item]);
        // the job's tasks: a copy of its template with ids shifted
        auto ti = templates.find(std::make_pair(jp.plan, jp.dsr));
        JobTemplate& T = ti->second;
        if (T.bn0 < 0) {  // nodes and subtree lists: once per template, shared by its jobs
            T.bn0 = (int)bn.size();
            T.sub0 = (int)L.subtree_list.size();
            bn.insert(bn.end(), T.bn.begin(), T.bn.end());
            for (int x : T.subtree) L.subtree_list.push_back(T.bn0 + x);
        }
        job_tmpl[ji] = &T;
        job_task0[ji] = (int)bt.size();
        const int bn0 = T.bn0, sub0 = T.sub0, c0 = ncounters;
        for (const BTask& t0 : T.bt) {
            BTask t = t0;
            t.job = (int)ji;
            if (t.kind == BT_PERM || t.kind == BT_GEMM || t.kind == BT_REDUCE) t.node += bn0;
            if (t.kind == BT_SUBTREE) t.node += sub0;
            if (t.dep0 >= 0) t.dep0 += c0;
            if (t.dep1 >= 0) t.dep1 += c0;
            if (t.signal >= 0) t.signal += c0;
            bt.push_back(t);
        }
        ncounters += T.ncounters;
        L.total_ops += T.ops;
        L.total_bytes += T.bytes;
    }
    clk.mark("templates", jobs.size());
    // every job goes to one XCC queue (longest-processing-time first on the
    // estimated work: semiring ops plus a fixed cost per task)
    const int nq = std::max(1, std::min(16, device_cu_count(ctx) / 32));
    std::vector<int> jq(jobs.size(), 0), jorder(jobs.size());
    for (size_t k = 0; k < jorder.size(); k++) jorder[k] = (int)k;
    std::stable_sort(jorder.begin(), jorder.end(),
                     [&](int a, int b) { return job_tmpl[a]->work > job_tmpl[b]->work; });
    std::vector<double> qload(nq, 0.0);
    for (int j : jorder) {
        int best = (int)(std::min_element(qload.begin(), qload.end()) - qload.begin());
        jq[j] = best;
        qload[best] += job_tmpl[j]->work;
    }
    // ticket order inside a queue.  Each job's tasks follow its template's
    // earliest-start-first order: every task has a rough cost (per-workgroup
    // rates) and a bottom level (its cost plus the longest chain of dependent
    // tasks after it); a simulation of the queue's workgroups hands the next
    // ticket to the task that can start first, the largest bottom level
    // among those ready.  The jobs of a queue are interleaved position by
    // position in proportion to their lengths, so every producer precedes its
    // consumers and a waiting workgroup only waits on smaller tickets of its
    // queue.
    std::vector<BTask> sorted;
    sorted.reserve(bt.size());
    std::vector<std::vector<int>> qjobs(nq);
    for (size_t j = 0; j < jobs.size(); j++) qjobs[jq[j]].push_back((int)j);
    for (int q = 0; q < nq; q++) {
        const std::vector<int>& J = qjobs[q];
        if (J.empty()) continue;
        bool same = true;
        for (int j : J) same = same && job_tmpl[j] == job_tmpl[J[0]];
        if (same) {
            const std::vector<int>& ord = job_tmpl[J[0]]->order;
            for (size_t k = 0; k < ord.size(); k++)
                for (int j : J) sorted.push_back(bt[(size_t)job_task0[j] + (size_t)ord[k]]);
            continue;
        }
        // different templates: a stable counting sort on the relative
        // position (k + 1/2) / length keeps every job's own order
        size_t nq_tasks = 0;
        for (int j : J) nq_tasks += job_tmpl[j]->order.size();
        std::vector<size_t> start(nq_tasks + 1, 0);
        auto bucket = [&](size_t k, size_t len) { return (size_t)(((double)k + 0.5) / (double)len * (double)nq_tasks); };
        for (int j : J) {
            const size_t len = job_tmpl[j]->order.size();
            for (size_t k = 0; k < len; k++) start[std::min(bucket(k, len), nq_tasks - 1) + 1]++;
        }
        for (size_t b = 0; b < nq_tasks; b++) start[b + 1] += start[b];
        std::vector<const BTask*> slot(nq_tasks);
        for (int j : J) {
            const std::vector<int>& ord = job_tmpl[j]->order;
            for (size_t k = 0; k < ord.size(); k++)
                slot[start[std::min(bucket(k, ord.size()), nq_tasks - 1)]++] = &bt[(size_t)job_task0[j] + (size_t)ord[k]];
        }
        for (const BTask* t : slot) sorted.push_back(*t);
    }
    L.ntasks = (int)sorted.size();
    L.nq = nq;
    L.qbegin.assign(nq, 0);
    L.qcount.assign(nq, 0);
    for (auto& t : sorted) L.qcount[jq[t.job]]++;
    for (int q = 1; q < nq; q++) L.qbegin[q] = L.qbegin[q - 1] + L.qcount[q - 1];
    if (ctx->profiling) L.host_tasks = sorted;

    clk.mark("queues", jobs.size());
    // ---- one upload: jobs | nodes | tasks | counters, tickets | subtrees |
    // qbegin, qcount | trace; then the weights
    size_t o_jobs = 0;
    size_t o_nodes = a256(o_jobs + sizeof(BJob) * bj.size());
    size_t o_tasks = a256(o_nodes + sizeof(BNode) * std::max<size_t>(bn.size(), 1));
    size_t o_cnt = a256(o_tasks + sizeof(BTask) * sorted.size());
    size_t o_tick = o_cnt + sizeof(int) * (size_t)ncounters;  // counters, tickets, abort flag: zero at every launch
    size_t o_sub = a256(o_tick + sizeof(int) * (size_t)(nq + 1));
    size_t o_q = a256(o_sub + sizeof(int) * std::max<size_t>(L.subtree_list.size(), 1));
    size_t o_trace = a256(o_q + sizeof(int) * 2 * (size_t)nq);
    size_t o_end = ctx->profiling ? a256(o_trace + 32 * sorted.size()) : o_trace;
    L.table_bytes = o_end;
    L.tables = alloc.alloc(L.table_bytes);
    if (!L.tables) return fail(TN_ENOMEM, "device allocation of the task table failed");
    size_t wbytes = weights_end;
    L.host_bytes = o_end + wbytes + kAccSlotBytes * jobs.size() + sizeof(int) * (nq + 1) + 1024;
    L.o_reset = o_cnt;
    L.reset_bytes = o_tick + sizeof(int) * (size_t)(nq + 1) - o_cnt;
    L.host = pinned_acquire(ctx, L.host_bytes);
    L.ctx = ctx;
    if (!L.host) return fail(TN_ENOMEM, "pinned staging allocation failed");
    unsigned char* h = (unsigned char*)L.host;
    std::memset(h, 0, o_end);
    std::memcpy(h + o_jobs, bj.data(), sizeof(BJob) * bj.size());
    if (!bn.empty()) std::memcpy(h + o_nodes, bn.data(), sizeof(BNode) * bn.size());
    std::memcpy(h + o_tasks, sorted.data(), sizeof(BTask) * sorted.size());
    if (!L.subtree_list.empty()) std::memcpy(h + o_sub, L.subtree_list.data(), sizeof(int) * L.subtree_list.size());
    std::memcpy(h + o_q, L.qbegin.data(), sizeof(int) * nq);
    std::memcpy(h + o_q + sizeof(int) * nq, L.qcount.data(), sizeof(int) * nq);
    unsigned char* d = (unsigned char*)L.tables;
    L.d_jobs = (BJob*)(d + o_jobs);
    L.d_nodes = (BNode*)(d + o_nodes);
    L.d_tasks = (BTask*)(d + o_tasks);
    L.d_counters = (int*)(d + o_cnt);
    L.d_ticket = (int*)(d + o_tick);
    L.d_subtree = (int*)(d + o_sub);
    L.d_qbegin = (int*)(d + o_q);
    L.d_qcount = L.d_qbegin + nq;
    L.d_trace = ctx->profiling ? (unsigned long long*)(d + o_trace) : nullptr;
    L.o_wstage = o_end;
    for (size_t i = 0; i < items.size(); i++)
        if (!items[i].net->wdev.empty())
            std::memcpy(h + o_end + item_w_off[i], items[i].net->wdev.data(), sizeof(float) * items[i].net->wdev.size());
    L.wbytes = wbytes;
    L.o_hacc = o_end + wbytes;
    L.o_hticket = a256(L.o_hacc + kAccSlotBytes * jobs.size());
    L.d_accs = dbase + o_accs;
    clk.mark("tables", jobs.size());
    return TN_OK;
}

// The context's wait limit in ticks of the device's constant wall clock.
long long wait_limit_ticks(tn_ctx* ctx) {
    if (ctx->wall_khz <= 0) {
        int khz = 0;
        if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, ctx->device) != hipSuccess || khz <= 0)
            khz = 100000;  // the 100 MHz clock of CDNA parts
        ctx->wall_khz = khz;
    }
    const double t = ctx->wait_limit_s * 1e3 * (double)ctx->wall_khz;
    return t < 1.0 ? 1 : (t > 9e18 ? (long long)9e18 : (long long)t);
}

tn_status batch_launch(tn_ctx* ctx, BatchLaunch& L, hipStream_t s) {
    if (L.njobs == 0) return TN_OK;
    hipError_t e = hipSuccess;
    if (!L.uploaded) {
        e = hipMemcpyAsync(L.tables, L.host, L.table_bytes, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && L.wbytes)
            e = hipMemcpyAsync(L.data, (unsigned char*)L.host + L.o_wstage, L.wbytes, hipMemcpyHostToDevice, s);
        L.uploaded = e == hipSuccess;
    } else {  // tables and weights are still in place: clear counters and tickets
        e = hipMemsetAsync((unsigned char*)L.tables + L.o_reset, 0, L.reset_bytes, s);
    }
    // two workgroups per CU: every XCC serves its queue
    int nwg = device_cu_count(ctx) * 2;
    if (e == hipSuccess) {
        int shape[4] = {0, 0, 0, 0};
        ProfScope ps(ctx, TN_K_BATCH, -1, -1, shape, L.total_bytes, L.total_ops,
                     L.wide ? "batch_kernel<true>" : "batch_kernel<false>");
        e = launch_batch(L.d_tasks, L.d_qbegin, L.d_qcount, L.nq, L.d_jobs, L.d_nodes, L.d_subtree, L.d_counters,
                         L.d_ticket, nwg, L.d_trace, L.wide, wait_limit_ticks(ctx), s);
    }
    // the tickets come back with the roots: a queue whose tickets did not all
    // go out was not served, and its jobs' results are not valid
    if (e == hipSuccess)
        e = hipMemcpyAsync((unsigned char*)L.host + L.o_hticket, L.d_ticket, sizeof(int) * (L.nq + 1),
                           hipMemcpyDeviceToHost, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync((unsigned char*)L.host + L.o_hacc, L.d_accs, kAccSlotBytes * (size_t)L.njobs, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return fail(TN_EDEVICE, std::string("batch launch failed: ") + hipGetErrorString(e));
    return TN_OK;
}

tn_status batch_finish(BatchLaunch& L, std::vector<tn_result>& out) {
    out.assign(L.items.size(), tn_result{});
    tn_status first = TN_OK;
    if (L.njobs > 0 && ((const int*)((unsigned char*)L.host + L.o_hticket))[L.nq] != 0)
        for (auto& st : L.items)
            if (st.status == TN_OK)
                st.status = fail(TN_EDEVICE, "a dependency wait of the persistent launch exceeded the context's wait "
                                             "limit; the launch was abandoned");
    for (int q = 0; q < L.nq && L.njobs > 0; q++) {
        int served = ((const int*)((unsigned char*)L.host + L.o_hticket))[q];
        if (L.qcount[q] > 0 && served < L.qcount[q]) {
            for (auto& st : L.items)
                if (st.status == TN_OK) st.status = fail(TN_EDEVICE, "a chiplet queue of the persistent launch was not served");
        }
    }
    for (size_t i = 0; i < L.items.size(); i++) {
        ItemState& st = L.items[i];
        tn_status s = st.status;
        if (s == TN_OK && st.raw) {
            out[i].semiring = -1;
            continue;
        }
        if (s == TN_OK) {
            std::vector<std::vector<unsigned char>> accs;
            for (int j : st.job_ids) {
                std::vector<unsigned char> a(kAccSlotBytes);
                std::memcpy(a.data(), (unsigned char*)L.host + L.o_hacc + kAccSlotBytes * j, kAccSlotBytes);
                accs.push_back(a);
            }
            s = decode_result(st.opts, st.passes, accs, out[i]);
        }
        if (s != TN_OK) {
            out[i].semiring = -1;
            if (first == TN_OK) first = s;
        }
        st.status = s;
    }
    return first;
}

void batch_release(BatchLaunch& L) {
    if (L.free_fn) {
        if (L.data) L.free_fn(L.data, L.data_bytes);
        if (L.tables) L.free_fn(L.tables, L.table_bytes);
    }
    if (L.host) pinned_release(L.ctx, L.host);
    L.data = L.tables = L.host = nullptr;
}

void collect_trace(tn_ctx* ctx, BatchLaunch& L) {
    std::vector<unsigned long long> tr(4 * (size_t)L.ntasks);
    if (hipMemcpy(tr.data(), L.d_trace, 32 * (size_t)L.ntasks, hipMemcpyDeviceToHost) != hipSuccess) return;
    unsigned long long t0 = ~0ull;
    for (int k = 0; k < L.ntasks; k++) t0 = std::min(t0, tr[4 * k]);
    const double us_per_tick = 0.01;  // wall_clock64 runs at 100 MHz
    for (int k = 0; k < L.ntasks; k++) {
        tn_task_record r;
        r.kind = L.host_tasks[k].kind;
        r.job = L.host_tasks[k].job;
        r.node = L.host_tasks[k].node;
        r.xcc = (int32_t)tr[4 * k + 3];
        r.t_start = (float)((tr[4 * k] - t0) * us_per_tick);
        r.t_ready = (float)((tr[4 * k + 1] - t0) * us_per_tick);
        r.t_end = (float)((tr[4 * k + 2] - t0) * us_per_tick);
        ctx->task_trace.push_back(r);
    }
}

// Identity of a synchronous batch: networks and plans by their unique ids,
// every option that changes what runs.
static std::vector<uint64_t> batch_key(const std::vector<BatchItem>& items) {
    std::vector<uint64_t> k;
    for (const BatchItem& it : items) {
        uint64_t beta;
        std::memcpy(&beta, &it.opts.beta, sizeof beta);
        k.insert(k.end(), {it.net->uid, it.plan->uid, (uint64_t)it.opts.semiring, beta, (uint64_t)it.opts.nprimes,
                           (uint64_t)it.opts.slice_begin, (uint64_t)it.opts.slice_end, (uint64_t)it.opts.executor});
        for (int q = 0; it.opts.primes && q < it.opts.nprimes; q++) k.push_back(it.opts.primes[q]);
        k.push_back(~0ull);
    }
    return k;
}

void batch_cache_drop(tn_ctx* ctx) {
    if (!ctx->batch_cache) return;
    batch_release(*ctx->batch_cache);
    delete ctx->batch_cache;
    ctx->batch_cache = nullptr;
    ctx->batch_cache_key.clear();
}

// Bump allocation in the context's grow-only scratch; what does not fit is
// allocated separately (and freed by scratch_regrow, which grows the scratch
// to the last call's need).
static DevAllocFn scratch_alloc(tn_ctx* ctx) {
    DevAllocFn alloc;
    ctx->batch_dev_used = 0;
    alloc.alloc = [ctx](size_t n) -> void* {
        n = (n + 255) & ~(size_t)255;
        ctx->batch_dev_peak = std::max(ctx->batch_dev_peak, ctx->batch_dev_used + n);
        if (ctx->batch_dev && ctx->batch_dev_used + n <= ctx->batch_dev_cap) {
            void* p = (unsigned char*)ctx->batch_dev + ctx->batch_dev_used;
            ctx->batch_dev_used += n;
            return p;
        }
        ctx->batch_dev_used += n;
        void* p = dev_alloc(ctx, n);
        if (p) ctx->batch_overflow.push_back({p, n});
        return p;
    };
    alloc.free = [](void*, size_t) {};
    return alloc;
}

static void scratch_regrow(tn_ctx* ctx) {
    if (ctx->batch_overflow.empty()) return;
    for (auto& b : ctx->batch_overflow) dev_free(ctx, b.first, b.second);
    ctx->batch_overflow.clear();
    if (ctx->batch_dev) dev_free(ctx, ctx->batch_dev, ctx->batch_dev_cap);
    ctx->batch_dev_cap = ctx->batch_dev_peak + (ctx->batch_dev_peak >> 3);
    ctx->batch_dev = dev_alloc(ctx, ctx->batch_dev_cap);
    if (!ctx->batch_dev) ctx->batch_dev_cap = 0;
}

tn_status solve_batch_sync(tn_ctx* ctx, std::vector<BatchItem>& items, std::vector<tn_result>& out) {
    auto t0 = std::chrono::steady_clock::now();
    // The same batch again (same networks, plans and options) reuses the last
    // launch's task table, weights and staging, which are still in place in
    // the context's scratch: only counters and tickets are cleared.
    std::vector<uint64_t> key = batch_key(items);
    if (ctx->batch_cache && !ctx->profiling && key == ctx->batch_cache_key) {
        BatchLaunch& C = *ctx->batch_cache;
        tn_status st = batch_launch(ctx, C, ctx->stream);
        if (st == TN_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = fail(TN_EDEVICE, "batch execution failed");
        if (st == TN_OK) st = batch_finish(C, out);
        if (st != TN_OK) batch_cache_drop(ctx);
        double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        for (auto& r : out) r.seconds = sec;
        return st;
    }
    batch_cache_drop(ctx);  // this call overwrites the scratch the cached launch lives in
    DevAllocFn alloc = scratch_alloc(ctx);
    BatchLaunch L;
    tn_status st = batch_prepare(ctx, items, L, alloc);
    if (st == TN_OK) st = batch_launch(ctx, L, ctx->stream);
    if (st == TN_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = fail(TN_EDEVICE, "batch execution failed");
    tn_status st2 = TN_OK;
    if (st == TN_OK) st2 = batch_finish(L, out);
    if (st == TN_OK && L.d_trace) collect_trace(ctx, L);
    if (L.host) (void)hipStreamSynchronize(ctx->stream);
    if (st == TN_OK && st2 == TN_OK && L.njobs > 0 && !L.d_trace && ctx->batch_overflow.empty()) {
        ctx->batch_cache = new BatchLaunch(std::move(L));
        ctx->batch_cache_key = std::move(key);
    } else {
        batch_release(L);
    }
    scratch_regrow(ctx);
    double sec = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    for (auto& r : out) r.seconds = sec;
    return st != TN_OK ? st : st2;
}

tn_status run_passes_sync(tn_ctx* ctx, const Net& net, const Plan& plan, const std::vector<PassSpec>& passes,
                          std::vector<std::array<unsigned char, kAccSlotBytes>>& accs) {
    BatchLaunch L;
    tn_status st = run_passes_keep(ctx, net, plan, passes, accs, L);
    batch_done(ctx, L);
    return st;
}

void batch_done(tn_ctx* ctx, BatchLaunch& L) {
    if (L.host) (void)hipStreamSynchronize(ctx->stream);
    batch_release(L);
    scratch_regrow(ctx);
}

tn_status run_passes_keep(tn_ctx* ctx, const Net& net, const Plan& plan, const std::vector<PassSpec>& passes,
                          std::vector<std::array<unsigned char, kAccSlotBytes>>& accs, BatchLaunch& L) {
    std::vector<BatchItem> items(1);
    items[0].net = &net;
    items[0].plan = &plan;
    items[0].opts = tn_solve_opts{};
    items[0].passes = &passes;
    batch_cache_drop(ctx);
    DevAllocFn alloc = scratch_alloc(ctx);
    tn_status st = batch_prepare(ctx, items, L, alloc);
    if (st == TN_OK) st = L.items[0].status;
    if (st == TN_OK) st = batch_launch(ctx, L, ctx->stream);
    if (st == TN_OK && hipStreamSynchronize(ctx->stream) != hipSuccess) st = fail(TN_EDEVICE, "batch execution failed");
    std::vector<tn_result> out;
    if (st == TN_OK) st = batch_finish(L, out);
    if (st == TN_OK && L.d_trace) collect_trace(ctx, L);
    if (st == TN_OK) {
        accs.assign(passes.size(), {});
        const std::vector<int>& ids = L.items[0].job_ids;
        for (size_t k = 0; k < ids.size() && k < accs.size(); k++)
            std::memcpy(accs[k].data(), (unsigned char*)L.host + L.o_hacc + kAccSlotBytes * (size_t)ids[k], kAccSlotBytes);
    }
    return st;
}

static int exec_mode() {  // TN_EXEC=stream | persistent forces a route (tests); -1: automatic
    static const int mode = [] {
        const char* e = std::getenv("TN_EXEC");
        return !e ? -1 : (std::strcmp(e, "stream") == 0 ? 0 : (std::strcmp(e, "persistent") == 0 ? 1 : -1));
    }();
    return mode;
}

bool use_persistent(const Plan& p) {
    if (!p.sliced.empty()) return false;
    if (exec_mode() >= 0) return exec_mode() == 1;
    // small trees: launch overhead dominates the per-node path.  A job of a
    // persistent launch runs on one chiplet, so trees with much work (more
    // than 2^27 semiring ops per pass) take the per-node path over the whole
    // chip instead.
    return p.max_rank <= 22 && p.tc <= 27.0;
}

bool use_persistent_shared(const Plan& p, int semiring) {
    if (use_persistent(p)) return true;
    if (exec_mode() >= 0 || !p.sliced.empty()) return false;
    // jobs launched together: mid-size trees of the exact algebras fill the
    // chiplets side by side (on the served mix, 2^27-2^29-op jobs ran three
    // times faster than one after the other on per-node launches, and
    // 2^29-2^31-op jobs 2.6 times faster), and their results do not depend on the
    // route: integer, modular and max-plus arithmetic are exact under any
    // tiling.  The real algebra keeps the single-job rule, so a Z job's sums
    // run in the same order alone and in any mix.
    const bool exact = semiring != TN_PARTITION_F32 && semiring != TN_PARTITION_BF16;
    return exact && p.max_rank <= 24 && p.tc <= 31.0;
}

}  // namespace tn
