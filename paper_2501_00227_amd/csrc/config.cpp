// One maximum configuration (the SingleConfigMax property of the Sec. 5
// table).  The max-plus float32 contraction runs once on the persistent
// executor in its dependency-graph layout, where every tensor of the tree
// keeps its own region, and stays resident; a one-workgroup kernel then
// walks the tree from the root and fixes, at every inner node, the summed
// indices to values whose two operand entries add up to the node's entry
// (the back-tracking reading of the tropical contraction, Sec. 5.1).  Indices
// that a leaf sums by itself (a vertex seen by one leaf only) are set on the
// host to the best value of that leaf's factors.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "batch_host.h"
#include "kernels.h"

namespace tn {

namespace {

// The leaf's factor product (a sum in max-plus) at the given vertex values.
double leaf_value(const Net& net, const Plan& plan, const Leaf& leaf, const std::vector<int>& cfg) {
    if (!net.fix.empty())
        for (int v : leaf.scope)
            if (net.fix[v] >= 0 && cfg[v] != net.fix[v]) return -INFINITY;
    double s = 0;
    for (int f : leaf.factors) {
        if (f >= 0) {
            const int u = plan.edges[f][0], v = plan.edges[f][1];
            if (net.kind == 1) {
                const double J = net.w[net.nv + f];
                s -= J * (2 * cfg[u] - 1) * (2 * cfg[v] - 1);
            } else if (cfg[u] && cfg[v]) {
                return -INFINITY;
            }
        } else {
            const int v = -f - 1;
            if (net.kind == 1)
                s -= (double)net.w[v] * (2 * cfg[v] - 1);
            else
                s += cfg[v] ? (net.w.empty() ? 1.0 : (double)net.w[v]) : 0.0;
        }
    }
    return s;
}

}  // namespace

tn_status single_config_max(tn_ctx* ctx, const Net& net, const Plan& plan, int32_t* config, float* value) {
    if (!config && net.nv > 0) return fail(TN_EINVAL, "config must hold nv entries");
    if (!plan.sliced.empty()) return fail(TN_EINVAL, "a maximum configuration needs an unsliced plan");
    if (plan.fingerprint != net.fingerprint || plan.nv != net.nv)
        return fail(TN_EINVAL, "plan was built for a different network");
    std::vector<int> cfg(net.nv, -1);
    float root = 0.0f;
    const int nleaf = plan.nleaf(), ninner = plan.ninner();
    if (nleaf > 0) {
        std::vector<PassSpec> passes(1);
        passes[0].dsr = DSR_TROP_F32;
        std::vector<std::array<unsigned char, kAccSlotBytes>> accs;
        BatchLaunch L;
        tn_status st = run_passes_keep(ctx, net, plan, passes, accs, L);
        if (st == TN_OK) std::memcpy(&root, accs[0].data(), 4);
        if (st == TN_OK && std::isinf(root) && root < 0)
            st = fail(TN_EINVAL, "no configuration satisfies the fixed vertices");
        if (st == TN_OK && ninner > 0) {
            // tables: inner nodes, storage orders, offsets; then assign, status
            const int nn = (int)plan.nodes.size();
            std::vector<int> nodes(3 * (size_t)ninner), ord_off(nn + 1, 0), ord_ids;
            for (int t = 0; t < ninner; t++) {
                nodes[3 * t] = plan.prog[t].node;
                nodes[3 * t + 1] = plan.prog[t].a;
                nodes[3 * t + 2] = plan.prog[t].b;
            }
            for (int x = 0; x < nn; x++) {
                ord_off[x] = (int)ord_ids.size();
                ord_ids.insert(ord_ids.end(), plan.order[x].begin(), plan.order[x].end());
            }
            ord_off[nn] = (int)ord_ids.size();
            std::vector<long long> off(plan.node_off_dag.begin(), plan.node_off_dag.end());
            // inner nodes by depth from the root: a node's output indices are
            // fixed once its parent is done, so each level runs in parallel
            std::vector<int> t_of(nn, -1), depth(ninner, 0);
            for (int t = 0; t < ninner; t++) t_of[plan.prog[t].node] = t;
            int nlevels = 0;
            for (int t = ninner - 1; t >= 0; t--) {  // parents come after their children
                nlevels = std::max(nlevels, depth[t] + 1);
                for (int c : {plan.prog[t].a, plan.prog[t].b})
                    if (t_of[c] >= 0) depth[t_of[c]] = depth[t] + 1;
            }
            std::vector<int> lvl_off(nlevels + 1, 0), lvl_nodes(ninner);
            for (int t = 0; t < ninner; t++) lvl_off[depth[t] + 1]++;
            for (int l = 0; l < nlevels; l++) lvl_off[l + 1] += lvl_off[l];
            {
                std::vector<int> fill(lvl_off.begin(), lvl_off.end() - 1);
                for (int t = ninner - 1; t >= 0; t--) lvl_nodes[fill[depth[t]]++] = t;
            }
            const size_t b_nodes = nodes.size() * 4, b_ooff = ord_off.size() * 4, b_oids = ord_ids.size() * 4 + 4,
                         b_off = off.size() * 8, b_loff = lvl_off.size() * 4, b_lnod = lvl_nodes.size() * 4,
                         b_asg = (size_t)net.nv * 4 + 4;
            const size_t o_ooff = (b_nodes + 15) & ~(size_t)15, o_oids = (o_ooff + b_ooff + 15) & ~(size_t)15,
                         o_off = (o_oids + b_oids + 15) & ~(size_t)15, o_loff = (o_off + b_off + 15) & ~(size_t)15,
                         o_lnod = (o_loff + b_loff + 15) & ~(size_t)15, o_asg = (o_lnod + b_lnod + 15) & ~(size_t)15,
                         o_stat = (o_asg + b_asg + 15) & ~(size_t)15, total = o_stat + 16;
            std::vector<unsigned char> host(total, 0);
            std::memcpy(host.data(), nodes.data(), b_nodes);
            std::memcpy(host.data() + o_ooff, ord_off.data(), b_ooff);
            if (!ord_ids.empty()) std::memcpy(host.data() + o_oids, ord_ids.data(), ord_ids.size() * 4);
            std::memcpy(host.data() + o_off, off.data(), b_off);
            std::memcpy(host.data() + o_loff, lvl_off.data(), b_loff);
            std::memcpy(host.data() + o_lnod, lvl_nodes.data(), b_lnod);
            std::memset(host.data() + o_asg, 0xff, (size_t)net.nv * 4);  // -1: unset
            unsigned char* d = nullptr;
            if (hipMalloc(&d, total) != hipSuccess) {
                st = fail(TN_ENOMEM, "back-trace tables");
            } else {
                int status = 0;
                hipStream_t s = ctx->stream;
                if (hipMemcpyAsync(d, host.data(), total, hipMemcpyHostToDevice, s) != hipSuccess ||
                    launch_backtrace((const float*)L.job_arena0[0], (const int*)d, ninner, (const int*)(d + o_ooff),
                                     (const int*)(d + o_oids), (const long long*)(d + o_off),
                                     (const int*)(d + o_loff), (const int*)(d + o_lnod), nlevels, (int*)(d + o_asg),
                                     (int*)(d + o_stat), nn, (int)ord_ids.size(), net.nv, s) != hipSuccess ||
                    hipMemcpyAsync(host.data() + o_asg, d + o_asg, total - o_asg, hipMemcpyDeviceToHost, s) != hipSuccess ||
                    hipStreamSynchronize(s) != hipSuccess) {
                    st = fail(TN_EDEVICE, "back-trace kernel failed");
                } else {
                    std::memcpy(&status, host.data() + o_stat, 4);
                    std::memcpy(cfg.data(), host.data() + o_asg, (size_t)net.nv * 4);
                    if (status == 2)
                        st = fail(TN_ETOOBIG, "a node sums more than 30 indices (or has rank > 62) in the back-trace");
                    else if (status != 0)
                        st = fail(TN_EDEVICE, "back-trace found no matching assignment");
                }
                (void)hipFree(d);
            }
        }
        batch_done(ctx, L);
        if (st != TN_OK) return st;
    }
    // vertices summed inside a leaf: the best value for that leaf alone
    for (const Leaf& leaf : plan.leaves) {
        std::vector<int> open;
        for (int v : leaf.scope)
            if (cfg[v] < 0) open.push_back(v);
        if (open.empty()) continue;
        double best = -INFINITY;
        int pick = 0;
        for (int m = 0; m < (1 << open.size()); m++) {
            for (size_t q = 0; q < open.size(); q++) cfg[open[q]] = (m >> q) & 1;
            const double v = leaf_value(net, plan, leaf, cfg);
            if (v > best) {
                best = v;
                pick = m;
            }
        }
        for (size_t q = 0; q < open.size(); q++) cfg[open[q]] = (pick >> q) & 1;
    }
    // every vertex set; for independent sets the result must be independent
    for (int v = 0; v < net.nv; v++)
        if (cfg[v] < 0) return fail(TN_EDEVICE, "back-trace left a vertex unset");
    if (net.kind == 0)
        for (const auto& e : plan.edges)
            if (cfg[e[0]] && cfg[e[1]]) return fail(TN_EDEVICE, "back-trace produced a dependent set");
    for (size_t v = 0; v < net.fix.size(); v++)
        if (net.fix[v] >= 0 && cfg[v] != net.fix[v]) return fail(TN_EDEVICE, "back-trace broke a fixed vertex");
    for (int v = 0; v < net.nv; v++) config[v] = cfg[v];
    if (value) *value = root;
    return TN_OK;
}

}  // namespace tn
