// Independent-set network construction (Sec. 3.2) and leaf grouping.
#include <algorithm>
#include <cmath>

#include "plan.h"

namespace tn {

// The integer algebras (max-plus int32, counting tropical) need every size a
// configuration can reach within |size| <= 2^28: the sum of |weights| (of
// |couplings| and |fields| for a spin glass) bounds it.
static constexpr double kIntSizeBound = 268435456.0;

static double abs_sum(const std::vector<float>& w) {
    double s = 0;
    for (float x : w) s += std::fabs((double)x);
    return s;
}


static thread_local std::string g_last_error;

void set_error(const std::string& msg) { g_last_error = msg; }
tn_status fail(tn_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}
const char* last_error_cstr() { return g_last_error.c_str(); }

tn_status make_net(int nv, int ne, const int32_t* edges, const float* weights, Net& out) {
    if (nv < 0 || ne < 0) return fail(TN_EINVAL, "negative vertex or edge count");
    if (nv > 4096) return fail(TN_EINVAL, "at most 4096 vertices are supported");
    if (ne > 0 && !edges) return fail(TN_EINVAL, "edges is NULL");
    out = Net();
    out.nv = nv;
    out.edges.reserve((size_t)ne);
    for (int e = 0; e < ne; e++) {
        int u = edges[2 * e], v = edges[2 * e + 1];
        if (u < 0 || v < 0 || u >= nv || v >= nv)
            return fail(TN_EINVAL, "edge " + std::to_string(e) + " has a vertex id out of range");
        if (u == v) return fail(TN_EINVAL, "self-loop at vertex " + std::to_string(u));
        out.edges.push_back({std::min(u, v), std::max(u, v)});
    }
    // merge duplicates, keeping the first occurrence so edge ids follow the input order
    {
        std::vector<std::array<int, 2>> sorted = out.edges, kept;
        std::sort(sorted.begin(), sorted.end());
        std::vector<char> used(sorted.size(), 0);
        for (auto& e : out.edges) {
            size_t k = (size_t)(std::lower_bound(sorted.begin(), sorted.end(), e) - sorted.begin());
            if (used[k]) continue;
            used[k] = 1;
            kept.push_back(e);
        }
        out.edges.swap(kept);
    }
    if (weights) {
        out.w.assign(weights, weights + nv);
        for (int v = 0; v < nv; v++) {
            if (!std::isfinite(out.w[v])) return fail(TN_EINVAL, "non-finite weight");
            if (out.w[v] != std::nearbyint(out.w[v]) || std::fabs(out.w[v]) > 65536.0f)
                out.integer_weights = false;
        }
        if (abs_sum(out.w) > kIntSizeBound) out.integer_weights = false;
    }
    // FNV-1a over the structure, so a plan can check it belongs to this network
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](uint64_t x) {
        for (int k = 0; k < 8; k++) {
            h ^= (x >> (8 * k)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    mix((uint64_t)nv);
    for (auto& e : out.edges) mix(((uint64_t)e[0] << 32) | (uint32_t)e[1]);
    out.fingerprint = h;
    set_dev_weights(out);
    return TN_OK;
}

void set_dev_weights(Net& net) {
    net.wdev = net.w;
    net.fix_off = -1;
    if (net.fix.empty()) return;
    if (net.wdev.empty()) net.wdev.assign((size_t)net.nv, 1.0f);
    net.fix_off = (int)net.wdev.size();
    for (int v = 0; v < net.nv; v++) net.wdev.push_back((float)net.fix[v]);
}

tn_status condition_net(const Net& src, int n, const int32_t* vertices, const int32_t* values, Net& out) {
    if (n < 0 || (n > 0 && (!vertices || !values))) return fail(TN_EINVAL, "vertices and values are required");
    std::vector<signed char> fix = src.fix.empty() ? std::vector<signed char>((size_t)src.nv, -1) : src.fix;
    for (int k = 0; k < n; k++) {
        const int v = vertices[k], x = values[k];
        if (v < 0 || v >= src.nv) return fail(TN_EINVAL, "fixed vertex " + std::to_string(v) + " out of range");
        if (x != 0 && x != 1) return fail(TN_EINVAL, "a fixed vertex takes the value 0 or 1");
        if (fix[v] >= 0 && fix[v] != x)
            return fail(TN_EINVAL, "vertex " + std::to_string(v) + " is fixed to both values");
        fix[v] = (signed char)x;
    }
    out = src;
    out.fix = fix;
    set_dev_weights(out);
    return TN_OK;
}

tn_status make_spin_glass(int nv, int ne, const int32_t* edges, const float* J, const float* h, Net& out) {
    tn_status st = make_net(nv, ne, edges, nullptr, out);
    if (st != TN_OK) return st;
    out.kind = 1;
    out.w.assign((size_t)nv + out.edges.size(), 0.0f);
    for (int v = 0; v < nv; v++) out.w[v] = h ? h[v] : 0.0f;
    std::vector<std::array<int, 2>> sorted = out.edges;  // kept edge id of every input edge
    std::vector<int> id(sorted.size());
    std::sort(sorted.begin(), sorted.end());
    for (size_t k = 0; k < out.edges.size(); k++)
        id[(size_t)(std::lower_bound(sorted.begin(), sorted.end(), out.edges[k]) - sorted.begin())] = (int)k;
    for (int e = 0; e < ne; e++) {
        std::array<int, 2> key{std::min(edges[2 * e], edges[2 * e + 1]), std::max(edges[2 * e], edges[2 * e + 1])};
        int k = id[(size_t)(std::lower_bound(sorted.begin(), sorted.end(), key) - sorted.begin())];
        out.w[(size_t)nv + k] += J ? J[e] : 1.0f;
    }
    out.integer_weights = true;
    for (float x : out.w) {
        if (!std::isfinite(x)) return fail(TN_EINVAL, "non-finite coupling or field");
        if (x != std::nearbyint(x) || std::fabs(x) > 65536.0f) out.integer_weights = false;
    }
    if (abs_sum(out.w) > kIntSizeBound) out.integer_weights = false;
    out.fingerprint = out.fingerprint * 1099511628211ull ^ 0x5397u;  // a spin glass differs from an IS network
    set_dev_weights(out);
    return TN_OK;
}

std::vector<Leaf> make_leaves(const Net& net, bool absorb) {
    std::vector<Leaf> leaves;
    std::vector<int> first(net.nv, -1);
    for (int e = 0; e < (int)net.edges.size(); e++) {
        Leaf l;
        l.factors.push_back(e);
        l.scope = {net.edges[e][0], net.edges[e][1]};
        for (int k = 0; k < 2; k++)
            if (first[net.edges[e][k]] < 0) first[net.edges[e][k]] = e;
        leaves.push_back(l);
    }
    for (int v = 0; v < net.nv; v++) {
        if (absorb && first[v] >= 0) {
            leaves[first[v]].factors.push_back(-v - 1);
        } else {
            Leaf l;
            l.factors.push_back(-v - 1);
            l.scope = {v};
            leaves.push_back(l);
        }
    }
    return leaves;
}

void flat_complexity(const Net& net, double& tc, double& sc, double& rwc) {
    // one node over every index: each edge tensor (rank 2) and vertex tensor
    // (rank 1) is read once and the scalar output written once
    tc = (double)net.nv;
    sc = 0.0;
    double rw = 4.0 * (double)net.edges.size() + 2.0 * (double)net.nv + 1.0;
    rwc = std::log2(rw);
}

}  // namespace tn
