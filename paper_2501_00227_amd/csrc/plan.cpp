// Plan assembly: tree in execution order, complexity (Sec. 4.1), operand
// layouts for the permute + batched-GEMM executor, and the memory plan.
#include <algorithm>
#include <cmath>
#include <functional>
#include <map>

#include "plan.h"

namespace tn {

tn_status optimize_tree(const Net& net, const std::vector<Leaf>& leaves, const PlanOptions& o,
                        std::vector<int>& L, std::vector<int>& R, std::vector<int>& sliced);

namespace {

std::vector<int> set_union(const std::vector<int>& a, const std::vector<int>& b) {
    std::vector<int> r;
    std::set_union(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
    return r;
}
std::vector<int> set_inter(const std::vector<int>& a, const std::vector<int>& b) {
    std::vector<int> r;
    std::set_intersection(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
    return r;
}
std::vector<int> set_minus(const std::vector<int>& a, const std::vector<int>& b) {
    std::vector<int> r;
    std::set_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
    return r;
}
bool has(const std::vector<int>& a, int x) { return std::binary_search(a.begin(), a.end(), x); }

// Validate a tree and fill node outputs by the einsum rule.  Nodes are given
// with leaves first and inner nodes whose children have smaller ids.  Open
// vertices count as held by the output as well, so they stay to the root.
tn_status build_nodes(const Net& net, const std::vector<Leaf>& leaves, const std::vector<int>& left,
                      const std::vector<int>& right, std::vector<Node>& nodes, const std::vector<int>& open = {}) {
    int nleaf = (int)leaves.size();
    int ninner = (int)left.size();
    if (nleaf < 1) return fail(TN_EINVAL, "a plan needs at least one leaf");
    if ((int)right.size() != ninner || ninner != nleaf - 1)
        return fail(TN_EINVAL, "a binary tree over n leaves has n-1 inner nodes");
    // every factor exactly once
    std::vector<int> seen(net.edges.size() + net.nv, 0);
    for (auto& l : leaves)
        for (int f : l.factors) {
            if (f >= (int)net.edges.size() || -f - 1 >= net.nv)
                return fail(TN_EINVAL, "leaf factor out of range");
            seen[f >= 0 ? f : (int)net.edges.size() + (-f - 1)]++;
        }
    for (int s : seen)
        if (s != 1) return fail(TN_EINVAL, "every edge and vertex tensor must occur in exactly one leaf");
    int nn = nleaf + ninner;
    std::vector<int> parent(nn, -1);
    for (int t = 0; t < ninner; t++) {
        int x = nleaf + t;
        if (left[t] < 0 || right[t] < 0 || left[t] >= x || right[t] >= x || left[t] == right[t])
            return fail(TN_EINVAL, "inner node children must be distinct earlier nodes");
        if (parent[left[t]] >= 0 || parent[right[t]] >= 0)
            return fail(TN_EINVAL, "a node is used twice in the tree");
        parent[left[t]] = parent[right[t]] = x;
    }
    for (int x = 0; x + 1 < nn; x++)
        if (parent[x] < 0) return fail(TN_EINVAL, "tree is not connected");
    // occurrences of each index over the leaves' scopes
    std::vector<int> total(net.nv, 0);
    for (auto& l : leaves)
        for (int x : l.scope) total[x]++;
    for (int v : open) total[v]++;
    nodes.assign(nn, Node());
    std::vector<std::map<int, int>> cnt(nn);
    for (int x = 0; x < nn; x++) {
        if (x < nleaf) {
            for (int v : leaves[x].scope) cnt[x][v] = 1;
        } else {
            int a = left[x - nleaf], b = right[x - nleaf];
            nodes[x].left = a;
            nodes[x].right = b;
            cnt[x] = cnt[a];
            for (auto& [v, c] : cnt[b]) cnt[x][v] += c;
            cnt[a].clear();
            cnt[b].clear();
        }
        for (auto& [v, c] : cnt[x])
            if (c < total[v]) nodes[x].out.push_back(v);
    }
    std::vector<int> want = open;
    std::sort(want.begin(), want.end());
    if (nodes.back().out != want) return fail(TN_EINVAL, "root keeps open indices");
    return TN_OK;
}

// Reorder inner nodes so that at every node the child subtree that needs
// more live memory runs first (fewer simultaneously live intermediates).
void reorder_for_memory(std::vector<Node>& nodes, int nleaf, const std::vector<char>& sl) {
    int nn = (int)nodes.size();
    auto rank = [&](int x) {
        int r = 0;
        for (int v : nodes[x].out) r += !sl[v];
        return r;
    };
    std::vector<double> need(nn, 0.0), size(nn, 0.0);
    for (int x = 0; x < nn; x++) {
        size[x] = x < nleaf ? 0.0 : std::exp2((double)rank(x));
        if (x < nleaf) continue;
        int a = nodes[x].left, b = nodes[x].right;
        double ab = std::max(need[a], size[a] + need[b]);
        double ba = std::max(need[b], size[b] + need[a]);
        if (ba < ab) std::swap(nodes[x].left, nodes[x].right);
        a = nodes[x].left;
        b = nodes[x].right;
        need[x] = std::max({need[a], size[a] + need[b], size[a] + size[b] + size[x]});
    }
    // post-order renumbering
    std::vector<int> id(nn, -1), post;
    for (int x = 0; x < nleaf; x++) id[x] = x;
    std::vector<std::pair<int, int>> st{{nn - 1, 0}};
    while (!st.empty()) {
        auto& [n, s] = st.back();
        if (n < nleaf || s == 2) {
            if (n >= nleaf) post.push_back(n);
            st.pop_back();
            continue;
        }
        int c = s == 0 ? nodes[n].left : nodes[n].right;
        s++;
        st.push_back({c, 0});
    }
    int next = nleaf;
    for (int n : post) id[n] = next++;
    std::vector<Node> nn2(nn);
    for (int x = 0; x < nleaf; x++) nn2[x] = nodes[x];
    for (int n : post) {
        Node m = nodes[n];
        m.left = id[m.left];
        m.right = id[m.right];
        nn2[id[n]] = m;
    }
    nodes.swap(nn2);
}

// First-fit allocator over an abstract arena of entries.
struct Arena {
    std::map<int64_t, int64_t> free_;  // offset -> size
    int64_t end = 0, peak = 0;
    static int64_t align(int64_t x) { return (x + 63) & ~(int64_t)63; }
    int64_t alloc(int64_t n) {
        n = align(std::max<int64_t>(n, 1));
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                int64_t off = it->first, sz = it->second;
                free_.erase(it);
                if (sz > n) free_[off + n] = sz - n;
                return off;
            }
        }
        // extend, reusing a free block that touches the end
        int64_t off = end;
        if (!free_.empty()) {
            auto last = std::prev(free_.end());
            if (last->first + last->second == end) {
                off = last->first;
                free_.erase(last);
            }
        }
        end = off + n;
        peak = std::max(peak, end);
        return off;
    }
    void release(int64_t off, int64_t n) {
        n = align(std::max<int64_t>(n, 1));
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
                it = pv;
            }
        }
        if (it->first + it->second == end) {
            end = it->first;
            free_.erase(it);
        }
    }
};

// Is C (storage order `ord`) directly usable by its parent, whose operand
// groups are: batch indices `pb` (must be the top bits) and the two other
// groups `pk`, `pf` (each contiguous, in either order below the batch)?
bool parent_compatible(const std::vector<int>& ord, const std::vector<int>& pb, const std::vector<int>& pk) {
    int r = (int)ord.size(), nb = (int)pb.size();
    for (int q = r - nb; q < r; q++)
        if (!has(pb, ord[q])) return false;
    // below the batch: runs of k and non-k; at most 2 runs
    int runs = 0;
    int prev = -1;
    for (int q = 0; q < r - nb; q++) {
        int g = has(pk, ord[q]) ? 1 : 0;
        if (g != prev) {
            runs++;
            prev = g;
        }
    }
    return runs <= 2;
}

}  // namespace

void plan_complexity(Plan& p) {
    std::vector<char> sl(p.nv, 0);
    for (int x : p.sliced) sl[x] = 1;
    auto rank = [&](const std::vector<int>& v) {
        int r = 0;
        for (int x : v) r += !sl[x];
        return r;
    };
    double tc = -1.0 / 0.0, rw = -1.0 / 0.0;
    int sc = 0;
    int nleaf = p.nleaf();
    for (int x = nleaf; x < (int)p.nodes.size(); x++) {
        const Node& n = p.nodes[x];
        auto u = set_union(p.nodes[n.left].out, p.nodes[n.right].out);
        int ra = rank(p.nodes[n.left].out), rb = rank(p.nodes[n.right].out), rc = rank(n.out);
        tc = log2_add(tc, (double)rank(u));
        rw = log2_add(rw, log2_add(log2_add((double)ra, (double)rb), (double)rc));
        sc = std::max(sc, rc);
    }
    if (p.nodes.size() == (size_t)nleaf) {  // a single leaf: nothing to contract
        tc = 0;
        rw = 0;
    }
    p.tc = tc + (double)p.sliced.size();
    p.rwc = rw + (double)p.sliced.size();
    p.sc = (double)sc;
    p.max_rank = sc;
}

tn_status plan_program(Plan& p) {
    int nleaf = p.nleaf();
    int nn = (int)p.nodes.size();
    std::vector<char> sl(p.nv, 0);
    for (int x : p.sliced) sl[x] = 1;
    auto kept = [&](int x) {
        std::vector<int> r;
        for (int v : p.nodes[x].out)
            if (!sl[v]) r.push_back(v);
        return r;
    };
    std::vector<int> parent(nn, -1);
    for (int x = nleaf; x < nn; x++) parent[p.nodes[x].left] = parent[p.nodes[x].right] = x;
    p.order.assign(nn, {});
    std::vector<char> decided(nn, 0);
    p.prog.clear();
    p.npermutes = 0;

    // leaves: fixed slots of 4 entries (rank <= 2)
    p.leaf_prog.assign(nleaf, LeafProg());
    for (int l = 0; l < nleaf; l++) {
        LeafProg& lp = p.leaf_prog[l];
        for (int f : p.leaves[l].factors) {
            if (f >= 0) {
                lp.has_edge = 1;
                lp.edge = f;
                lp.u = p.edges[f][0];
                lp.v = p.edges[f][1];
            }
        }
        for (int f : p.leaves[l].factors) {
            if (f < 0) {
                int v = -f - 1;
                if (!lp.has_edge) {
                    lp.u = v;
                    lp.wu = 1;
                } else if (v == lp.u) {
                    lp.wu = 1;
                } else {
                    lp.wv = 1;
                }
            }
        }
        lp.off = 4 * (int64_t)l;
    }
    p.leaf_entries = 4 * (int64_t)nleaf;

    Arena arena;
    arena.end = arena.peak = Arena::align(p.leaf_entries);
    std::vector<int64_t> off(nn, -1), dag_off(nn, -1);
    for (int l = 0; l < nleaf; l++) off[l] = dag_off[l] = p.leaf_prog[l].off;
    int64_t dag_end = Arena::align(p.leaf_entries);

    for (int x = nleaf; x < nn; x++) {
        const Node& nd = p.nodes[x];
        std::vector<int> A0 = kept(nd.left), B0 = kept(nd.right), C = kept(x);
        NodeProg best;
        double best_cost = 1.0 / 0.0;
        std::vector<int> best_ord_c, best_req_a, best_req_b;
        for (int swap = 0; swap < 2; swap++) {
            int a = swap ? nd.right : nd.left, b = swap ? nd.left : nd.right;
            const std::vector<int>& Aset = swap ? B0 : A0;
            const std::vector<int>& Bset = swap ? A0 : B0;
            std::vector<int> gb = set_inter(set_inter(Aset, Bset), C);
            std::vector<int> gk = set_minus(set_inter(Aset, Bset), C);
            std::vector<int> gi = set_minus(Aset, Bset);
            std::vector<int> gj = set_minus(Bset, Aset);
            // order of a group as it appears in a tensor's storage (bit 0 up)
            auto in_order = [&](const std::vector<int>& g, int t) {
                if (!decided[t]) return g;
                std::vector<int> r;
                for (int v : p.order[t])
                    if (has(g, v)) r.push_back(v);
                return r;
            };
            for (int ksrc = 0; ksrc < 2; ksrc++)
                for (int bsrc = 0; bsrc < 2; bsrc++)
                    for (int at = 0; at < 2; at++)
                        for (int bt = 0; bt < 2; bt++) {
                            auto ko = in_order(gk, ksrc ? b : a);
                            auto bo = in_order(gb, bsrc ? b : a);
                            auto io = in_order(gi, a);
                            auto jo = in_order(gj, b);
                            std::vector<int> ra, rb, rc;
                            // A: [b][i][k] (k fastest) or [b][k][i]
                            if (at) {
                                ra = io;
                                ra.insert(ra.end(), ko.begin(), ko.end());
                            } else {
                                ra = ko;
                                ra.insert(ra.end(), io.begin(), io.end());
                            }
                            ra.insert(ra.end(), bo.begin(), bo.end());
                            // B: [b][k][j] (j fastest) or [b][j][k]
                            if (bt) {
                                rb = ko;
                                rb.insert(rb.end(), jo.begin(), jo.end());
                            } else {
                                rb = jo;
                                rb.insert(rb.end(), ko.begin(), ko.end());
                            }
                            rb.insert(rb.end(), bo.begin(), bo.end());
                            rc = jo;
                            rc.insert(rc.end(), io.begin(), io.end());
                            rc.insert(rc.end(), bo.begin(), bo.end());
                            bool pa = a >= nleaf && p.order[a] != ra;
                            bool pb = b >= nleaf && p.order[b] != rb;
                            double cost = (pa ? 2.0 * std::exp2((double)ra.size()) : 0.0) +
                                          (pb ? 2.0 * std::exp2((double)rb.size()) : 0.0);
                            int par = parent[x];
                            if (par >= 0) {
                                int sib = p.nodes[par].left == x ? p.nodes[par].right : p.nodes[par].left;
                                auto S = kept(sib), Pout = kept(par);
                                auto pbg = set_inter(set_inter(C, S), Pout);
                                auto pkg = set_minus(set_inter(C, S), Pout);
                                if (!parent_compatible(rc, pbg, pkg)) cost += std::exp2((double)rc.size());
                            }
                            // mild preference for transposition-free kernels
                            cost += 1e-3 * (at + bt);
                            if (cost < best_cost) {
                                best_cost = cost;
                                best = NodeProg();
                                best.node = x;
                                best.a = a;
                                best.b = b;
                                best.perm_a = pa;
                                best.perm_b = pb;
                                best.lb = (int)gb.size();
                                best.li = (int)gi.size();
                                best.lj = (int)gj.size();
                                best.lk = (int)gk.size();
                                best.a_t = at;
                                best.b_t = bt;
                                best_ord_c = rc;
                                best_req_a = ra;
                                best_req_b = rb;
                            }
                        }
        }
        // permutation tables: output bit q takes input bit src[q]
        auto perm_src = [&](const std::vector<int>& cur, const std::vector<int>& req) {
            std::vector<int> src(req.size());
            for (size_t q = 0; q < req.size(); q++)
                src[q] = (int)(std::find(cur.begin(), cur.end(), req[q]) - cur.begin());
            return src;
        };
        for (int side = 0; side < 2; side++) {
            int t = side ? best.b : best.a;
            const auto& req = side ? best_req_b : best_req_a;
            if (t < nleaf) {  // leaves are written in whatever order the node wants
                p.order[t] = req;
                decided[t] = 1;
                LeafProg& lp = p.leaf_prog[t];
                lp.rank = (int)req.size();
                lp.var[0] = req.size() > 0 ? req[0] : -1;
                lp.var[1] = req.size() > 1 ? req[1] : -1;
            }
        }
        if (best.perm_a) best.perm_a_src = perm_src(p.order[best.a], best_req_a);
        if (best.perm_b) best.perm_b_src = perm_src(p.order[best.b], best_req_b);
        p.npermutes += (int)best.perm_a + (int)best.perm_b;
        p.order[x] = best_ord_c;
        decided[x] = 1;

        // memory: temporaries for permuted operands, then C, then free
        int64_t sa = (int64_t)1 << best_req_a.size(), sb = (int64_t)1 << best_req_b.size();
        int64_t scn = (int64_t)1 << best_ord_c.size();
        if (best.perm_a) best.a_tmp_off = arena.alloc(sa);
        if (best.perm_b) best.b_tmp_off = arena.alloc(sb);
        best.c_off = arena.alloc(scn);
        if (best.perm_a) {
            best.dag_a_tmp = dag_end;
            dag_end += Arena::align(sa);
        }
        if (best.perm_b) {
            best.dag_b_tmp = dag_end;
            dag_end += Arena::align(sb);
        }
        best.dag_c_off = dag_end;
        dag_off[x] = dag_end;
        dag_end += Arena::align(scn);
        off[x] = best.c_off;
        if (best.perm_a) arena.release(best.a_tmp_off, sa);
        if (best.perm_b) arena.release(best.b_tmp_off, sb);
        for (int ch : {nd.left, nd.right})
            if (ch >= nleaf) arena.release(off[ch], (int64_t)1 << p.order[ch].size());
        p.prog.push_back(best);
    }
    // single-leaf network: the leaf is the root; give it its (empty) order
    if (nn == nleaf) {
        p.order[0] = kept(0);
        p.leaf_prog[0].rank = (int)p.order[0].size();
    }
    p.arena_entries = arena.peak;
    p.node_off = off;
    p.node_off_dag = dag_off;
    p.arena_entries_dag = dag_end;
    return TN_OK;
}

static tn_status finish_plan(const Net& net, Plan& p) {
    std::vector<char> sl(net.nv, 0);
    for (int x : p.sliced) sl[x] = 1;
    reorder_for_memory(p.nodes, p.nleaf(), sl);
    plan_complexity(p);
    if (p.max_rank > 40) return fail(TN_ETOOBIG, "largest intermediate above 2^40 entries; slice more indices");
    return plan_program(p);
}

tn_status plan_create(const Net& net, const PlanOptions& o, Plan& out) {
    out = Plan();
    out.nv = net.nv;
    out.edges = net.edges;
    out.fingerprint = net.fingerprint;
    out.kind = net.kind;
    out.leaves = make_leaves(net, o.absorb);
    {
        std::vector<char> seen(net.nv, 0);
        for (int v : o.open) {
            if (v < 0 || v >= net.nv) return fail(TN_EINVAL, "open vertex out of range");
            if (seen[v]++) return fail(TN_EINVAL, "open vertex listed twice");
        }
        if ((int)o.open.size() > kMaxOpen) return fail(TN_EINVAL, "at most 16 open vertices");
    }
    out.open = o.open;
    if (out.leaves.empty()) {  // nv = 0: the empty network, result is the identity
        return TN_OK;
    }
    std::vector<int> L, R, sliced;
    tn_status st = optimize_tree(net, out.leaves, o, L, R, sliced);
    if (st != TN_OK) return st;
    st = build_nodes(net, out.leaves, L, R, out.nodes, o.open);
    if (st != TN_OK) return st;
    out.sliced = sliced;
    std::sort(out.sliced.begin(), out.sliced.end());
    return finish_plan(net, out);
}

tn_status plan_from_tree(const Net& net, const std::vector<Leaf>& leaves0, const std::vector<int>& left,
                         const std::vector<int>& right, const std::vector<int>& sliced, Plan& out) {
    out = Plan();
    out.nv = net.nv;
    out.edges = net.edges;
    out.fingerprint = net.fingerprint;
    out.kind = net.kind;
    out.leaves = leaves0;
    for (auto& l : out.leaves) {
        l.scope.clear();
        for (int f : l.factors) {
            if (f >= (int)net.edges.size() || (f < 0 && -f - 1 >= net.nv))
                return fail(TN_EINVAL, "leaf factor out of range");
            if (f >= 0) {
                l.scope.push_back(net.edges[f][0]);
                l.scope.push_back(net.edges[f][1]);
            } else {
                l.scope.push_back(-f - 1);
            }
        }
        std::sort(l.scope.begin(), l.scope.end());
        l.scope.erase(std::unique(l.scope.begin(), l.scope.end()), l.scope.end());
        if (l.scope.size() > 2) return fail(TN_EINVAL, "a leaf may hold one edge and vertex factors of its ends");
        int ne = 0;
        for (int f : l.factors) ne += f >= 0;
        if (ne > 1 || l.factors.empty()) return fail(TN_EINVAL, "a leaf holds one edge and/or vertex factors");
    }
    for (int s : sliced)
        if (s < 0 || s >= net.nv) return fail(TN_EINVAL, "sliced index out of range");
    tn_status st = build_nodes(net, out.leaves, left, right, out.nodes);
    if (st != TN_OK) return st;
    out.sliced = sliced;
    std::sort(out.sliced.begin(), out.sliced.end());
    out.sliced.erase(std::unique(out.sliced.begin(), out.sliced.end()), out.sliced.end());
    return finish_plan(net, out);
}

}  // namespace tn
