// Contraction-order optimizers (Sec. 4.2): greedy / hyper-greedy, TreeSA
// local search with slicing.  Trees are binary; leaves are the network's leaf
// tensors, each index has dimension 2 so a tensor's size is 2^rank.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <thread>
#include <unordered_set>

#include "plan.h"

namespace tn {

namespace {

// A binary tree over nleaf leaves: ids [0, nleaf) leaves, [nleaf, 2nleaf-1) inner.
struct Tree {
    int nleaf = 0;
    std::vector<int> L, R;  // children of inner node n at index n - nleaf
    int root = 0;
};

template <int W>
struct Cost {
    double tc = 0, rw = 0;  // linear sums (entries)
    int sc = 0;
};

// Output indices of every node: out(N) = U(N) & O(N) where U is the union of
// leaf indices below N and O the union of leaf indices outside N's subtree
// (an index stays open while it is still needed elsewhere, Sec. 3.2 einsum).
template <int W>
void outputs(const Tree& t, const std::vector<Bits<W>>& leaf_ix, std::vector<Bits<W>>& out, const Bits<W>& open) {
    int nn = 2 * t.nleaf - 1;
    std::vector<Bits<W>> U(nn), O(nn);
    std::vector<int> post;
    post.reserve(nn);
    // iterative post-order
    std::vector<std::pair<int, int>> st{{t.root, 0}};
    while (!st.empty()) {
        auto& [n, s] = st.back();
        if (n < t.nleaf || s == 2) {
            post.push_back(n);
            st.pop_back();
            continue;
        }
        int c = s == 0 ? t.L[n - t.nleaf] : t.R[n - t.nleaf];
        s++;
        st.push_back({c, 0});
    }
    for (int n : post)
        U[n] = n < t.nleaf ? leaf_ix[n] : U[t.L[n - t.nleaf]] | U[t.R[n - t.nleaf]];
    O[t.root] = open;  // open vertices are held by the output
    for (int k = (int)post.size() - 1; k >= 0; k--) {
        int n = post[k];
        if (n < t.nleaf) continue;
        int a = t.L[n - t.nleaf], b = t.R[n - t.nleaf];
        O[a] = O[n] | U[b];
        O[b] = O[n] | U[a];
    }
    out.assign(nn, Bits<W>());
    for (int n = 0; n < nn; n++) out[n] = U[n] & O[n];
}

template <int W>
Cost<W> tree_cost(const Tree& t, const std::vector<Bits<W>>& out) {
    Cost<W> c;
    for (int n = t.nleaf; n < 2 * t.nleaf - 1; n++) {
        const auto& a = out[t.L[n - t.nleaf]];
        const auto& b = out[t.R[n - t.nleaf]];
        c.tc += std::exp2((double)(a | b).count());
        c.rw += std::exp2((double)a.count()) + std::exp2((double)b.count()) +
                std::exp2((double)out[n].count());
        c.sc = std::max(c.sc, out[n].count());
    }
    return c;
}

// ------------------------------------------------------------- greedy ---
// Sec. 4.2.1: repeatedly contract the pair with the smallest
// L = size(Ti*Tj) - alpha (size(Ti) + size(Tj)); with temperature T > 0 the
// pair is sampled with probability proportional to e^{-L/T}.
template <int W>
Tree greedy_once(const std::vector<Bits<W>>& leaf_ix, int nv, double alpha, double T, Rng& rng,
                 const Bits<W>& open) {
    int n = (int)leaf_ix.size();
    Tree t;
    t.nleaf = n;
    if (n == 1) {
        t.root = 0;
        return t;
    }
    std::vector<Bits<W>> ix(2 * n - 1);
    for (int i = 0; i < n; i++) ix[i] = leaf_ix[i];
    std::vector<int> cnt(nv, 0);
    std::vector<std::vector<int>> holders(nv);
    std::vector<char> alive(2 * n - 1, 0);
    for (int i = 0; i < n; i++) {
        alive[i] = 1;
        ix[i].for_each([&](int x) {
            cnt[x]++;
            holders[x].push_back(i);
        });
    }
    open.for_each([&](int x) { cnt[x]++; });  // held by the output: never summed
    int next = n, nalive = n;
    std::vector<uint64_t> pairs;
    std::vector<double> costs;
    std::vector<Bits<W>> outs;
    while (nalive > 1) {
        pairs.clear();
        for (int x = 0; x < nv; x++) {
            auto& h = holders[x];
            for (size_t a = 0; a < h.size(); a++)
                for (size_t b = a + 1; b < h.size(); b++) {
                    int p = std::min(h[a], h[b]), q = std::max(h[a], h[b]);
                    pairs.push_back(((uint64_t)p << 32) | (uint32_t)q);
                }
        }
        std::sort(pairs.begin(), pairs.end());
        pairs.erase(std::unique(pairs.begin(), pairs.end()), pairs.end());
        if (pairs.empty()) {
            // disconnected components: join the two smallest tensors
            int p = -1, q = -1;
            for (int i = 0; i < next; i++) {
                if (!alive[i]) continue;
                if (p < 0 || ix[i].count() < ix[p].count()) {
                    q = p;
                    p = i;
                } else if (q < 0 || ix[i].count() < ix[q].count()) {
                    q = i;
                }
            }
            pairs.push_back(((uint64_t)std::min(p, q) << 32) | (uint32_t)std::max(p, q));
        }
        costs.resize(pairs.size());
        outs.resize(pairs.size());
        double best = 1.0 / 0.0;
        for (size_t k = 0; k < pairs.size(); k++) {
            int a = (int)(pairs[k] >> 32), b = (int)(uint32_t)pairs[k];
            Bits<W> u = ix[a] | ix[b], o;
            u.for_each([&](int x) {
                int inside = (int)ix[a].has(x) + (int)ix[b].has(x);
                if (cnt[x] > inside) o.set(x);
            });
            outs[k] = o;
            costs[k] = std::exp2((double)o.count()) -
                       alpha * (std::exp2((double)ix[a].count()) + std::exp2((double)ix[b].count()));
            best = std::min(best, costs[k]);
        }
        size_t pick = 0;
        if (T > 0) {
            double tot = 0;
            for (auto c : costs) tot += std::exp(-(c - best) / T);
            double r = rng.uniform() * tot;
            for (pick = 0; pick + 1 < costs.size(); pick++) {
                r -= std::exp(-(costs[pick] - best) / T);
                if (r <= 0) break;
            }
        } else {
            // uniform among the minimisers (seeded tie-break)
            int nmin = 0;
            for (size_t k = 0; k < costs.size(); k++)
                if (costs[k] == best) nmin++;
            int r = (int)rng.below((uint32_t)nmin);
            for (size_t k = 0; k < costs.size(); k++)
                if (costs[k] == best && r-- == 0) {
                    pick = k;
                    break;
                }
        }
        int a = (int)(pairs[pick] >> 32), b = (int)(uint32_t)pairs[pick];
        int c = next++;
        ix[c] = outs[pick];
        t.L.push_back(a);
        t.R.push_back(b);
        for (int s : {a, b}) {
            alive[s] = 0;
            ix[s].for_each([&](int x) {
                cnt[x]--;
                auto& h = holders[x];
                h.erase(std::find(h.begin(), h.end(), s));
            });
        }
        alive[c] = 1;
        ix[c].for_each([&](int x) {
            cnt[x]++;
            holders[x].push_back(c);
        });
        nalive--;
    }
    t.root = next - 1;
    return t;
}

template <int W>
bool better(const Cost<W>& a, const Cost<W>& b) {
    if (a.tc != b.tc) return a.tc < b.tc;
    return a.sc < b.sc;
}

template <int W>
Tree greedy(const std::vector<Bits<W>>& leaf_ix, int nv, double alpha, double T, int nrepeat,
            uint64_t seed, const Bits<W>& open) {
    Tree best;
    Cost<W> bc;
    std::vector<Bits<W>> out;
    for (int r = 0; r < std::max(1, nrepeat); r++) {
        Rng rng(seed * 1000003ull + (uint64_t)r);
        Tree t = greedy_once<W>(leaf_ix, nv, alpha, T, rng, open);
        outputs<W>(t, leaf_ix, out, open);
        Cost<W> c = tree_cost<W>(t, out);
        if (r == 0 || better<W>(c, bc)) {
            best = t;
            bc = c;
        }
    }
    return best;
}

// ------------------------------------------------------------- TreeSA ---
// Sec. 4.2.2: simulated annealing over the rotations
//   (A*B)*C -> (A*C)*B | (C*B)*A   and   A*(B*C) -> B*(A*C) | C*(B*A),
// cost tc + w_s * max(0, sc - sc_target) + w_rw * rwc in log2 units,
// Metropolis acceptance min(1, e^{-beta dL}).
template <int W>
struct Annealer {
    int nleaf, nn;
    std::vector<int> L, R, P;
    std::vector<Bits<W>> out;
    std::vector<double> tterm, rterm;  // per inner node: 2^t and read-write entries
    std::vector<int> hist;             // number of inner nodes of each rank
    double TC = 0, RW = 0;
    double sc_target, ws, wrw;
    Bits<W> open;  // open vertices: kept to the root, never sliced

    void load(const Tree& t, const std::vector<Bits<W>>& leaf_ix) {
        nleaf = t.nleaf;
        nn = 2 * nleaf - 1;
        L.assign(nn, -1);
        R.assign(nn, -1);
        P.assign(nn, -1);
        for (int n = nleaf; n < nn; n++) {
            L[n] = t.L[n - nleaf];
            R[n] = t.R[n - nleaf];
            P[L[n]] = P[R[n]] = n;
        }
        outputs<W>(t, leaf_ix, out, open);
        refresh();
    }
    int root() const {
        for (int n = 0; n < nn; n++)
            if (P[n] < 0) return n;
        return 0;
    }
    void refresh() {
        tterm.assign(nn, 0);
        rterm.assign(nn, 0);
        hist.assign(W * 64 + 2, 0);
        TC = RW = 0;
        for (int n = nleaf; n < nn; n++) {
            tterm[n] = std::exp2((double)(out[L[n]] | out[R[n]]).count());
            rterm[n] = std::exp2((double)out[L[n]].count()) + std::exp2((double)out[R[n]].count()) +
                       std::exp2((double)out[n].count());
            TC += tterm[n];
            RW += rterm[n];
            hist[out[n].count()]++;
        }
    }
    int sc() const {
        for (int r = (int)hist.size() - 1; r >= 0; r--)
            if (hist[r]) return r;
        return 0;
    }
    double cost(double tc, double rw, int s) const {
        return std::log2(tc) + ws * std::max(0.0, (double)s - sc_target) + wrw * std::log2(rw);
    }
    Tree tree() const {
        Tree t;
        t.nleaf = nleaf;
        // renumber inner nodes in post-order so children precede parents
        std::vector<int> id(nn, -1);
        for (int n = 0; n < nleaf; n++) id[n] = n;
        int next = nleaf;
        std::vector<std::pair<int, int>> st{{root(), 0}};
        std::vector<int> post;
        while (!st.empty()) {
            auto& [n, s] = st.back();
            if (n < nleaf || s == 2) {
                if (n >= nleaf) post.push_back(n);
                st.pop_back();
                continue;
            }
            int c = s == 0 ? L[n] : R[n];
            s++;
            st.push_back({c, 0});
        }
        for (int n : post) id[n] = next++;
        t.L.resize(nleaf - 1);
        t.R.resize(nleaf - 1);
        for (int n : post) {
            t.L[id[n] - nleaf] = id[L[n]];
            t.R[id[n] - nleaf] = id[R[n]];
        }
        t.root = nn - 1;
        return t;
    }
    // Try one random rotation at inner node p; returns true if accepted.
    bool move(int p, double beta, Rng& rng) {
        bool li = L[p] >= nleaf, ri = R[p] >= nleaf;
        if (!li && !ri) return false;
        int side = li && ri ? (int)rng.below(2) : (li ? 0 : 1);
        int n = side == 0 ? L[p] : R[p];
        int z = side == 0 ? R[p] : L[p];
        int swap_x = (int)rng.below(2);
        int x = L[n], y = R[n];
        int moved = swap_x ? x : y;  // goes up to p
        int c1 = swap_x ? z : x, c2 = swap_x ? y : z;
        Bits<W> new_out = (out[c1] | out[c2]) & (out[moved] | out[p]);
        double t_n = std::exp2((double)(out[c1] | out[c2]).count());
        double t_p = std::exp2((double)(new_out | out[moved]).count());
        double r_n = std::exp2((double)out[c1].count()) + std::exp2((double)out[c2].count()) +
                     std::exp2((double)new_out.count());
        double r_p = std::exp2((double)new_out.count()) + std::exp2((double)out[moved].count()) +
                     std::exp2((double)out[p].count());
        double nTC = TC - tterm[n] - tterm[p] + t_n + t_p;
        double nRW = RW - rterm[n] - rterm[p] + r_n + r_p;
        int old_rank = out[n].count(), new_rank = new_out.count();
        int s_old = sc();
        hist[old_rank]--;
        hist[new_rank]++;
        int s_new = sc();
        double dL = cost(nTC, nRW, s_new) - cost(TC, RW, s_old);
        if (dL > 0 && rng.uniform() >= std::exp(-beta * dL)) {
            hist[new_rank]--;
            hist[old_rank]++;
            return false;
        }
        // apply
        L[n] = c1;
        R[n] = c2;
        P[c1] = P[c2] = n;
        if (side == 0)
            R[p] = moved;
        else
            L[p] = moved;
        P[moved] = p;
        out[n] = new_out;
        tterm[n] = t_n;
        tterm[p] = t_p;
        rterm[n] = r_n;
        rterm[p] = r_p;
        TC = nTC;
        RW = nRW;
        return true;
    }
    // Anneal over the inverse temperatures; the lowest-cost tree seen at the
    // end of any temperature step is restored at the end.
    void anneal(const std::vector<double>& betas, int niters, Rng& rng) {
        std::vector<int> inner;
        for (int n = nleaf; n < nn; n++) inner.push_back(n);
        double best = cost(TC, RW, sc());
        std::vector<int> bL = L, bR = R, bP = P;
        std::vector<Bits<W>> bout = out;
        for (double beta : betas) {
            for (int it = 0; it < niters; it++) {
                for (size_t k = inner.size(); k > 1; k--) std::swap(inner[k - 1], inner[rng.below((uint32_t)k)]);
                for (int p : inner) move(p, beta, rng);
            }
            refresh();  // drop accumulated rounding in the running sums
            double c = cost(TC, RW, sc());
            if (c < best) {
                best = c;
                bL = L;
                bR = R;
                bP = P;
                bout = out;
            }
        }
        L.swap(bL);
        R.swap(bR);
        P.swap(bP);
        out.swap(bout);
        refresh();
    }
};

template <int W>
struct SAResult {
    Tree tree;
    std::vector<int> sliced;
    double cost = 1.0 / 0.0;
};

// Slice the index whose removal best lowers the largest intermediate: the
// one contained in the most maximum-rank nodes, ties broken by the smaller
// resulting tc.
template <int W>
int choose_slice(const Annealer<W>& a) {
    int s = a.sc();
    std::vector<int> hits(W * 64, 0);
    std::vector<double> gain(W * 64, 0.0);
    for (int n = a.nleaf; n < a.nn; n++) {
        if (a.out[n].count() == s) a.out[n].for_each([&](int x) { hits[x]++; });
        Bits<W> u = a.out[a.L[n]] | a.out[a.R[n]];
        double t = a.tterm[n];
        u.for_each([&](int x) { gain[x] += t / 2; });
    }
    int best = -1;
    for (int x = 0; x < W * 64; x++) {
        if (!hits[x] || a.open.has(x)) continue;
        if (best < 0 || hits[x] > hits[best] || (hits[x] == hits[best] && gain[x] > gain[best])) best = x;
    }
    return best;
}

template <int W>
SAResult<W> treesa_trial(const std::vector<Bits<W>>& leaf_ix0, int nv, const PlanOptions& o,
                         uint64_t seed, const Bits<W>& open) {
    Rng rng(seed);
    std::vector<Bits<W>> leaf_ix = leaf_ix0;
    Tree t0 = greedy<W>(leaf_ix, nv, 0.0, 0.0, 1, seed, open);
    SAResult<W> res;
    if ((int)leaf_ix.size() < 3) {
        res.tree = t0;
        res.cost = 0;
        return res;
    }
    std::vector<double> betas;
    for (double b = o.beta_start; b <= o.beta_stop + 1e-12; b += o.beta_step) betas.push_back(b);
    if (betas.empty()) betas.push_back(o.beta_stop);
    Annealer<W> a;
    a.sc_target = o.sc_target;
    a.ws = o.sc_weight;
    a.wrw = o.rw_weight;
    a.open = open;
    a.load(t0, leaf_ix);
    a.anneal(betas, o.niters, rng);
    // slicing: fix one index at a time while the largest intermediate is
    // above the target, re-annealing the sliced network at low temperature
    std::vector<int> sliced;
    Bits<W> smask;
    std::vector<double> cool;
    for (size_t k = betas.size() / 2; k < betas.size(); k++) cool.push_back(betas[k]);
    while ((int)sliced.size() < o.nslices && a.sc() > (int)o.sc_target) {
        int x = choose_slice<W>(a);
        if (x < 0) break;
        sliced.push_back(x);
        smask.set(x);
        for (auto& b : leaf_ix) b.clear(x);
        Tree cur = a.tree();
        a.load(cur, leaf_ix);
        a.anneal(cool, std::max(1, o.niters / 4), rng);
    }
    res.tree = a.tree();
    res.sliced = sliced;
    res.cost = a.cost(a.TC, a.RW, a.sc()) + (double)sliced.size();
    return res;
}

template <int W>
tn_status optimize_w(const Net& net, const std::vector<Leaf>& leaves, const PlanOptions& o,
                     std::vector<int>& L, std::vector<int>& R, std::vector<int>& sliced) {
    int nleaf = (int)leaves.size();
    // open indices of each leaf: drop indices that occur in no other leaf
    std::vector<int> occ(net.nv, 0);
    for (auto& l : leaves)
        for (int x : l.scope) occ[x]++;
    Bits<W> open;
    for (int x : o.open) open.set(x);
    std::vector<Bits<W>> leaf_ix(nleaf);
    for (int i = 0; i < nleaf; i++)
        for (int x : leaves[i].scope)
            if (occ[x] > 1 || open.has(x)) leaf_ix[i].set(x);
    Tree best;
    sliced.clear();
    if (o.method == 0) {
        best = greedy<W>(leaf_ix, net.nv, o.alpha, o.temperature, o.nrepeat, o.seed, open);
        // optional slicing on a greedy tree
        if (o.nslices > 0) {
            Annealer<W> a;
            a.sc_target = o.sc_target;
            a.ws = o.sc_weight;
            a.wrw = o.rw_weight;
            a.open = open;
            a.load(best, leaf_ix);
            while ((int)sliced.size() < o.nslices && a.sc() > (int)o.sc_target) {
                int x = choose_slice<W>(a);
                if (x < 0) break;
                sliced.push_back(x);
                for (auto& b : leaf_ix) b.clear(x);
                Tree cur = a.tree();
                a.load(cur, leaf_ix);
            }
            best = a.tree();
        }
    } else {
        auto anneal = [&]() {  // best of ntrials TreeSA trials, on host threads
            int nt = std::max(1, o.ntrials);
            std::vector<SAResult<W>> res(nt);
            int nth = o.nthreads > 0 ? o.nthreads : (int)std::thread::hardware_concurrency();
            nth = std::max(1, std::min(nth, nt));
            std::atomic<int> next{0};
            std::vector<std::thread> pool;
            for (int th = 0; th < nth; th++)
                pool.emplace_back([&]() {
                    for (int k; (k = next.fetch_add(1)) < nt;)
                        res[k] = treesa_trial<W>(leaf_ix, net.nv, o, o.seed * 7919ull + (uint64_t)k, open);
                });
            for (auto& th : pool) th.join();
            int bi = 0;
            for (int k = 1; k < nt; k++)
                if (res[k].cost < res[bi].cost) bi = k;
            return res[bi];
        };
        if (o.method == 1) {
            SAResult<W> r = anneal();
            best = r.tree;
            sliced = r.sliced;
        } else {
            // automatic: the greedy tree, and when it needs more than 2^26
            // semiring ops TreeSA as well; the tree of lower annealing cost
            // (tc, sc above the target, read-write) wins
            best = greedy<W>(leaf_ix, net.nv, o.alpha, o.temperature, o.nrepeat, o.seed, open);
            Annealer<W> a;
            a.sc_target = o.sc_target;
            a.ws = o.sc_weight;
            a.wrw = o.rw_weight;
            a.open = open;
            a.load(best, leaf_ix);
            if (std::log2(a.TC) > 26.0) {
                SAResult<W> r = anneal();
                if (r.cost < a.cost(a.TC, a.RW, a.sc())) {
                    best = r.tree;
                    sliced = r.sliced;
                }
            }
        }
    }
    L = best.L;
    R = best.R;
    return TN_OK;
}

}  // namespace

tn_status optimize_tree(const Net& net, const std::vector<Leaf>& leaves, const PlanOptions& o,
                        std::vector<int>& L, std::vector<int>& R, std::vector<int>& sliced) {
    int nv = net.nv;
    if (nv <= 64) return optimize_w<1>(net, leaves, o, L, R, sliced);
    if (nv <= 128) return optimize_w<2>(net, leaves, o, L, R, sliced);
    if (nv <= 256) return optimize_w<4>(net, leaves, o, L, R, sliced);
    if (nv <= 512) return optimize_w<8>(net, leaves, o, L, R, sliced);
    if (nv <= 1024) return optimize_w<16>(net, leaves, o, L, R, sliced);
    return optimize_w<64>(net, leaves, o, L, R, sliced);
}

}  // namespace tn
