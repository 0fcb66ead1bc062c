// Host-side network and plan structures: the independent-set network
// (Sec. 3.2), the binary contraction tree and its complexity (Sec. 4.1), the
// order optimizers (Sec. 4.2) and the executor program derived from a tree.
#pragma once

#include <array>
#include <cstdint>
#include <string>
#include <vector>

#include "common.h"

namespace tn {

struct Net {
    int nv = 0;
    std::vector<std::array<int, 2>> edges;  // u < v, unique, in input order
    std::vector<float> w;                   // empty = unit weights
    bool integer_weights = true;            // every weight is an exact integer
    uint64_t fingerprint = 0;
    uint64_t uid = 0;  // unique per created network (cache keys)
    // 0: independent set (w = vertex weights, or empty for unit weights);
    // 1: spin glass H = sum J s_u s_v + sum h s_v (w = h[nv] then J[edges])
    int kind = 0;
    // fixed vertices (conditioning): fix[v] = -1 free, 0 or 1; empty = none
    std::vector<signed char> fix;
    // the array the leaf kernels read: w (unit weights written out when
    // vertices are fixed), then the fix codes as floats from fix_off on
    std::vector<float> wdev;
    int fix_off = -1;
};

tn_status make_net(int nv, int ne, const int32_t* edges, const float* weights, Net& out);
// Spin glass on the graph: J per input edge (NULL: all 1; duplicates add up),
// h per vertex (NULL: all 0).
tn_status make_spin_glass(int nv, int ne, const int32_t* edges, const float* J, const float* h, Net& out);
// A copy of src with vertices[k] fixed to values[k] (0 or 1), on top of the
// fixings src already has; same structure, so src's plans fit it.
tn_status condition_net(const Net& src, int n, const int32_t* vertices, const int32_t* values, Net& out);
void set_dev_weights(Net& net);

// One leaf tensor: the product of some edge / vertex factors of the network.
struct Leaf {
    std::vector<int> factors;  // edge id e >= 0, vertex v as -v-1
    std::vector<int> scope;    // vertices the factors touch, ascending
};

// A tree node.  Leaves come first (ids 0..nleaf-1), inner nodes follow in
// execution order: both children of an inner node have smaller ids; the last
// node is the root.  `out` are the node's output indices, ascending; sliced
// indices are not removed here.
struct Node {
    int left = -1, right = -1;
    std::vector<int> out;
};

// Executor program for one inner node.  "Storage order" of a tensor is the
// list of its (unsliced) indices from bit 0 of the linear offset upward; every
// index has dimension 2, so a tensor of rank r has 2^r entries.
struct NodeProg {
    int node = -1;
    int a = -1, b = -1;            // node ids of the GEMM's A and B operands
    bool perm_a = false, perm_b = false;
    std::vector<int> perm_a_src;   // permute: output bit q <- input bit perm_a_src[q]
    std::vector<int> perm_b_src;
    int lb = 0, li = 0, lj = 0, lk = 0;  // log2 of batch, M, N, K
    bool a_t = false;              // A stored [b][k][i] (i fastest) instead of [b][i][k]
    bool b_t = false;              // B stored [b][j][k] (k fastest) instead of [b][k][j]
    int64_t c_off = 0;             // arena offsets (entries)
    int64_t a_tmp_off = -1, b_tmp_off = -1;
    // the same tensors in the dependency-graph layout: every tensor has its
    // own region, so nodes of independent subtrees may run concurrently
    int64_t dag_c_off = 0, dag_a_tmp = -1, dag_b_tmp = -1;
};

struct LeafProg {
    int u = -1, v = -1;     // the leaf's edge (u < v) or u = the vertex of a vertex-only leaf
    int has_edge = 0;
    int edge = -1;          // the edge factor's edge id
    int wu = 0, wv = 0;     // vertex factors of u / v folded into this leaf
    int rank = 0;           // unsliced output indices
    int var[2] = {-1, -1};  // vertex at bit 0 / bit 1 of the leaf tensor
    int64_t off = 0;        // arena offset (entries)
};

struct Plan {
    // network identity
    int nv = 0;
    std::vector<std::array<int, 2>> edges;
    uint64_t fingerprint = 0;
    int kind = 0;  // the network kind (Net::kind)
    // tree
    std::vector<Leaf> leaves;
    std::vector<Node> nodes;
    std::vector<int> sliced;
    std::vector<int> open;  // open vertices in the caller's order: bit q of a result entry is open[q]
    // complexity (log2), Sec. 4.1; tc includes the 2^nsliced factor
    double tc = 0, sc = 0, rwc = 0;
    int max_rank = 0;
    // executor program
    std::vector<std::vector<int>> order;  // storage order of every node's tensor
    std::vector<LeafProg> leaf_prog;
    std::vector<NodeProg> prog;           // one per inner node, execution order
    std::vector<int64_t> node_off;        // arena offset of every node's tensor
    std::vector<int64_t> node_off_dag;    // same, dependency-graph layout (no reuse)
    int64_t arena_entries_dag = 0;
    int64_t arena_entries = 0;            // per plane, per slice
    int64_t leaf_entries = 0;
    int npermutes = 0;
    uint64_t uid = 0;                     // unique id (device-program cache key)

    int nleaf() const { return (int)leaves.size(); }
    int ninner() const { return (int)nodes.size() - (int)leaves.size(); }
};

struct PlanOptions {
    int method = 0;
    double alpha = 0, temperature = 0;
    int nrepeat = 10;
    uint64_t seed = 0;
    double sc_target = 20, sc_weight = 1.0, rw_weight = 0.2;
    double beta_start = 0.01, beta_step = 0.05, beta_stop = 15.0;
    int ntrials = 10, niters = 50, nslices = 0;
    bool absorb = true;
    int nthreads = 0;
    std::vector<int> open;  // open vertices (kept to the root), in the caller's order
};

constexpr int kMaxOpen = 16;

// Leaves of the network: one per edge, plus one per vertex unless the
// vertex tensor is folded into its first incident edge.
std::vector<Leaf> make_leaves(const Net& net, bool absorb);

// Run the optimizer and build the full plan (tree, complexity, program).
tn_status plan_create(const Net& net, const PlanOptions& o, Plan& out);
// Build a plan from an explicit tree (validated).
tn_status plan_from_tree(const Net& net, const std::vector<Leaf>& leaves,
                         const std::vector<int>& left, const std::vector<int>& right,
                         const std::vector<int>& sliced, Plan& out);
// Complexity of a tree (fills tc/sc/rwc/max_rank).
void plan_complexity(Plan& p);
// Derive storage orders, operand permutes and the memory plan.
tn_status plan_program(Plan& p);

void flat_complexity(const Net& net, double& tc, double& sc, double& rwc);

}  // namespace tn
