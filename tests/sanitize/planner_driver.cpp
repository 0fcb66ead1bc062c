// Host driver for sanitizer builds (AddressSanitizer + UndefinedBehavior-
// Sanitizer, ThreadSanitizer) of the planner: network construction (independent
// sets, spin glasses, conditioning), the greedy and TreeSA optimizers (TreeSA
// trials on several host threads), slicing, open vertices, explicit trees
// (valid and invalid), complexity and the executor program.  No GPU call is
// made.  Exits non-zero on an inconsistent plan; the sanitizers abort on a
// memory error, undefined behaviour or a data race.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <set>
#include <string>
#include <vector>

#include "../../paper_2501_00227_amd/csrc/plan.h"

using namespace tn;

static int g_bad = 0;
#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            std::fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            g_bad++;                                                \
        }                                                           \
    } while (0)

// random simple graph: each pair an edge with probability p, plus a 3-regular-ish ring
static std::vector<int32_t> random_edges(int n, double p, std::mt19937_64& rng) {
    std::vector<int32_t> e;
    std::uniform_real_distribution<double> u(0, 1);
    for (int a = 0; a < n; a++)
        for (int b = a + 1; b < n; b++)
            if (u(rng) < p) {
                e.push_back(a);
                e.push_back(b);
            }
    return e;
}

static void check_plan(const Plan& p, int nleaf_expect) {
    CHECK(p.nleaf() == nleaf_expect || nleaf_expect < 0);
    CHECK(std::isfinite(p.tc) && std::isfinite(p.sc) && std::isfinite(p.rwc));
    CHECK(p.max_rank >= 0 && p.max_rank <= 62);
    CHECK(p.prog.size() == (size_t)p.ninner());
    CHECK(p.order.size() == p.nodes.size());
    for (size_t t = 0; t < p.prog.size(); t++) {
        const NodeProg& np = p.prog[t];
        CHECK(np.lb >= 0 && np.li >= 0 && np.lj >= 0 && np.lk >= 0);
        CHECK(np.a >= 0 && np.b >= 0 && np.a < (int)p.nodes.size() && np.b < (int)p.nodes.size());
        CHECK(np.c_off >= 0 && np.c_off < p.arena_entries + 1);
    }
}

int main(int argc, char** argv) {
    const int rounds = argc > 1 ? std::atoi(argv[1]) : 12;
    std::mt19937_64 rng(12345);
    for (int r = 0; r < rounds; r++) {
        const int n = 6 + (int)(rng() % 40);
        std::vector<int32_t> e = random_edges(n, r % 3 == 0 ? 0.15 : 0.08, rng);
        const int ne = (int)e.size() / 2;
        std::vector<float> w(n);
        for (int v = 0; v < n; v++) w[v] = (float)(1 + rng() % 4);
        Net net, sg, cond;
        CHECK(make_net(n, ne, e.empty() ? nullptr : e.data(), r % 2 ? w.data() : nullptr, net) == TN_OK);
        CHECK(make_spin_glass(n, ne, e.empty() ? nullptr : e.data(), nullptr, nullptr, sg) == TN_OK);
        const int32_t vs[2] = {0, 1}, xs[2] = {1, 0};
        CHECK(condition_net(net, 2, vs, xs, cond) == TN_OK);
        set_dev_weights(cond);
        double tc, sc, rw;
        flat_complexity(net, tc, sc, rw);
        for (int method = 0; method < 2; method++) {
            PlanOptions o;
            o.method = method;
            o.seed = (uint64_t)r;
            o.ntrials = 4;
            o.niters = 4;
            o.nthreads = 4;  // TreeSA trials on host threads
            o.absorb = r % 2 == 0;
            if (r % 4 == 1) {
                o.sc_target = 3;
                o.nslices = 4;
            }
            if (r % 5 == 2 && n > 3) o.open = {0, 2};
            Plan p;
            CHECK(plan_create(net, o, p) == TN_OK);
            check_plan(p, -1);
            Plan q;
            CHECK(plan_create(sg, o, q) == TN_OK);
            check_plan(q, -1);
            // the same tree again, from its node list
            std::vector<int> left, right;
            for (size_t t = p.leaves.size(); t < p.nodes.size(); t++) {
                left.push_back(p.nodes[t].left);
                right.push_back(p.nodes[t].right);
            }
            if (p.open.empty()) {
                Plan t2;
                CHECK(plan_from_tree(net, p.leaves, left, right, p.sliced, t2) == TN_OK);
                check_plan(t2, (int)p.leaves.size());
                CHECK(std::fabs(t2.tc - p.tc) < 1e-9 && t2.max_rank == p.max_rank);
                // invalid trees are refused
                if (!left.empty()) {
                    std::vector<int> bad = left;
                    bad.back() = (int)p.nodes.size() + 3;
                    Plan t3;
                    CHECK(plan_from_tree(net, p.leaves, bad, right, p.sliced, t3) != TN_OK);
                    std::vector<int> dup = left;
                    dup[0] = right[0];
                    Plan t4;
                    CHECK(plan_from_tree(net, p.leaves, dup, right, p.sliced, t4) != TN_OK);
                }
            }
        }
    }
    // invalid networks
    Net x;
    const int32_t loop[2] = {1, 1}, oor[2] = {0, 9};
    CHECK(make_net(3, 1, loop, nullptr, x) != TN_OK);
    CHECK(make_net(3, 1, oor, nullptr, x) != TN_OK);
    const float nan = std::nanf("");
    const int32_t ok[2] = {0, 1};
    const float wn[3] = {1, nan, 1};
    CHECK(make_net(3, 1, ok, wn, x) != TN_OK);
    std::printf("planner driver: %d rounds, %d failed checks\n", rounds, g_bad);
    return g_bad == 0 ? 0 : 1;
}
