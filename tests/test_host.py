"""Host-side tests of the C-ABI library (no GPU needed): symbol exports,
network validation, the contraction-complexity definitions of Sec. 4.1, and
the planner's trees checked by the oracle's independent plan follower."""
import json
import math
import os
import re

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2501_00227_amd as tn

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_values.json")))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "tn.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    names = set(re.findall(r"\b(tn_[a-z0-9_]+)\s*\(", hdr))
    assert len(names) >= 25
    L = tn.lib()
    missing = [n for n in sorted(names) if not hasattr(L, n)]
    assert not missing, missing
    # and the binding declares a signature for each of them
    assert names <= {s[0] for s in tn.SIGNATURES}


def test_network_validation():
    with pytest.raises(tn.TnError) as ei:
        tn.Net(3, [[0, 0]])
    assert ei.value.code == tn.TN_EINVAL
    with pytest.raises(tn.TnError):
        tn.Net(3, [[0, 3]])
    with pytest.raises(tn.TnError):
        tn.Net(2, [[0, 1]], np.array([1.0, np.nan], np.float32))
    n = tn.Net(3, [[0, 1], [1, 0], [1, 2]])
    nv, ne = np.zeros(1, np.int32), np.zeros(1, np.int32)
    tn.lib().tn_net_info(n.h, tn._p32(nv), tn._p32(ne))
    assert (nv[0], ne[0]) == (3, 2)  # duplicate edge merged


def _square2_code():
    # EinCode of Sec. 4.1: tensors [1,2],[2,3],[3,4],[4,1],[1],[2],[3],[4]
    return tn.Net(4, np.array([[0, 1], [1, 2], [2, 3], [0, 3]], np.int32))


def test_flat_complexity_matches_paper():
    want = GOLD["square2"]["flat_complexity_log2"]["value"]
    tc, sc, rw = _square2_code().flat_complexity()
    assert (tc, sc) == (want["tc"], want["sc"])
    assert rw == pytest.approx(want["rwc"], abs=1e-12)


def _paper_tree_plan():
    net = _square2_code()
    leaves = [[0], [1], [2], [3], [-1], [-2], [-3], [-4]]
    left = [2, 8, 5, 10, 11, 3, 13]
    right = [6, 7, 1, 9, 0, 12, 4]
    return net, tn.Plan.from_tree(net, leaves, left, right)


def test_tree_complexity_matches_paper():
    want = GOLD["square2"]["tree_complexity_log2"]["value"]
    net, plan = _paper_tree_plan()
    tc, sc, rw = plan.complexity()
    assert tc == pytest.approx(want["tc"], abs=1e-12)
    assert sc == want["sc"]
    assert rw == pytest.approx(want["rwc"], abs=1e-12)


def test_paper_tree_is_followed_by_the_oracle():
    net, plan = _paper_tree_plan()
    g = gg.Graph(4, np.array([[0, 1], [1, 2], [2, 3], [0, 3]], np.int32))
    t = plan.export()
    assert oracle.follow_plan(g, t, "count")["count"] == 7


def test_invalid_trees_rejected():
    net = _square2_code()
    leaves = [[0], [1], [2], [3], [-1], [-2], [-3], [-4]]
    with pytest.raises(tn.TnError):  # node used twice
        tn.Plan.from_tree(net, leaves, [2, 2, 5, 10, 11, 3, 13], [6, 7, 1, 9, 0, 12, 4])
    with pytest.raises(tn.TnError):  # a factor missing
        tn.Plan.from_tree(net, leaves[:-1] + [[-3]], [2, 8, 5, 10, 11, 3, 13], [6, 7, 1, 9, 0, 12, 4])
    with pytest.raises(tn.TnError):  # child after parent
        tn.Plan.from_tree(net, leaves, [2, 8, 5, 10, 11, 3, 14], [6, 7, 1, 9, 0, 12, 4])


def test_plan_option_validation():
    net = tn.Net.from_graph(gg.cycle(5))
    with pytest.raises(tn.TnError):
        tn.Plan.create(net, method=7)
    with pytest.raises(tn.TnError):
        tn.Plan.create(net, method="treesa", beta_step=0.0)


def _random_plans():
    cases = []
    for s in range(16):
        g = [gg.random_regular(14, 3, s), gg.kings_subgraph(4, 0.8, s), gg.gnp(12, 0.3, s),
             gg.disjoint_union(gg.path(4), gg.empty(3))][s % 4]
        if s % 2:
            g = g.with_weights(gg.dyadic_weights(g.nv, s))
        kw = [dict(), dict(method="treesa", ntrials=2, niters=4), dict(absorb=False),
              dict(sc_target=2, nslices=3), dict(temperature=2.0, nrepeat=3)][s % 5]
        kw["seed"] = s
        cases.append((g, kw))
    return cases


@pytest.mark.parametrize("case", range(16))
def test_planner_trees_evaluate_correctly_in_the_oracle(case):
    g, kw = _random_plans()[case]
    plan = tn.Plan.create(tn.Net.from_graph(g), **kw)
    t = plan.export()
    bf = oracle.brute_force(g, [0.5])
    ct = oracle.follow_plan(g, t, "counting_tropical")
    assert ct["size"] == bf["size_max"]
    assert oracle.follow_plan(g, t, "count")["count"] == bf["count_all"]
    assert oracle.follow_plan(g, t, "partition", 0.5)["z"] == pytest.approx(bf["z"][0], rel=1e-13)


def test_greedy_meets_small_config_space_bound():
    for s in range(20):
        plan = tn.Plan.create(tn.Net.from_graph(gg.random_regular(20, 3, s)), seed=s)
        assert plan.complexity()[1] <= 8


def test_treesa_never_worse_than_its_greedy_start():
    g = gg.random_regular(60, 3, 3)
    net = tn.Net.from_graph(g)
    gr = tn.Plan.create(net, nrepeat=1, seed=1)
    sa = tn.Plan.create(net, method="treesa", ntrials=2, niters=5, seed=1, sc_target=30)
    # cost = tc + 0.2 rwc (sc below target): annealing keeps its best tree
    c = lambda p: p.complexity()[0] + 0.2 * p.complexity()[2]
    assert c(sa) <= c(gr) + 1e-9


def test_automatic_planner_keeps_greedy_for_small_and_anneals_large_networks():
    """method "auto": the greedy tree below 2^26 semiring ops, else the better
    (by the TreeSA cost) of the greedy tree and TreeSA's."""
    small = tn.Net.from_graph(gg.random_regular(60, 3, 1))
    a = tn.Plan.create(small, method="auto", ntrials=2, niters=4, seed=3)
    gr = tn.Plan.create(small, seed=3)
    assert a.export() == gr.export() and a.complexity()[0] <= 26
    g = gg.random_regular(170, 3, 170)
    net = tn.Net.from_graph(g)
    gr = tn.Plan.create(net, seed=1, sc_target=22)
    au = tn.Plan.create(net, method="auto", ntrials=2, niters=10, seed=1, sc_target=22)
    assert gr.complexity()[0] > 26
    cost = lambda p: p.complexity()[0] + max(0.0, p.complexity()[1] - 22) + 0.2 * p.complexity()[2]
    assert cost(au) <= cost(gr) + 1e-9
    assert au.complexity()[0] < gr.complexity()[0]  # here annealing wins: 2^31.1 against 2^35.0 ops
    t = au.export()
    sub = tn.Plan.create(tn.Net.from_graph(gg.random_regular(24, 3, 0)), method="auto", seed=0)
    bf = oracle.brute_force(gg.random_regular(24, 3, 0), [1.0])
    assert oracle.follow_plan(gg.random_regular(24, 3, 0), sub.export(), "count")["count"] == bf["count_all"]
    assert len(t["left"]) == len(t["right"]) > 0


def test_slicing_reaches_the_space_target():
    g = gg.random_regular(40, 3, 2)
    net = tn.Net.from_graph(g)
    full = tn.Plan.create(net, seed=2)
    sl = tn.Plan.create(net, seed=2, sc_target=full.complexity()[1] - 3, nslices=10)
    info = sl.info()
    assert info["nsliced"] >= 1
    assert sl.complexity()[1] <= full.complexity()[1] - 3
    # each sliced index doubles the work (Sec. 4.2): tc includes the 2^s factor
    assert sl.complexity()[0] >= full.complexity()[0] - 3


def test_peak_bytes_scale_with_element_size():
    plan = tn.Plan.create(tn.Net.from_graph(gg.random_regular(40, 3, 1)))
    b32 = plan.peak_bytes("tropical_i32")
    bct = plan.peak_bytes("counting_tropical")
    assert bct > 2.5 * b32 - 20000
    assert plan.info()["arena_entries"] * 4 <= b32


def test_spin_glass_network_validation_and_structure():
    g = gg.fullerene()
    assert (g.nv, g.ne) == (60, 90)
    with pytest.raises(tn.TnError) as ei:
        tn.Net.spin_glass(g, J=[float("nan")] + [1.0] * (g.ne - 1))
    assert ei.value.code == tn.TN_EINVAL
    with pytest.raises(tn.TnError) as ei:
        tn.Net.spin_glass(g, h=[float("inf")] * g.nv)
    assert ei.value.code == tn.TN_EINVAL
    sg, isn = tn.Net.spin_glass(g), tn.Net.from_graph(g)
    # same structure, same planner result; the plans are not interchangeable
    a = tn.Plan.create(sg, seed=3).complexity()
    b = tn.Plan.create(isn, seed=3).complexity()
    assert a == b


SEMIRINGS = ["tropical_i32", "tropical_f32", "counting_tropical", "count_exact", "partition_f32", "partition_bf16"]


def test_every_planned_gemm_shape_is_accepted_by_the_kernels():
    """Dense small graphs give nodes with wide batch groups (b up to 2^8) and
    narrow M / N; sparse and lattice graphs give the wide tiles.  Every node of
    every algebra must get a launch shape the kernels accept."""
    graphs = [gg.gnp(n, p, 700 + n) for n in (10, 16, 20, 24) for p in (0.3, 0.6, 0.9)]
    graphs += [gg.complete(12), gg.complete_bipartite(8, 9), gg.square_lattice(10), gg.kings_subgraph(10, 0.8, 1),
               gg.random_regular(120, 3, 0)]
    seen = set()
    for g in graphs:
        net = tn.Net.from_graph(g)
        for kw in ({"seed": 0}, {"method": "treesa", "ntrials": 1, "niters": 2, "seed": 1}):
            plan = tn.Plan.create(net, **kw)
            for sr in SEMIRINGS:
                for row in plan.gemm_shapes(sr):
                    seen.add((sr, row["kind"]))
                    assert row["valid"] == 1, (g.name, kw, sr, row)
    # the sweep reaches the small-tile, register-tiled and long-K families
    kinds = {k for _, k in seen}
    assert {"gemm", "gemm_big", "gemm_dot", "gemm_mfma"} <= kinds, kinds


def test_open_vertices_stay_to_the_root_and_are_never_sliced():
    g = gg.random_regular(40, 3, 0)
    net = tn.Net.from_graph(g)
    opn = [5, 3, 17]
    for kw in ({"seed": 0}, {"method": "treesa", "ntrials": 1, "niters": 3, "seed": 0},
               {"method": "treesa", "ntrials": 1, "niters": 3, "seed": 0, "sc_target": 6, "nslices": 4}):
        plan = tn.Plan.create(net, open=opn, **kw)
        e = plan.export()
        assert e["indices"][-1] == sorted(opn)  # the root's indices
        assert not set(e["sliced"]) & set(opn)
        for sr in SEMIRINGS:
            assert all(r["valid"] for r in plan.gemm_shapes(sr))
    assert tn.Plan.create(net, method="treesa", ntrials=1, niters=3, seed=0, sc_target=6, nslices=4,
                          open=opn).info()["nsliced"] > 0
    # an isolated open vertex (its only tensor is its own leaf) stays open too
    iso = tn.Net.from_graph(gg.disjoint_union(gg.path(3), gg.empty(1)))
    assert tn.Plan.create(iso, open=[3]).export()["indices"][-1] == [3]
    for bad in ([40], [1, 1], list(range(17)), [-1]):
        with pytest.raises(tn.TnError) as ei:
            tn.Plan.create(net, open=bad)
        assert ei.value.code == tn.TN_EINVAL


def test_wide_tree_reaches_2_30_entries_on_the_register_tiled_kernels():
    """The explicit tree of the full-size parity tests (3 x 29 grid): its
    largest tensors have 2^30 entries, every node's launch shape is one the
    kernels accept, the 2^35-operation node runs on the register-tiled VALU
    kernels (matrix cores for Z), and the oracle's plan follower accepts the
    tree's index lists on a narrower grid built the same way."""
    import sys
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from wide_trees import three_row_gemm_tree

    g = gg.grid(3, 29)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.from_tree(net, *three_row_gemm_tree(29, 5, g.edges))
    info = plan.info()
    assert info["max_rank"] == 30 and info["nsliced"] == 0
    for sr, kind in (("tropical_i32", "gemm_big"), ("tropical_f32", "gemm_big"), ("counting_tropical", "gemm_big"),
                     ("count_exact", "gemm_big"), ("partition_f32", "gemm_mfma")):
        rows = plan.gemm_shapes(sr)
        assert all(r["valid"] for r in rows)
        big = [r for r in rows if r["lb"] + r["li"] + r["lj"] + r["lk"] == 35]
        assert len(big) == 1 and big[0]["kind"] == kind, (sr, big)
        assert (big[0]["li"], big[0]["lj"], big[0]["lk"]) == (24, 6, 5)
    # the same construction on a 3 x 9 grid: O3 follows the exported tree and
    # agrees with brute force
    g9 = gg.grid(3, 9)
    p9 = tn.Plan.from_tree(tn.Net.from_graph(g9), *three_row_gemm_tree(9, 3, g9.edges))
    assert p9.info()["max_rank"] == 10
    tree = p9.export()
    bf = oracle.brute_force(g9)
    ct = oracle.follow_plan(g9, tree, "counting_tropical")
    assert (ct["size"], ct["count"]) == (bf["size_max"], bf["count_max"])
    assert oracle.follow_plan(g9, tree, "count")["count"] == bf["count_all"]


def test_tuning_table_file_overrides_the_heuristic(tmp_path):
    """A table entry (tn_tune_load) replaces the heuristic launch shape of
    exactly its node shape; entries the kernels do not accept are refused
    with nothing of the file taken; save / clear / load round-trip."""
    tn.tune_clear()
    net = tn.Net.from_graph(gg.random_regular(120, 3, 0))
    plan = tn.Plan.create(net, method="treesa", ntrials=2, niters=5, seed=0)
    rows = plan.gemm_shapes("tropical_f32")
    rows_i32 = plan.gemm_shapes("tropical_i32")
    big = [r for r in rows if r["kind"] == "gemm_big" and r["tk"] >= 2]
    assert big, "the n=120 plan has a register-tiled node"
    r0 = big[0]
    key = (1, r0["lb"], r0["li"], r0["lj"], r0["lk"], r0["a_t"], r0["b_t"])
    entry = "%d %d %d %d %d %d %d : 0 0 %d %d %d 8 8 0 0\n" % (key + (r0["ti"], r0["tj"], r0["tk"] - 1))
    path = tmp_path / "tiles.tune"
    path.write_text("# comment\n" + entry)
    assert tn.tune_load(str(path)) == 1
    same = lambda r: (1, r["lb"], r["li"], r["lj"], r["lk"], r["a_t"], r["b_t"]) == key
    for r in plan.gemm_shapes("tropical_f32"):
        want_tk = r0["tk"] - 1 if same(r) else next(x for x in rows if x["node"] == r["node"])["tk"]
        assert r["tk"] == want_tk and r["valid"] == 1
    # the other algebras keep the heuristic
    assert plan.gemm_shapes("tropical_i32") == rows_i32
    out = tmp_path / "saved.tune"
    assert tn.tune_save(str(out)) == 1
    assert entry.split(":")[1].split() == out.read_text().splitlines()[1].split(":")[1].split()
    # unusable entries: a tile larger than the node, a K step beyond K, garbage
    for bad in ("%d %d %d %d %d %d %d : 0 0 %d %d %d 8 8 0 0\n" % (key + (8, 8, 5)),
                "%d %d %d %d %d %d %d : 0 0 %d %d %d 8 8 0 0\n" % (key + (r0["ti"], r0["tj"], r0["lk"] + 1)),
                "1 2 3 : 0\n"):
        p2 = tmp_path / "bad.tune"
        p2.write_text(entry + bad)
        tn.tune_clear()
        with pytest.raises(tn.TnError) as ei:
            tn.tune_load(str(p2))
        assert ei.value.code == tn.TN_EINVAL
        assert plan.gemm_shapes("tropical_f32") == rows  # nothing taken
    tn.tune_clear()
    assert plan.gemm_shapes("tropical_f32") == rows
    assert tn.tune_load(str(out)) == 1
    tn.tune_clear()


def test_committed_tuning_table_loads():
    """The table the benchmark uses (written by bench.py --tune-out on an
    MI355X) holds only entries the kernels accept."""
    path = os.path.join(ROOT, "paper_2501_00227_amd", "mi355x_tiles.tune")
    tn.tune_clear()
    n = tn.tune_load(path)
    lines = [l for l in open(path) if l.strip() and not l.startswith("#")]
    assert n == len(lines) > 50
    tn.tune_clear()
