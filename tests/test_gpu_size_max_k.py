"""GPU tests of SizeMax(k) for any weights (Sec. 5 table; Sec. 5.3 shows the
Petersen value): max-plus over lists of the eight largest values, on both
executors.  Checked against the paper's Petersen value, the oracle's
enumeration (weighted independent sets, spin glasses, fixed vertices, a
sliced plan) and, at n = 60, the expansion of the oracle's independence
polynomial."""
import itertools
import json
import os
import random

import pytest

import graphgen as gg
import oracle
import paper_2501_00227_amd as tn

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


@pytest.fixture(scope="module")
def ctx():
    tn.lib()
    c = tn.Context(0)
    yield c
    c.synchronize()


EXECUTORS = ("stream", "persistent")


def test_petersen_matches_paper(ctx):
    net = tn.Net.from_graph(gg.petersen())
    plan = tn.Plan.create(net)
    for ex in EXECUTORS:
        assert ctx.solve_size_max_k(net, plan, 2, ex) == [float(x) for x in GOLD["petersen"]["size_max_2"]["value"]]
        assert ctx.solve_size_max_k(net, plan, 8, ex) == oracle.brute_force_topk(gg.petersen(), 8)


@pytest.mark.parametrize("ex", EXECUTORS)
@pytest.mark.parametrize("weights", ["unit", "integer", "dyadic"])
def test_random_graphs_vs_enumeration(ctx, weights, ex):
    rng = random.Random({"unit": 1, "integer": 2, "dyadic": 3}[weights])
    for t in range(10):
        n = rng.randint(1, 18)
        g = gg.gnp(n, rng.uniform(0.1, 0.6), 1200 + t)
        if weights == "integer":
            g = g.with_weights(gg.integer_weights(n, 1200 + t, 1, 5))
        elif weights == "dyadic":
            g = g.with_weights(gg.dyadic_weights(n, 1200 + t))
        net = tn.Net.from_graph(g)
        plan = tn.Plan.create(net, seed=t)
        for k in (1, 4, 8):
            assert ctx.solve_size_max_k(net, plan, k, ex) == oracle.brute_force_topk(g, k), (t, k)


@pytest.mark.parametrize("ex", EXECUTORS)
def test_spin_glasses_and_fixed_vertices(ctx, ex):
    rng = random.Random(7)
    for t in range(8):
        n = rng.randint(3, 16)
        g = gg.gnp(n, rng.uniform(0.2, 0.6), 1300 + t)
        J = [float(rng.randint(-2, 2)) for _ in range(g.ne)]
        h = [float(rng.randint(-1, 1)) for _ in range(n)]
        net = tn.Net.spin_glass(g, J, h)
        plan = tn.Plan.create(net, seed=t)
        assert ctx.solve_size_max_k(net, plan, 8, ex) == oracle.spin_glass_topk(g, 8, J, h), t
        fixed = {v: rng.randint(0, 1) for v in rng.sample(range(n), 2)}
        assert ctx.solve_size_max_k(net.condition(fixed), plan, 5, ex) == oracle.spin_glass_topk(g, 5, J, h, fixed), t
        gw = g.with_weights(gg.integer_weights(n, 1300 + t, 1, 4))
        wnet = tn.Net.from_graph(gw)
        wplan = tn.Plan.create(wnet, seed=t)
        fixed = {v: 0 for v in rng.sample(range(n), 2)}
        assert ctx.solve_size_max_k(wnet.condition(fixed), wplan, 6, ex) == oracle.brute_force_topk(gw, 6, fixed), t


def test_sliced_plan(ctx):
    g = gg.random_regular(24, 3, 5).with_weights(gg.integer_weights(24, 5, 1, 6))
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=1, niters=3, sc_target=3, nslices=4, seed=5)
    assert plan.info()["nsliced"] > 0
    assert ctx.solve_size_max_k(net, plan, 8) == oracle.brute_force_topk(g, 8)
    with pytest.raises(tn.TnError) as ei:
        ctx.solve_size_max_k(net, plan, 8, "persistent")
    assert ei.value.code == tn.TN_EINVAL


@pytest.mark.parametrize("seed", [36, 5, 3])
def test_unit_weights_agree_with_the_polynomial(ctx, seed):
    """60-vertex 3-regular graphs with 1, 2 and 7 maximum sets, so the eight
    largest sizes reach below the maximum."""
    g = gg.random_regular(60, 3, seed)
    poly = oracle.eliminate_polynomial(g, max_width=20)["poly"]
    # the eight largest sizes with multiplicity (taken lazily: the counts are huge)
    expanded = list(itertools.islice((float(s) for s in range(len(poly) - 1, -1, -1) for _ in range(poly[s])), 8))
    assert expanded[-1] < expanded[0]
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=2, niters=5, seed=seed)
    for ex in EXECUTORS:
        assert ctx.solve_size_max_k(net, plan, 8, ex) == expanded
    assert ctx.solve_max_k(net, plan, 8)["size_max_k"] == [int(x) for x in expanded]


def test_weighted_regular_graph_largest_is_the_maximum(ctx):
    g = gg.random_regular(100, 3, 4).with_weights(gg.dyadic_weights(100, 4))
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=2, niters=5, seed=4)
    top = ctx.solve_size_max_k(net, plan, 8, "persistent")
    assert ctx.solve_size_max_k(net, plan, 8, "stream") == top
    assert top[0] == oracle.eliminate(g, "tropical")["size"]
    assert all(a >= b for a, b in zip(top, top[1:])) and top[-1] > float("-inf")


def test_rejections_and_empty_network(ctx):
    net = tn.Net.from_graph(gg.path(5))
    plan = tn.Plan.create(net)
    for k, ex in ((0, "auto"), (9, "auto"), (2, 3), (2, -1)):
        with pytest.raises(tn.TnError) as ei:
            ctx.solve_size_max_k(net, plan, k, ex)
        assert ei.value.code == tn.TN_EINVAL
    for ex in ("auto",) + EXECUTORS:
        with pytest.raises(tn.TnError) as ei:
            ctx.solve_size_max_k(net, tn.Plan.create(net, open=[1]), 2, ex)
        assert ei.value.code == tn.TN_EINVAL
    with pytest.raises(tn.TnError) as ei:
        ctx.solve_size_max_k(net, tn.Plan.create(tn.Net.from_graph(gg.path(6))), 2)
    assert ei.value.code == tn.TN_EINVAL
    e = tn.Net.from_graph(gg.empty(0))
    for ex in EXECUTORS:
        assert ctx.solve_size_max_k(e, tn.Plan.create(e), 3, ex) == [0.0, float("-inf"), float("-inf")]
