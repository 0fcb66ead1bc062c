"""GPU parity: the HIP path against the CPU oracle on the same seeded inputs.

Integer algebras (tropical int32, counting tropical, exact counts) must be
bit-exact; tropical float32 is exact on dyadic weights; the float32 partition
function must be within 1e-5 relative of the oracle's extended-precision
value; bfloat16-input Z is reported against a loose bound only.
"""
import json
import math
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2501_00227_amd as tn

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
Z_RTOL = 1e-5


@pytest.fixture(scope="module")
def ctx():
    tn.lib()  # fails loudly when the library is not built
    c = tn.Context(0)
    yield c
    c.synchronize()


def _small_graphs():
    gs = [gg.petersen(), gg.path(1), gg.path(2), gg.path(7), gg.cycle(9), gg.complete(6), gg.empty(5),
          gg.complete_bipartite(3, 4), gg.star(6), gg.disjoint_union(gg.cycle(5), gg.empty(2))]
    for s in range(12):
        gs.append(gg.random_regular(2 * (5 + s % 4), 3, s))
        gs.append(gg.gnp(8 + s % 8, 0.25, s))
        gs.append(gg.kings_subgraph(4, 0.8, s))
    return gs


def _weighted(g, s):
    if s % 3 == 1:
        return g.with_weights(gg.dyadic_weights(g.nv, s))
    if s % 3 == 2:
        return g.with_weights(gg.integer_weights(g.nv, s, 1, 4))
    return g


def _check_all(ctx, g, plan_kw, beta=0.7, label="", executor="auto"):
    ref = oracle.brute_force(g, [beta])
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, **plan_kw)
    integer = g.weights is None or np.all(g.weights == np.round(g.weights))
    print(f"case {label} {g.name} nv={g.nv} ne={g.ne} plan={plan_kw} executor={executor}", flush=True)
    ex = {"executor": executor}
    if integer:
        r = ctx.solve(net, plan, "tropical_i32", **ex)
        assert r["size"] == ref["size_max"], (label, r, ref)
        r = ctx.solve(net, plan, "counting_tropical", **ex)
        assert (r["size"], r["count_mod_2_64"]) == (ref["size_max"], ref["count_max"]), (label, r, ref)
    r = ctx.solve(net, plan, "tropical_f32", **ex)
    assert r["size"] == pytest.approx(ref["size_max"], abs=0), (label, r, ref)
    r = ctx.solve(net, plan, "count_exact", **ex)
    assert r["count"] == ref["count_all"], (label, r, ref)
    assert r["count_mod_2_64"] == ref["count_all"] % (1 << 64)
    r = ctx.solve(net, plan, "partition_f32", beta=beta, **ex)
    assert abs(r["z"] - ref["z"][0]) <= Z_RTOL * ref["z"][0], (label, r, ref)
    r = ctx.solve(net, plan, "partition_bf16", beta=beta, **ex)
    assert abs(r["z"] - ref["z"][0]) <= 5e-2 * ref["z"][0], (label, r, ref)


@pytest.mark.parametrize("absorb", [True, False])
@pytest.mark.parametrize("executor", ["stream", "persistent"])
def test_small_graphs_every_algebra(ctx, absorb, executor):
    for s, g in enumerate(_small_graphs()):
        _check_all(ctx, _weighted(g, s), {"absorb": absorb, "seed": s}, label=f"s{s}", executor=executor)


def test_empty_network(ctx):
    net = tn.Net(0, np.zeros((0, 2), np.int32))
    plan = tn.Plan.create(net)
    assert ctx.solve(net, plan, "count_exact")["count"] == 1
    assert ctx.solve(net, plan, "tropical_i32")["size"] == 0
    assert ctx.solve(net, plan, "partition_f32", beta=1.0)["z"] == 1.0


@pytest.mark.parametrize("executor", ["stream", "persistent"])
def test_treesa_plans(ctx, executor):
    for s in range(4):
        g = _weighted(gg.random_regular(16, 3, 100 + s), s)
        _check_all(ctx, g, {"method": "treesa", "ntrials": 2, "niters": 5, "seed": s}, label=f"sa{s}",
                   executor=executor)


def test_sliced_plans_match(ctx):
    for s in range(6):
        g = _weighted(gg.random_regular(18, 3, 200 + s), s)
        _check_all(ctx, g, {"sc_target": 2, "nslices": 1 + s % 4, "seed": s}, label=f"slice{s}")


def test_paper_tree_on_the_square(ctx):
    # the contraction tree printed in Sec. 4.1 for the 4-cycle (vertices 1..4)
    edges = np.array([[0, 1], [1, 2], [2, 3], [0, 3]], np.int32)
    net = tn.Net(4, edges)
    # leaves: edges (1,2),(2,3),(3,4),(4,1) then vertices 1..4
    leaves = [[0], [1], [2], [3], [-1], [-2], [-3], [-4]]
    # N6 = (3∘4, 3); N5 = (N6, 4); N4 = (2, 2∘3); N3 = (N4, N5); N2 = (N3, 1∘2); N1 = (4∘1, N2); root = (N1, 1)
    left = [2, 8, 5, 10, 11, 3, 13]
    right = [6, 7, 1, 9, 0, 12, 4]
    plan = tn.Plan.from_tree(net, leaves, left, right)
    assert ctx.solve(net, plan, "count_exact")["count"] == 7
    r = ctx.solve(net, plan, "counting_tropical")
    assert (r["size"], r["count_mod_2_64"]) == (2.0, 2)


def test_k1_counting_tropical_twenty_seeds(ctx):
    gold = json.load(open(os.path.join(GOLD, "k1.json")))["cases"]
    for case in gold:
        g = gg.random_regular(20, 3, case["seed"])
        net = tn.Net.from_graph(g)
        plan = tn.Plan.create(net, seed=case["seed"])
        assert plan.complexity()[1] <= 8
        r = ctx.solve(net, plan, "counting_tropical")
        assert (r["size"], r["count_mod_2_64"]) == (case["size_max"], case["count_max"]), case


@pytest.mark.parametrize("method,executor", [("greedy", "stream"), ("treesa", "stream"), ("treesa", "persistent")])
def test_k2_three_contractions(ctx, method, executor):
    gold = json.load(open(os.path.join(GOLD, "k2.json")))["cases"]
    for case in gold:
        g = gg.random_regular(120, 3, case["seed"])
        net = tn.Net.from_graph(g)
        kw = {"seed": case["seed"]}
        if method == "treesa":
            kw.update(method="treesa", ntrials=4, niters=10)
        plan = tn.Plan.create(net, **kw)
        print(f"k2 seed {case['seed']} {method} {executor} complexity {plan.complexity()}", flush=True)
        r = ctx.solve(net, plan, "tropical_i32", executor=executor)
        assert r["size"] == case["size_max"]
        r = ctx.solve(net, plan, "count_exact", executor=executor)
        assert r["count"] == int(case["count_all"])
        assert r["count"] > 2 ** 64  # the CRT result needs more than 64 bits
        r = ctx.solve(net, plan, "counting_tropical", executor=executor)
        assert r["count_mod_2_64"] == int(case["count_max"])
        r = ctx.solve(net, plan, "partition_f32", beta=0.0, executor=executor)
        assert abs(r["log_z"] - case["log_z_beta0"]) <= Z_RTOL, (r, case)


def test_integer_algebras_are_deterministic(ctx):
    g = gg.random_regular(60, 3, 7)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, seed=7)
    for sr in ("tropical_i32", "counting_tropical", "count_exact"):
        a = ctx.solve(net, plan, sr)
        b = ctx.solve(net, plan, sr)
        a.pop("seconds")
        b.pop("seconds")
        assert a == b, sr


def test_plan_for_another_network_is_rejected(ctx):
    n1 = tn.Net.from_graph(gg.cycle(6))
    n2 = tn.Net.from_graph(gg.path(6))
    p1 = tn.Plan.create(n1)
    with pytest.raises(tn.TnError) as ei:
        ctx.solve(n2, p1, "count_exact")
    assert ei.value.code == tn.TN_EINVAL


def test_integer_algebra_rejects_fractional_weights(ctx):
    g = gg.cycle(5).with_weights(np.array([0.5, 1, 1, 1, 1], np.float32))
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net)
    with pytest.raises(tn.TnError):
        ctx.solve(net, plan, "tropical_i32")
    assert ctx.solve(net, plan, "tropical_f32")["size"] == oracle.brute_force(g)["size_max"]


def test_exact_count_range_and_overflow(ctx):
    """Counts are exact below the product of the CRT primes and flagged above
    it by the check prime.  By default the number of primes follows an upper
    bound on the count (at most sixteen primes, fifteen of them for CRT,
    about 2^449); given primes set the range.  The empty graph on n vertices
    has 2^n independent sets."""
    for n in (140, 160, 200, 300, 440):
        net = tn.Net.from_graph(gg.empty(n))
        r = ctx.solve(net, tn.Plan.create(net), "count_exact")
        assert r["count"] == 2 ** n and r["count_mod_2_64"] == 0
        assert len(r["primes"]) >= (n + 29) // 30 + 1
    net = tn.Net.from_graph(gg.empty(480))
    with pytest.raises(tn.TnError) as ei:
        ctx.solve(net, tn.Plan.create(net), "count_exact")
    assert ei.value.code == tn.TN_EOVERFLOW
    net = tn.Net.from_graph(gg.empty(40))
    plan = tn.Plan.create(net)
    with pytest.raises(tn.TnError) as ei:  # one CRT prime: range below 2^30
        ctx.solve(net, plan, "count_exact", primes=[1073741789, 1073741783])
    assert ei.value.code == tn.TN_EOVERFLOW
    primes = [1073741789, 1073741783, 1073741741]
    r = ctx.solve(net, plan, "count_exact", primes=primes)
    assert r["count"] == 2 ** 40
    assert r["primes"] == primes and all(res == pow(2, 40, p) for res, p in zip(r["residues"], primes))


def test_solve_log_lines(ctx, tmp_path, monkeypatch):
    """TN_LOG: one JSON line per tn_solve with the plan's complexity, the
    executor and the result's key values."""
    path = tmp_path / "solves.jsonl"
    monkeypatch.setenv("TN_LOG", str(path))
    g = gg.random_regular(20, 3, 0)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net)
    ref = oracle.brute_force(g, [0.5])
    r1 = ctx.solve(net, plan, "counting_tropical", executor="stream")
    r2 = ctx.solve(net, plan, "partition_f32", beta=0.5, executor="persistent")
    monkeypatch.delenv("TN_LOG")
    ctx.solve(net, plan, "tropical_i32")  # not logged
    lines = [json.loads(x) for x in path.read_text().splitlines()]
    assert len(lines) == 2
    tc, sc, rwc = plan.complexity()
    assert lines[0]["status"] == 0 and lines[0]["executor"] == "per-node"
    assert (lines[0]["size"], lines[0]["count_mod_2_64"]) == (r1["size"], r1["count_mod_2_64"]) == \
        (ref["size_max"], ref["count_max"])
    assert lines[1]["executor"] == "persistent" and abs(lines[1]["log_z"] - r2["log_z"]) < 1e-12
    assert all(abs(x["tc_log2"] - tc) < 1e-3 and abs(x["sc_log2"] - sc) < 1e-3 for x in lines)
