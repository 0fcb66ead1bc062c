"""GPU tests of open vertices (the open vertices of the Sec. 5 network
object): the contraction keeps them to the root, whose entries are the
property restricted to each assignment of the open vertices.  Entry e is the
oracle's brute force with the open vertices fixed to the bits of e; on larger
graphs, the oracle's elimination on the reduced graph."""
import math
import random

import pytest

import graphgen as gg
import oracle
import paper_2501_00227_amd as tn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    tn.lib()
    c = tn.Context(0)
    yield c
    c.synchronize()


def _assignment(opn, e):
    return {v: (e >> q) & 1 for q, v in enumerate(opn)}


def _reduced(g, fixed):
    adj = g.adjacency()
    drop = set(fixed)
    for v, x in fixed.items():
        if x == 1:
            drop.update(adj[v])
    return gg.induced(g, [v for v in range(g.nv) if v not in drop])


@pytest.mark.parametrize("sliced", [False, True])
def test_small_graphs_vs_brute_force(ctx, sliced):
    rng = random.Random(31 + sliced)
    for t in range(8):
        n = rng.randint(6, 16)
        g = gg.gnp(n, rng.uniform(0.2, 0.5), 800 + t)
        if t % 2:
            g = g.with_weights(gg.integer_weights(n, 800 + t, 1, 4))
        opn = rng.sample(range(n), rng.randint(1, 4))
        net = tn.Net.from_graph(g)
        kw = {"method": "treesa", "ntrials": 1, "niters": 3, "sc_target": 2, "nslices": 3} if sliced else {}
        plan = tn.Plan.create(net, seed=t, open=opn, **kw)
        if sliced:
            print(f"t={t}: {plan.info()['nsliced']} sliced", flush=True)
        res = {sr: ctx.solve_open(net, plan, sr, beta=0.5)
               for sr in ("tropical_i32", "tropical_f32", "counting_tropical", "count_exact", "partition_f32")}
        for e in range(1 << len(opn)):
            bf = oracle.brute_force(g, betas=[0.5], fixed=_assignment(opn, e))
            assert res["count_exact"][e]["count"] == bf["count_all"], (t, e)
            assert res["tropical_i32"][e]["size"] == bf["size_max"], (t, e)
            assert res["tropical_f32"][e]["size"] == bf["size_max"], (t, e)
            ct = res["counting_tropical"][e]
            want_ct = (bf["size_max"], bf["count_max"]) if bf["count_all"] else (float("-inf"), 0)
            assert (ct["size"], ct["count_mod_2_64"]) == want_ct, (t, e)
            if bf["count_all"]:
                assert abs(res["partition_f32"][e]["log_z"] - bf["log_z"][0]) <= 1e-5, (t, e)


def test_marginals_on_a_3_regular_graph(ctx):
    g = gg.random_regular(60, 3, 4)
    opn = [7, 0, 33]
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=2, niters=5, seed=4, open=opn)
    cnt = ctx.solve_open(net, plan, "count_exact")
    ct = ctx.solve_open(net, plan, "counting_tropical")
    z = ctx.solve_open(net, plan, "partition_f32", beta=0.3)
    total = oracle.eliminate(g, "count")["count"]
    assert sum(r["count"] for r in cnt) == total
    zall = oracle.eliminate(g, "partition", beta=0.3)["log_z"]
    lz = [r["log_z"] for r in z if r["log_z"] != float("-inf")]
    m = max(lz)
    assert abs(m + math.log(sum(math.exp(x - m) for x in lz)) - zall) <= 1e-5
    for e in range(8):
        fixed = _assignment(opn, e)
        red = _reduced(g, fixed)
        feasible = all(not (fixed.get(u) == 1 and fixed.get(v) == 1) for u, v in g.edges.tolist())
        if not feasible:
            assert cnt[e]["count"] == 0
            continue
        want = oracle.eliminate(red, "counting_tropical")
        ones = sum(fixed.values())
        assert cnt[e]["count"] == oracle.eliminate(red, "count")["count"], e
        assert (ct[e]["size"], ct[e]["count_mod_2_64"]) == (want["size"] + ones, want["count"] % 2 ** 64), e


def test_spin_glass_open_spins(ctx):
    rng = random.Random(37)
    n = 12
    g = gg.gnp(n, 0.4, 870)
    J = [float(rng.randint(-2, 2)) for _ in range(g.ne)]
    h = [float(rng.randint(-1, 1)) for _ in range(n)]
    opn = [2, 9]
    net = tn.Net.spin_glass(g, J, h)
    plan = tn.Plan.create(net, seed=1, open=opn)
    ct = ctx.solve_open(net, plan, "counting_tropical")
    z = ctx.solve_open(net, plan, "partition_f32", beta=0.6)
    for e in range(4):
        bf = oracle.spin_glass_brute_force(g, J, h, betas=[0.6], fixed=_assignment(opn, e))
        assert (-ct[e]["size"], ct[e]["count_mod_2_64"]) == (bf["energy_min"], bf["count_min"]), e
        assert abs(z[e]["log_z"] - bf["log_z"][0]) <= 1e-5, e


def test_open_plans_need_the_tensor_entry_point(ctx):
    g = gg.random_regular(20, 3, 0)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, open=[1, 2])
    for ex in ("auto", "stream", "persistent"):
        with pytest.raises(tn.TnError) as ei:
            ctx.solve(net, plan, "count_exact", executor=ex)
        assert ei.value.code == tn.TN_EINVAL
    with pytest.raises(tn.TnError) as ei:
        ctx.solve_batch([net], [plan], "count_exact")
    assert ei.value.code == tn.TN_EINVAL
    # a plan without open vertices gives one entry, equal to tn_solve
    closed = tn.Plan.create(net)
    one = ctx.solve_open(net, closed, "count_exact")
    assert len(one) == 1 and one[0]["count"] == ctx.solve(net, closed, "count_exact")["count"]
