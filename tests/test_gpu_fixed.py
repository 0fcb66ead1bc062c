"""GPU tests of fixed vertices (conditioning; the fixed vertices of the Sec. 5
network object): a conditioned copy of a network runs on the plan of the
original, every algebra on both executors, against the oracle's brute force
with the same fixings, and on larger graphs against the oracle's elimination
on the reduced graph (fixing n_v = 0 deletes v; n_v = 1 deletes v's closed
neighbourhood and adds v's weight)."""
import math
import random

import numpy as np
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


def _random_fixing(rng, g, k):
    adj = g.adjacency()
    fixed = {}
    for v in rng.sample(range(g.nv), min(k, g.nv)):
        # keep it feasible: a vertex next to one fixed to 1 is fixed to 0
        fixed[v] = 0 if any(fixed.get(u) == 1 for u in adj[v]) else rng.randint(0, 1)
    return fixed


def _reduced(g, fixed):
    adj = g.adjacency()
    drop = set(fixed)
    for v, x in fixed.items():
        if x == 1:
            drop.update(adj[v])
    return gg.induced(g, [v for v in range(g.nv) if v not in drop])


def test_small_graphs_vs_brute_force(ctx):
    rng = random.Random(23)
    for t in range(12):
        n = rng.randint(2, 16)
        g = gg.gnp(n, rng.uniform(0.15, 0.6), 500 + t)
        if t % 2:
            g = g.with_weights(gg.integer_weights(n, 500 + t, 1, 4))
        fixed = _random_fixing(rng, g, rng.randint(1, 4))
        bf = oracle.brute_force(g, betas=[0.5], fixed=fixed)
        base = tn.Net.from_graph(g)
        net = base.condition(fixed)
        plan = tn.Plan.create(base, seed=t)  # the original's plan fits the copy
        for ex in ("stream", "persistent"):
            ct = ctx.solve(net, plan, "counting_tropical", executor=ex)
            assert (ct["size"], ct["count_mod_2_64"]) == (bf["size_max"], bf["count_max"]), (t, ex, fixed)
            assert ctx.solve(net, plan, "tropical_i32", executor=ex)["size"] == bf["size_max"]
            assert ctx.solve(net, plan, "tropical_f32", executor=ex)["size"] == bf["size_max"]
            assert ctx.solve(net, plan, "count_exact", executor=ex)["count"] == bf["count_all"]
            z = ctx.solve(net, plan, "partition_f32", beta=0.5, executor=ex)["log_z"]
            assert abs(z - bf["log_z"][0]) <= 1e-5, (t, ex)
        if g.weights is None:
            poly = bf["poly"]
            while len(poly) > 1 and poly[-1] == 0:
                poly.pop()
            assert ctx.solve_polynomial(net, plan) == poly
        r = ctx.solve_single_config_max(net, plan)
        assert r["value"] == bf["size_max"]
        assert all(r["config"][v] == x for v, x in fixed.items())
        # the unconditioned network is unchanged
        assert ctx.solve(base, plan, "count_exact")["count"] == oracle.brute_force(g)["count_all"]


@pytest.mark.parametrize("n,seed", [(60, 0), (120, 1)])
def test_regular_graphs_vs_reduced_elimination(ctx, n, seed):
    g = gg.random_regular(n, 3, seed).with_weights(gg.dyadic_weights(n, seed))
    rng = random.Random(seed)
    fixed = _random_fixing(rng, g, 12)
    red = _reduced(g, fixed)
    offset = sum(float(g.weights[v]) for v, x in fixed.items() if x == 1)
    base = tn.Net.from_graph(g)
    net = base.condition(fixed)
    plan = tn.Plan.create(base, method="treesa", ntrials=2, niters=5, seed=seed)
    want_size = oracle.eliminate(red, "tropical")["size"] + offset
    want_z = oracle.eliminate(red, "partition", beta=0.5)["log_z"] + 0.5 * offset
    print(f"n={n}: fixed {len(fixed)}, reduced graph {red.nv} vertices", flush=True)
    ug = gg.random_regular(n, 3, seed)  # unit weights for the counting algebras
    ured = _reduced(ug, fixed)
    want_ct = oracle.eliminate(ured, "counting_tropical")
    ones = sum(fixed.values())
    ubase = tn.Net.from_graph(ug)
    unet = ubase.condition(fixed)
    uplan = tn.Plan.create(ubase, method="treesa", ntrials=2, niters=5, seed=seed)
    for ex in ("stream", "persistent"):
        assert ctx.solve(net, plan, "tropical_f32", executor=ex)["size"] == want_size
        assert abs(ctx.solve(net, plan, "partition_f32", beta=0.5, executor=ex)["log_z"] - want_z) <= 1e-5
        ct = ctx.solve(unet, uplan, "counting_tropical", executor=ex)
        assert (ct["size"], ct["count_mod_2_64"]) == (want_ct["size"] + ones, want_ct["count"] % 2 ** 64)
    assert ctx.solve(unet, uplan, "count_exact")["count"] == oracle.eliminate(ured, "count")["count"]
    r = ctx.solve_single_config_max(net, plan)
    assert r["value"] == want_size
    assert all(r["config"][v] == x for v, x in fixed.items())
    assert sum(float(g.weights[v]) for v in range(n) if r["config"][v]) == want_size
    for u, v in g.edges.tolist():
        assert not (r["config"][u] and r["config"][v])


def test_batched_mix_of_fixings(ctx):
    """One persistent launch over several fixings of one network."""
    g = gg.random_regular(40, 3, 7)
    base = tn.Net.from_graph(g)
    plan = tn.Plan.create(base, seed=7)
    rng = random.Random(7)
    fixings = [_random_fixing(rng, g, k) for k in (0, 1, 3, 6, 10)]
    nets = [base.condition(f) for f in fixings]
    res = ctx.solve_batch(nets, [plan] * len(nets), "counting_tropical")
    for f, r in zip(fixings, res):
        want = oracle.eliminate(_reduced(g, f), "counting_tropical")
        off = sum(1 for x in f.values() if x == 1)
        assert (r["size"], r["count_mod_2_64"]) == (want["size"] + off, want["count"] % 2 ** 64), f


def test_spin_glass_fixed_spins(ctx):
    rng = random.Random(29)
    for t in range(8):
        n = rng.randint(3, 14)
        g = gg.gnp(n, rng.uniform(0.2, 0.6), 600 + t)
        J = [float(rng.randint(-2, 2)) for _ in range(g.ne)]
        h = [float(rng.randint(-1, 1)) for _ in range(n)]
        fixed = {v: rng.randint(0, 1) for v in rng.sample(range(n), rng.randint(1, 3))}
        bf = oracle.spin_glass_brute_force(g, J, h, betas=[0.7], fixed=fixed)
        base = tn.Net.spin_glass(g, J, h)
        net = base.condition(fixed)
        plan = tn.Plan.create(base, seed=t)
        for ex in ("stream", "persistent"):
            ct = ctx.solve(net, plan, "counting_tropical", executor=ex)
            assert (-ct["size"], ct["count_mod_2_64"]) == (bf["energy_min"], bf["count_min"]), (t, ex)
            z = ctx.solve(net, plan, "partition_f32", beta=0.7, executor=ex)["log_z"]
            assert abs(z - bf["log_z"][0]) <= 1e-5
            assert ctx.solve(net, plan, "count_exact", executor=ex)["count"] == 2 ** (n - len(fixed))
        r = ctx.solve_single_config_max(net, plan)
        assert r["value"] == -bf["energy_min"] and all(r["config"][v] == x for v, x in fixed.items())


def test_infeasible_and_invalid_fixings(ctx):
    g = gg.path(4)
    base = tn.Net.from_graph(g)
    plan = tn.Plan.create(base)
    net = base.condition({1: 1, 2: 1})  # both ends of an edge in the set
    assert ctx.solve(net, plan, "count_exact")["count"] == 0
    assert ctx.solve(net, plan, "tropical_i32")["size"] == float("-inf")
    assert ctx.solve(net, plan, "tropical_f32")["size"] == float("-inf")
    with pytest.raises(tn.TnError) as ei:
        ctx.solve_single_config_max(net, plan)
    assert ei.value.code == tn.TN_EINVAL
    for bad in ({4: 0}, {-1: 1}, {0: 2}):
        with pytest.raises(tn.TnError) as ei:
            base.condition(bad)
        assert ei.value.code == tn.TN_EINVAL
    with pytest.raises(tn.TnError) as ei:
        base.condition({0: 1}).condition({0: 0})
    assert ei.value.code == tn.TN_EINVAL
    both = base.condition({0: 1}).condition({3: 1})
    assert ctx.solve(both, plan, "count_exact")["count"] == oracle.brute_force(g, fixed={0: 1, 3: 1})["count_all"] == 1
    assert math.isfinite(ctx.solve(both, plan, "partition_f32", beta=1.0)["log_z"])
    assert np.isclose(ctx.solve(both, plan, "partition_f32", beta=1.0)["log_z"], 2.0)
