"""The partition function's reported dynamic range (tn_result.z_range_log2).

Every Z contraction reports the largest log2(max / smallest nonzero entry)
over the tensors it stores (float32 entries under one power-of-two exponent
per tensor), or over the two operands of a product added together (the span
their products need).  On small graphs the value is checked against every
node tensor of the plan computed by brute force from the definition (a
node's tensor is the sum, over the assignments of its subtree's vertices
with its open indices fixed, of the product of its leaves' factors), on both
executors; at a large beta, where small products underflow, it passes 100.
"""
import math

import numpy as np
import pytest

import graphgen as gg
import paper_2501_00227_amd as tn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    tn.lib()
    c = tn.Context(0)
    yield c
    c.synchronize()


def _brute_force_range(g, plan, beta):
    """max over the plan's node tensors of log2(max / smallest nonzero)."""
    t = plan.export()
    n = g.nv
    edges = g.edges.tolist()
    w = g.weights if g.weights is not None else np.ones(n)
    x = (np.arange(1 << n)[:, None] >> np.arange(n)[None, :]) & 1  # every assignment, one row each
    nl = len(t["leaf_factors"])
    fac_val = {}

    def factor(f):
        if f not in fac_val:
            if f >= 0:
                u, v = edges[f]
                fac_val[f] = np.where((x[:, u] == 1) & (x[:, v] == 1), 0.0, 1.0)
            else:
                v = -f - 1
                fac_val[f] = np.where(x[:, v] == 1, math.exp(beta * float(w[v])), 1.0)
        return fac_val[f]

    prod = [None] * (nl + len(t["left"]))
    for leaf, facs in enumerate(t["leaf_factors"]):
        p = np.ones(1 << n)
        for f in facs:
            p = p * factor(f)
        prod[leaf] = p
    for k, (a, b) in enumerate(zip(t["left"], t["right"])):
        prod[nl + k] = prod[a] * prod[b]
    rng = []
    for node, p in enumerate(prod):
        idx = t["indices"][node]
        key = np.zeros(1 << n, np.int64)
        for q, v in enumerate(idx):
            key |= x[:, v].astype(np.int64) << q
        tens = np.bincount(key, weights=p, minlength=1 << len(idx))  # vertices outside the subtree: a common factor
        nz = tens[tens > 0]
        rng.append(math.log2(nz.max()) - math.log2(nz.min()))
    # a product node also spans the sum of its operands' ranges
    return max(rng + [rng[a] + rng[b] for a, b in zip(t["left"], t["right"])])


@pytest.mark.parametrize("name,seed", [("rr12", 1), ("gnp11", 2), ("ksg", 3)])
def test_range_matches_brute_force_of_every_node_tensor(ctx, name, seed):
    g = {"rr12": gg.random_regular(12, 3, seed), "gnp11": gg.gnp(11, 0.3, seed),
         "ksg": gg.kings_subgraph(4, 0.8, seed)}[name]
    g = g.with_weights(gg.dyadic_weights(g.nv, seed))
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, seed=seed)
    for beta in (0.5, 2.0):
        want = _brute_force_range(g, plan, beta)
        for ex in ("stream", "persistent"):
            r = ctx.solve(net, plan, "partition_f32", beta=beta, executor=ex)
            print(f"{name} beta {beta} {ex}: range {r['z_range_log2']:.5f} vs {want:.5f}", flush=True)
            assert abs(r["z_range_log2"] - want) <= 1e-3 * max(1.0, want)


def test_range_grows_with_beta_and_flags_flushing(ctx):
    g = gg.random_regular(40, 3, 0)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, seed=0)
    r1 = ctx.solve(net, plan, "partition_f32", beta=1.0)
    r8 = ctx.solve(net, plan, "partition_f32", beta=8.0)
    # a vertex tensor alone spans e^beta
    assert r1["z_range_log2"] >= math.log2(math.e) - 1e-4
    assert r8["z_range_log2"] > r1["z_range_log2"]
    r = ctx.solve(net, plan, "partition_f32", beta=60.0)
    print("ranges", r1["z_range_log2"], r8["z_range_log2"], r["z_range_log2"], flush=True)
    assert r["z_range_log2"] > 100  # terms far below a tensor's maximum flush at this beta
    rs = ctx.solve(net, plan, "tropical_i32")
    assert rs.get("z_range_log2", 0.0) == 0.0
