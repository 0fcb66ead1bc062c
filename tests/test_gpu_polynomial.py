"""GPU tests of the independence polynomial (Sec. 5.3 GraphPolynomial, the
finite-field method of Sec. 6.2): mod-p evaluations of the counting network
at x = 0 .. alpha in persistent launches, interpolation and CRT on the host.
Checked against the paper's Petersen polynomial, the oracle's brute-force
size histogram and its elimination over polynomial-valued tables, and, on the
120-vertex network, against identities every independence polynomial obeys.
"""
import itertools
import json
import math
import os

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


def _poly(ctx, g, **kw):
    net = tn.Net.from_graph(g)
    return ctx.solve_polynomial(net, tn.Plan.create(net, **kw))


def _trim(p):
    p = list(p)
    while len(p) > 1 and p[-1] == 0:
        p.pop()
    return p


def test_petersen_matches_paper(ctx):
    assert _poly(ctx, gg.petersen()) == GOLD["petersen"]["independence_polynomial"]["value"]


def test_small_graphs_match_brute_force(ctx):
    for seed in range(10):
        g = gg.random_regular(20, 3, seed)
        assert _poly(ctx, g, seed=seed) == _trim(oracle.brute_force(g)["poly"]), seed
    for g in (gg.path(1), gg.cycle(7), gg.complete(6), gg.empty(9), gg.star(8), gg.complete_bipartite(4, 7)):
        assert _poly(ctx, g) == _trim(oracle.brute_force(g)["poly"]), g.name


@pytest.mark.parametrize("n,seed", [(40, 0), (60, 1), (80, 2)])
def test_medium_graphs_match_polynomial_elimination(ctx, n, seed):
    g = gg.random_regular(n, 3, seed)
    want = oracle.eliminate_polynomial(g, max_width=20)["poly"]
    got = _poly(ctx, g, method="treesa", ntrials=2, niters=5, seed=seed)
    print(f"n={n}: degree {len(got) - 1}, c_max {got[-1]}", flush=True)
    assert got == want


def test_empty_network(ctx):
    assert _poly(ctx, gg.empty(0)) == [1]


def test_k2_network_identities(ctx):
    g = gg.random_regular(120, 3, 0)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=8, niters=20, seed=0)
    p = ctx.solve_polynomial(net, plan)
    count = ctx.solve(net, plan, "count_exact")["count"]
    ct = ctx.solve(net, plan, "counting_tropical")
    print(f"n=120: degree {len(p) - 1}, sum {sum(p)}", flush=True)
    assert sum(p) == count
    assert (len(p) - 1, p[-1] % 2 ** 64) == (ct["size"], ct["count_mod_2_64"])
    assert p[0] == 1 and p[1] == g.nv and p[2] == math.comb(g.nv, 2) - g.ne
    adj = [set() for _ in range(g.nv)]
    for u, v in g.edges:
        adj[u].add(v)
        adj[v].add(u)
    c3 = sum(1 for a, b, c in itertools.combinations(range(g.nv), 3)
             if b not in adj[a] and c not in adj[a] and c not in adj[b])
    assert p[3] == c3


def test_rejected_inputs(ctx):
    g = gg.random_regular(20, 3, 0)
    wnet = tn.Net.from_graph(g.with_weights(gg.integer_weights(g.nv, 1, 1, 3)))
    with pytest.raises(tn.TnError) as ei:
        ctx.solve_polynomial(wnet, tn.Plan.create(wnet))
    assert ei.value.code == tn.TN_EINVAL
    big = gg.random_regular(240, 3, 0)
    net = tn.Net.from_graph(big)
    sliced = tn.Plan.create(net, method="treesa", ntrials=1, niters=2, sc_target=20, nslices=10, seed=0)
    with pytest.raises(tn.TnError) as ei:
        ctx.solve_polynomial(net, sliced)
    assert ei.value.code == tn.TN_EINVAL
    huge = gg.empty(600)
    hnet = tn.Net.from_graph(huge)
    with pytest.raises(tn.TnError) as ei:
        ctx.solve_polynomial(hnet, tn.Plan.create(hnet))
    assert ei.value.code == tn.TN_ETOOBIG


def test_size_max_k_and_counting_max_k(ctx):
    """SizeMax(k) / CountingMax(k) (Sec. 5.3): the paper's Petersen values, then
    the brute-force size histogram of random graphs."""
    net = tn.Net.from_graph(gg.petersen())
    r = ctx.solve_max_k(net, tn.Plan.create(net), 2)
    assert r["size_max_k"] == GOLD["petersen"]["size_max_2"]["value"]
    assert r["counting_max_k"] == {int(s): c for s, c in GOLD["petersen"]["counting_max_2"]["value"].items()}
    for seed in range(4):
        g = gg.random_regular(20, 3, seed)
        hist = _trim(oracle.brute_force(g)["poly"])
        net = tn.Net.from_graph(g)
        for k in (1, 3, 7):
            r = ctx.solve_max_k(net, tn.Plan.create(net, seed=seed), k)
            alpha = len(hist) - 1
            want_sizes = [s for s in range(alpha, -1, -1) for _ in range(hist[s])][:k]
            assert r["size_max_k"] == want_sizes
            assert r["counting_max_k"] == {alpha - d: hist[alpha - d] for d in range(k) if alpha - d >= 0}
