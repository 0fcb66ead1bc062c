"""Pins for the CPU oracle (brute force O1, elimination O2, plan following O3).

Each pin comes from outside the oracle: values the paper prints (golden file,
cited), closed forms from combinatorics, an independent transfer-matrix count,
or agreement between the three independent oracle programs.
"""
import json
import math
import os
import random

import numpy as np
import pytest

import graphgen as gg
import oracle

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
SEMIRINGS = ["tropical", "counting_tropical", "count", "partition"]


def fib(n):
    a, b = 0, 1
    for _ in range(n):
        a, b = b, a + b
    return a


def lucas(n):
    a, b = 2, 1
    for _ in range(n):
        a, b = b, a + b
    return a


# ----------------------------------------------------------- paper pins ---

def test_petersen_paper_values_brute_force():
    g = gg.petersen()
    p = GOLD["petersen"]
    r = oracle.brute_force(g, [0.0], sets_cap=16)
    assert r["size_max"] == p["size_max"]["value"]
    assert [r["size_max"], r["count_max"]] == p["counting_max"]["value"]
    assert r["count_all"] == p["counting_all"]["value"]
    poly = p["independence_polynomial"]["value"]
    assert r["poly"][: len(poly)] == poly and not any(r["poly"][len(poly):])
    # CountingMax(2): the two largest sizes and their counts
    c2 = p["counting_max_2"]["value"]
    assert {str(k): r["poly"][k] for k in (3, 4)} == c2
    # the five maximum sets, character k <-> vertex k-1
    printed = {sum(1 << i for i, ch in enumerate(s) if ch == "1") for s in p["max_sets"]["value"]}
    assert set(r["max_sets"]) == printed


@pytest.mark.parametrize("sr", SEMIRINGS)
def test_petersen_paper_values_elimination(sr):
    g = gg.petersen()
    p = GOLD["petersen"]
    r = oracle.eliminate(g, sr, beta=0.7)
    poly = p["independence_polynomial"]["value"]
    if sr == "tropical":
        assert r["size"] == p["size_max"]["value"]
    elif sr == "counting_tropical":
        assert [r["size"], r["count"]] == p["counting_max"]["value"]
    elif sr == "count":
        assert r["count"] == p["counting_all"]["value"]
    else:
        # unit weights: Z(beta) is the independence polynomial at x = e^beta
        want = sum(c * math.exp(0.7 * k) for k, c in enumerate(poly))
        assert r["z"] == pytest.approx(want, rel=1e-14)


@pytest.mark.slow
def test_square20_partition_function_matches_paper():
    """Z(beta=0) of the 20x20 grid printed in Float64 in Sec. 5.1."""
    want = GOLD["square20"]["partition_beta0"]["value"]
    r = oracle.eliminate(gg.square_lattice(20), "partition", 0.0, max_width=21)
    # the paper's Float64 contraction carries its own rounding; 1e-14 is ~50 ulp
    assert abs(r["z"] - want) / want < 1e-14


def test_square20_stored_values_match_paper():
    """The stored exact count of the 20x20 grid (tests/golden/square20.json,
    written by the oracle's elimination) rounds to the Float64 value printed
    in Sec. 5.1, and its ln Z(0) is the log of that count."""
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "square20.json")))
    want = GOLD["square20"]["partition_beta0"]["value"]
    count = int(gold["count"])
    assert abs(count - want) / want < 1e-15
    assert count.bit_length() == 240  # about 2^239: beyond 7 CRT primes below 2^30
    assert gold["log_z"]["0.0"] == pytest.approx(math.log(count), rel=1e-14)
    # the checkerboards are the two largest sets of an even grid
    assert gold["counting_tropical"] == [200.0, "2"]


def _transfer_matrix_count(L):
    """Independent sets of the L x L grid by rows: a row is a mask with no two
    adjacent ones, consecutive rows must not share a one."""
    rows = [s for s in range(1 << L) if s & (s >> 1) == 0]
    v = {s: 1 for s in rows}
    for _ in range(L - 1):
        v = {t: sum(c for s, c in v.items() if s & t == 0) for t in rows}
    return sum(v.values())


@pytest.mark.parametrize("L", [1, 2, 3, 5, 8, 10])
def test_square_lattice_counts_transfer_matrix(L):
    g = gg.square_lattice(L)
    assert oracle.eliminate(g, "count")["count"] == _transfer_matrix_count(L)


def test_square2_label_invariant_facts():
    # Sec. 3.2 example: the 4-cycle has 7 independent sets, 2 of size 2
    g = gg.cycle(4)
    r = oracle.brute_force(g)
    assert r["count_all"] == GOLD["square2"]["count_all"]["value"]
    assert (r["size_max"], r["count_max"]) == (2.0, 2)


# --------------------------------------------------------- closed forms ---

@pytest.mark.parametrize("n", list(range(1, 21)))
def test_path_fibonacci(n):
    g = gg.path(n)
    r = oracle.brute_force(g)
    assert r["count_all"] == fib(n + 2)
    assert r["size_max"] == (n + 1) // 2
    assert r["count_max"] == (n // 2 + 1 if n % 2 == 0 else 1)
    assert oracle.eliminate(g, "count")["count"] == fib(n + 2)


@pytest.mark.parametrize("n", list(range(3, 21)))
def test_cycle_lucas(n):
    g = gg.cycle(n)
    r = oracle.brute_force(g)
    assert r["count_all"] == lucas(n)
    assert r["size_max"] == n // 2
    assert r["count_max"] == (2 if n % 2 == 0 else n)
    e = oracle.eliminate(g, "counting_tropical")
    assert (e["size"], e["count"]) == (n // 2, 2 if n % 2 == 0 else n)


def test_long_path_exact_count_beyond_int64():
    # F_{302} needs ~208 bits: exercises the 256-bit counts of O2
    g = gg.path(300)
    assert oracle.eliminate(g, "count")["count"] == fib(302)


def test_count_overflow_flagged():
    # F_{402} needs ~278 bits > 256: must be reported, not wrapped silently
    with pytest.raises(oracle.OracleError) as ei:
        oracle.eliminate(gg.path(400), "count")
    assert ei.value.code == oracle.ORC_EOVERFLOW


@pytest.mark.parametrize("n", [1, 2, 5, 9])
def test_complete_graph(n):
    r = oracle.brute_force(gg.complete(n))
    assert (r["count_all"], r["size_max"], r["count_max"]) == (n + 1, 1.0, n)


@pytest.mark.parametrize("n", [0, 1, 7, 16])
def test_empty_graph(n):
    g = gg.empty(n)
    r = oracle.brute_force(g, [0.3])
    assert (r["count_all"], r["size_max"], r["count_max"]) == (2 ** n, float(n), 1)
    assert r["z"][0] == pytest.approx((1 + math.exp(0.3)) ** n, rel=1e-15)
    for sr in SEMIRINGS:
        oracle.eliminate(g, sr)  # nv = 0 and isolated vertices are valid


@pytest.mark.parametrize("a,b", [(1, 1), (2, 3), (4, 4), (3, 7)])
def test_complete_bipartite(a, b):
    r = oracle.brute_force(gg.complete_bipartite(a, b))
    assert r["count_all"] == 2 ** a + 2 ** b - 1
    assert r["size_max"] == max(a, b)
    assert r["count_max"] == (2 if a == b else 1)


def test_weighted_closed_forms():
    beta = 0.9
    w = gg.dyadic_weights(12, seed=3)
    # empty graph: Z = prod (1 + e^{beta w}), max = sum of weights
    g = gg.empty(12).with_weights(w)
    r = oracle.brute_force(g, [beta])
    assert r["z"][0] == pytest.approx(np.prod(1 + np.exp(beta * w.astype(np.float64))), rel=1e-14)
    assert r["size_max"] == pytest.approx(float(np.sum(w.astype(np.float64))), abs=0)
    # complete graph: Z = 1 + sum e^{beta w}, max = max w
    g = gg.complete(12).with_weights(w)
    r = oracle.brute_force(g, [beta])
    assert r["z"][0] == pytest.approx(1 + np.sum(np.exp(beta * w.astype(np.float64))), rel=1e-14)
    assert r["size_max"] == float(w.max())
    # star: centre alone, or any subset of the leaves
    g = gg.star(9).with_weights(w[:10])
    wd = w[:10].astype(np.float64)
    for sr in ("partition",):
        z = oracle.eliminate(g, sr, beta)["z"]
        assert z == pytest.approx(math.exp(beta * wd[0]) + np.prod(1 + np.exp(beta * wd[1:])), rel=1e-14)
    t = oracle.eliminate(g, "tropical")["size"]
    assert t == max(wd[0], wd[1:].sum())


def test_disjoint_union_multiplies_counts_and_adds_sizes():
    g, h = gg.random_regular(10, 3, 1), gg.cycle(7)
    u = gg.disjoint_union(g, h)
    rg, rh, ru = (oracle.brute_force(x, [0.4]) for x in (g, h, u))
    assert ru["count_all"] == rg["count_all"] * rh["count_all"]
    assert ru["size_max"] == rg["size_max"] + rh["size_max"]
    assert ru["count_max"] == rg["count_max"] * rh["count_max"]
    assert ru["z"][0] == pytest.approx(rg["z"][0] * rh["z"][0], rel=1e-14)


def test_tropical_is_zero_temperature_limit_of_log_z():
    # reading of Sec. 5.2: ln Z(beta) - beta * SizeMax -> ln(count at max)
    g = gg.random_regular(16, 3, 4).with_weights(gg.integer_weights(16, 4))
    r = oracle.brute_force(g, [40.0])
    assert r["log_z"][0] - 40.0 * r["size_max"] == pytest.approx(math.log(r["count_max"]), abs=1e-9)


def test_partition_at_beta_zero_is_count():
    g = gg.random_regular(18, 3, 9)
    r = oracle.brute_force(g, [0.0])
    assert r["z"][0] == r["count_all"]
    assert oracle.eliminate(g, "partition", 0.0)["z"] == r["count_all"]


# --------------------------------------------------- O2 against O1 -------

def _random_graphs(count):
    out = []
    for s in range(count):
        kind = s % 4
        if kind == 0:
            g = gg.random_regular(2 * (4 + s % 6), 3, s)
        elif kind == 1:
            g = gg.gnp(8 + s % 9, 0.15 + 0.05 * (s % 5), s)
        elif kind == 2:
            g = gg.kings_subgraph(4, 0.8, s)
        else:
            g = gg.gnp(6 + s % 10, 0.4, s)
        if s % 3 == 1:
            g = g.with_weights(gg.dyadic_weights(g.nv, s))
        elif s % 3 == 2:
            g = g.with_weights(gg.integer_weights(g.nv, s, 1, 3))
        out.append(g)
    return out


def test_elimination_matches_brute_force_on_200_graphs():
    beta = 1.3
    for g in _random_graphs(200):
        bf = oracle.brute_force(g, [beta])
        t = oracle.eliminate(g, "tropical")
        ct = oracle.eliminate(g, "counting_tropical")
        c = oracle.eliminate(g, "count")
        z = oracle.eliminate(g, "partition", beta)
        assert t["size"] == bf["size_max"], g.name
        assert (ct["size"], ct["count"]) == (bf["size_max"], bf["count_max"]), g.name
        assert c["count"] == bf["count_all"], g.name
        assert z["z"] == pytest.approx(bf["z"][0], rel=1e-13), g.name


# --------------------------------------------------- O3 plan following ---

def leaves_of(g, absorb):
    """Leaf factor lists: one per edge, one per vertex (or vertex tensors
    folded into the first incident edge when absorb is set)."""
    leaves = [[e] for e in range(g.ne)]
    first = {}
    for e, (u, v) in enumerate(g.edges.tolist()):
        first.setdefault(u, e)
        first.setdefault(v, e)
    for v in range(g.nv):
        if absorb and v in first:
            leaves[first[v]].append(-v - 1)
        else:
            leaves.append([-v - 1])
    return leaves


def random_tree(g, seed, absorb=False, nsliced=0):
    """A random binary contraction tree in the oracle's plan format."""
    rng = random.Random(seed)
    leaves = leaves_of(g, absorb)
    edges = g.edges.tolist()

    def scope(fs):
        s = set()
        for f in fs:
            s.update(edges[f] if f >= 0 else [-f - 1])
        return s

    counts = [dict.fromkeys(scope(fs), 1) for fs in leaves]
    total = {}
    for c in counts:
        for k in c:
            total[k] = total.get(k, 0) + 1

    def open_of(c):
        return sorted(k for k, n in c.items() if n < total[k])

    indices = [open_of(c) for c in counts]
    live = list(range(len(leaves)))
    left, right = [], []
    while len(live) > 1:
        a, b = rng.sample(live, 2)
        live.remove(a)
        live.remove(b)
        c = dict(counts[a])
        for k, n in counts[b].items():
            c[k] = c.get(k, 0) + n
        counts.append(c)
        indices.append(open_of(c))
        left.append(a)
        right.append(b)
        live.append(len(counts) - 1)
    sliced = rng.sample(range(g.nv), nsliced) if nsliced else []
    return {"leaf_factors": leaves, "left": left, "right": right, "indices": indices, "sliced": sliced}


@pytest.mark.parametrize("seed", range(12))
def test_follow_plan_random_trees_match_brute_force(seed):
    g = [gg.random_regular(12, 3, seed), gg.kings_subgraph(3, 0.9, seed), gg.gnp(11, 0.3, seed)][seed % 3]
    if seed % 2:
        g = g.with_weights(gg.dyadic_weights(g.nv, seed))
    tree = random_tree(g, seed, absorb=bool(seed % 4 >= 2), nsliced=seed % 3)
    bf = oracle.brute_force(g, [0.8])
    assert oracle.follow_plan(g, tree, "tropical")["size"] == bf["size_max"]
    ct = oracle.follow_plan(g, tree, "counting_tropical")
    assert (ct["size"], ct["count"]) == (bf["size_max"], bf["count_max"])
    assert oracle.follow_plan(g, tree, "count")["count"] == bf["count_all"]
    assert oracle.follow_plan(g, tree, "partition", 0.8)["z"] == pytest.approx(bf["z"][0], rel=1e-13)


def _paper_square_tree():
    """The TreeSA tree printed in Sec. 4.1, in the oracle's plan format."""
    t = GOLD["square2"]["tree"]
    code = t["eincode"]
    # graph vertices 1..4 -> 0..3; edges in the EinCode's order
    edges = [tuple(sorted((a - 1, b - 1))) for a, b in code[:4]]
    g = gg.Graph(4, np.array(edges, np.int32), None, "square2")
    leaf_names = ["L:" + "∘".join(map(str, c)) for c in code]
    leaf_factors = [[e] for e in range(4)] + [[-v - 1] for v in range(4)]
    nodes = {n.get("id", "root"): n for n in t["nodes"]}
    ids = {name: i for i, name in enumerate(leaf_names)}
    order = ["N6", "N5", "N4", "N3", "N2", "N1", "root"]
    for k, name in enumerate(order):
        ids[name] = len(leaf_names) + k
    left, right, inner_out = [], [], []
    for name in order:
        a, b = nodes[name]["children"]
        left.append(ids[a])
        right.append(ids[b])
        inner_out.append(sorted(x - 1 for x in nodes[name]["out"]))
    leaf_out = [sorted(x - 1 for x in c) for c in code]
    tree = {"leaf_factors": leaf_factors, "left": left, "right": right,
            "indices": leaf_out + inner_out, "sliced": []}
    return g, tree


def test_follow_plan_on_the_papers_printed_tree():
    g, tree = _paper_square_tree()
    assert oracle.follow_plan(g, tree, "count")["count"] == 7
    ct = oracle.follow_plan(g, tree, "counting_tropical")
    assert (ct["size"], ct["count"]) == (2.0, 2)


def test_follow_plan_rejects_a_wrong_output_list():
    # plant a mistake in the plan: keep an index open after its last use
    g = gg.cycle(5)
    tree = random_tree(g, 1)
    bad = dict(tree)
    bad["indices"] = [list(x) for x in tree["indices"]]
    bad["indices"][-2] = sorted(set(bad["indices"][-2]) | {0, 1, 2, 3, 4})
    with pytest.raises(oracle.OracleError):
        oracle.follow_plan(g, bad, "count")
    bad2 = dict(tree)
    bad2["leaf_factors"] = tree["leaf_factors"][:-1] + [tree["leaf_factors"][0]]
    with pytest.raises(oracle.OracleError):
        oracle.follow_plan(g, bad2, "count")


def test_follow_plan_slicing_every_subset_agrees():
    g = gg.random_regular(10, 3, 5).with_weights(gg.dyadic_weights(10, 5))
    base = random_tree(g, 3)
    ref = oracle.follow_plan(g, base, "counting_tropical")
    for k in range(1, 5):
        t = dict(base)
        t["sliced"] = list(range(k))
        r = oracle.follow_plan(g, t, "counting_tropical")
        assert r == ref


def _oplus(sr, a, b):
    """The algebra's (+) of two O3 results (max-plus, counting tropical, counts, Z)."""
    if sr == "tropical":
        return {"size": max(a["size"], b["size"])}
    if sr == "counting_tropical":
        if a["size"] != b["size"]:
            return a if a["size"] > b["size"] else b
        return {"size": a["size"], "count": a["count"] + b["count"]}
    if sr == "count":
        return {"count": a["count"] + b["count"]}
    return {"z": a["z"] + b["z"]}


@pytest.mark.parametrize("seed", range(6))
def test_follow_plan_slice_ranges(seed):
    """O3's slice-range path (slice s fixes sliced[k] to bit k of s, Sec. 4.2
    slicing): every single slice equals the brute force conditioned on those
    fixed values, and the (+) of the results over any partition of the slice
    range into contiguous ranges equals the whole contraction."""
    g = [gg.random_regular(12, 3, seed), gg.kings_subgraph(3, 0.9, seed), gg.gnp(11, 0.35, seed)][seed % 3]
    if seed % 2:
        g = g.with_weights(gg.dyadic_weights(g.nv, seed))
    ns = 3 + seed % 2
    tree = random_tree(g, 100 + seed, absorb=bool(seed % 4 >= 2), nsliced=ns)
    sl = tree["sliced"]
    beta = 0.6
    whole = {sr: oracle.follow_plan(g, tree, sr, beta) for sr in SEMIRINGS}
    bf = oracle.brute_force(g, [beta])
    assert whole["count"]["count"] == bf["count_all"]
    for s in range(1 << ns):
        fixed = {sl[k]: (s >> k) & 1 for k in range(ns)}
        ref = oracle.brute_force(g, [beta], fixed=fixed)
        one = {sr: oracle.follow_plan(g, tree, sr, beta, slices=(s, s + 1)) for sr in SEMIRINGS}
        assert one["count"]["count"] == ref["count_all"], (s, fixed)
        if ref["count_all"] == 0:
            assert one["tropical"]["size"] == float("-inf")
            assert one["counting_tropical"] == {"size": float("-inf"), "count": 0}
            assert one["partition"]["z"] == 0.0
            continue
        assert one["tropical"]["size"] == ref["size_max"]
        assert (one["counting_tropical"]["size"], one["counting_tropical"]["count"]) == (ref["size_max"],
                                                                                       ref["count_max"])
        assert one["partition"]["z"] == pytest.approx(ref["z"][0], rel=1e-13)
    rng = random.Random(seed)
    for _ in range(3):
        cuts = sorted(rng.sample(range(1, 1 << ns), rng.randint(1, (1 << ns) - 1)))
        bounds = [0] + cuts + [1 << ns]
        for sr in SEMIRINGS:
            acc = None
            for a, b in zip(bounds[:-1], bounds[1:]):
                r = oracle.follow_plan(g, tree, sr, beta, slices=(a, b))
                acc = r if acc is None else _oplus(sr, acc, r)
            if sr == "partition":
                assert acc["z"] == pytest.approx(whole[sr]["z"], rel=1e-13)
            else:
                assert {k: acc[k] for k in whole[sr]} == {k: whole[sr][k] for k in whole[sr]}, (sr, bounds)


# ---------------------------------------------------- independence polynomial
# O2 over polynomial-valued tables (Sec. 5.3 GraphPolynomial; Sec. 6.2).

def test_polynomial_petersen_matches_paper():
    want = GOLD["petersen"]["independence_polynomial"]["value"]
    r = oracle.eliminate_polynomial(gg.petersen())
    assert r["poly"] == want and r["degree"] == len(want) - 1


@pytest.mark.parametrize("n", [1, 2, 3, 7, 12, 30, 60])
def test_polynomial_path_and_cycle_closed_forms(n):
    # paths: c_k = C(n - k + 1, k); cycles (n >= 3): c_k = n / (n - k) * C(n - k, k)
    p = oracle.eliminate_polynomial(gg.path(n))["poly"]
    assert p == [math.comb(n - k + 1, k) for k in range((n + 1) // 2 + 1)]
    if n >= 3:
        c = oracle.eliminate_polynomial(gg.cycle(n))["poly"]
        assert c == [1] + [n * math.comb(n - k, k) // (n - k) for k in range(1, n // 2 + 1)]


@pytest.mark.parametrize("a,b", [(1, 1), (2, 5), (6, 6), (3, 9)])
def test_polynomial_complete_bipartite_star_complete_empty(a, b):
    # K_{a,b}: (1+x)^a + (1+x)^b - 1 (independent sets lie on one side)
    want = [math.comb(a, k) + math.comb(b, k) - (k == 0) for k in range(max(a, b) + 1)]
    assert oracle.eliminate_polynomial(gg.complete_bipartite(a, b))["poly"] == want
    assert oracle.eliminate_polynomial(gg.complete(a + b))["poly"] == [1, a + b]
    assert oracle.eliminate_polynomial(gg.empty(b))["poly"] == [math.comb(b, k) for k in range(b + 1)]


def test_polynomial_matches_brute_force_histogram():
    rng = random.Random(11)
    for t in range(80):
        n = rng.randint(1, 16)
        g = gg.gnp(n, rng.uniform(0.05, 0.7), t) if t % 2 else gg.random_regular(n - n % 2 or 2, 3 if n > 4 else 1, t)
        bf = oracle.brute_force(g)["poly"]
        while len(bf) > 1 and bf[-1] == 0:
            bf.pop()
        assert oracle.eliminate_polynomial(g)["poly"] == bf, (t, g.nv)


def test_polynomial_multiplies_over_disjoint_union_and_agrees_with_other_algebras():
    g1, g2 = gg.random_regular(14, 3, 1), gg.cycle(9)
    p1 = oracle.eliminate_polynomial(g1)["poly"]
    p2 = oracle.eliminate_polynomial(g2)["poly"]
    prod = [sum(p1[i] * p2[k - i] for i in range(len(p1)) if 0 <= k - i < len(p2)) for k in range(len(p1) + len(p2) - 1)]
    assert oracle.eliminate_polynomial(gg.disjoint_union(g1, g2))["poly"] == prod
    for seed in range(3):  # larger graphs: sum = total count, top coefficient = count at the maximum size
        g = gg.random_regular(50, 3, seed)
        p = oracle.eliminate_polynomial(g)["poly"]
        ct = oracle.eliminate(g, "counting_tropical")
        assert sum(p) == oracle.eliminate(g, "count")["count"]
        assert (len(p) - 1, p[-1]) == (ct["size"], ct["count"])
        assert p[1] == g.nv and p[2] == math.comb(g.nv, 2) - g.ne


# ---------------------------------------------------------------- spin glass
# H(s) = sum_(u,v) J_uv s_u s_v + sum_v h_v s_v, s = +-1 (Sec. 2); the
# tropical algebras maximise -H (Sec. 6.4 CountingMin).

def test_spin_glass_fullerene_matches_paper():
    g = gg.fullerene()
    fp = GOLD["fullerene"]
    assert [g.nv, g.ne] == fp["size"]["value"]
    lz = oracle.spin_glass_eliminate(g, "partition", beta=1.0)["log_z"]
    assert abs(lz / g.nv - fp["log_z_per_vertex_beta1"]["value"]) <= 1e-14
    ct = oracle.spin_glass_eliminate(g, "counting_tropical")
    assert [-ct["size"], ct["count"]] == fp["counting_min"]["value"]


def test_spin_glass_petersen_printed_energy_and_brute_force():
    g = gg.petersen()
    spins = GOLD["petersen"]["spin_glass_energy"]["value"]["spins"]
    # the energy of one configuration: a field-free spin glass on the graph
    # with each vertex's spin pinned by a huge field, minus the pinning
    big = 1000.0
    h = [-big * s for s in spins]
    bf = oracle.spin_glass_brute_force(g, h=h)
    assert bf["count_min"] == 1
    assert bf["energy_min"] + big * len(spins) == GOLD["petersen"]["spin_glass_energy"]["value"]["energy"]


@pytest.mark.parametrize("n", [2, 5, 8, 13])
def test_ising_chain_and_ring_closed_forms(n):
    for beta in (0.3, 1.0):
        c, s = 2 * math.cosh(beta), 2 * math.sinh(beta)
        zp = oracle.spin_glass_eliminate(gg.path(n), "partition", beta=beta)["z"]
        assert abs(zp - 2 * c ** (n - 1)) <= 1e-12 * zp
        if n >= 3:
            zr = oracle.spin_glass_eliminate(gg.cycle(n), "partition", beta=beta)["z"]
            # transfer matrix [[e^-b, e^b], [e^b, e^-b]]: eigenvalues 2 cosh b, -2 sinh b
            assert abs(zr - (c ** n + (-s) ** n)) <= 1e-12 * zr
    if n >= 3:  # antiferromagnetic ring: frustrated when n is odd
        ct = oracle.spin_glass_eliminate(gg.cycle(n), "counting_tropical")
        assert (-ct["size"], ct["count"]) == ((-(n - 2), 2 * n) if n % 2 else (-n, 2))
    fm = oracle.spin_glass_eliminate(gg.path(n), "counting_tropical", J=[-1.0] * (n - 1))  # ferromagnet
    assert (-fm["size"], fm["count"]) == (-(n - 1), 2)


def test_spin_glass_fields_only_and_counts():
    g = gg.empty(7)
    h = [0.5, -1.0, 0.0, 2.0, 0.0, -0.25, 1.5]
    z = oracle.spin_glass_eliminate(g, "partition", h=h, beta=0.7)["z"]
    assert abs(z - math.prod(2 * math.cosh(0.7 * x) for x in h)) <= 1e-12 * z
    ct = oracle.spin_glass_eliminate(g, "counting_tropical", h=h)
    assert (ct["size"], ct["count"]) == (sum(abs(x) for x in h), 4)
    g2 = gg.random_regular(30, 3, 2)
    assert oracle.spin_glass_eliminate(g2, "count")["count"] == 2 ** 30
    assert abs(oracle.spin_glass_eliminate(g2, "partition", beta=0.0)["z"] - 2.0 ** 30) <= 1e-6


def test_spin_glass_elimination_matches_brute_force():
    rng = random.Random(5)
    for t in range(60):
        n = rng.randint(1, 14)
        g = gg.gnp(n, rng.uniform(0.1, 0.8), 100 + t)
        J = [float(rng.randint(-2, 2)) for _ in range(g.ne)]
        h = [float(rng.randint(-1, 1)) for _ in range(n)] if t % 2 else None
        bf = oracle.spin_glass_brute_force(g, J, h, betas=[0.4])
        ct = oracle.spin_glass_eliminate(g, "counting_tropical", J=J, h=h)
        assert (-ct["size"], ct["count"]) == (bf["energy_min"], bf["count_min"]), t
        z = oracle.spin_glass_eliminate(g, "partition", J=J, h=h, beta=0.4)["z"]
        assert abs(z - bf["z"][0]) <= 1e-12 * bf["z"][0], t
        assert oracle.spin_glass_eliminate(g, "tropical", J=J, h=h)["size"] == -bf["energy_min"]


# ----------------------------------------------------- fixed vertices ----
# Conditioning on n_v (the fixed vertices of the Sec. 5 network object) is
# pinned by graph identities the oracle computes on other graphs: n_v = 0
# is the graph without v; n_v = 1 is the graph without v's closed
# neighbourhood, plus v's weight (Z times e^(beta w_v), the polynomial times
# x); the two conditionings add up to the unconditioned result.

def _without(g, drop):
    return gg.induced(g, [v for v in range(g.nv) if v not in set(drop)])


def test_fixed_vertex_identities_brute_force():
    rng = random.Random(17)
    for t in range(30):
        n = rng.randint(2, 14)
        g = gg.gnp(n, rng.uniform(0.1, 0.6), 900 + t)
        if t % 2:
            g = g.with_weights(gg.integer_weights(n, 900 + t, 1, 5))
        w = g.weights if g.weights is not None else np.ones(n, np.float32)
        v = rng.randrange(n)
        beta = 0.3
        full = oracle.brute_force(g, betas=[beta])
        f0 = oracle.brute_force(g, betas=[beta], fixed={v: 0}, sets_cap=50)
        f1 = oracle.brute_force(g, betas=[beta], fixed={v: 1}, sets_cap=50)
        g0 = oracle.brute_force(_without(g, [v]), betas=[beta])
        nb = [u for u in g.adjacency()[v]]
        g1 = oracle.brute_force(_without(g, [v] + nb), betas=[beta])
        assert (f0["size_max"], f0["count_all"], f0["count_max"]) == (g0["size_max"], g0["count_all"], g0["count_max"])
        assert f0["poly"][: n] == g0["poly"] + [0] * (n - len(g0["poly"]))
        assert f1["size_max"] == g1["size_max"] + float(w[v]) and f1["count_all"] == g1["count_all"]
        assert f1["poly"] == [0] + g1["poly"] + [0] * (n - len(g1["poly"]))
        assert math.isclose(f1["z"][0], g1["z"][0] * math.exp(beta * float(w[v])), rel_tol=1e-12)
        assert f0["count_all"] + f1["count_all"] == full["count_all"]
        assert [a + b for a, b in zip(f0["poly"], f1["poly"])] == full["poly"]
        assert math.isclose(f0["z"][0] + f1["z"][0], full["z"][0], rel_tol=1e-12)
        for S in f0["max_sets"]:
            assert not (S >> v) & 1
        for S in f1["max_sets"]:
            assert (S >> v) & 1
    # conflicting fixings leave nothing: an edge with both ends fixed to 1
    g = gg.path(3)
    r = oracle.brute_force(g, fixed={0: 1, 1: 1})
    assert r["count_all"] == 0 and r["size_max"] == float("-inf")


def test_fixed_spin_identities_brute_force():
    rng = random.Random(19)
    for t in range(12):
        n = rng.randint(2, 12)
        g = gg.gnp(n, rng.uniform(0.2, 0.7), 950 + t)
        J = [float(rng.randint(-3, 3)) for _ in range(g.ne)]
        v = rng.randrange(n)
        full = oracle.spin_glass_brute_force(g, J, betas=[0.4])
        up = oracle.spin_glass_brute_force(g, J, betas=[0.4], fixed={v: 1})
        dn = oracle.spin_glass_brute_force(g, J, betas=[0.4], fixed={v: 0})
        # without fields H is even under flipping every spin
        assert (up["energy_min"], up["count_min"]) == (dn["energy_min"], dn["count_min"])
        assert up["count_min"] + dn["count_min"] == full["count_min"] and up["energy_min"] == full["energy_min"]
        assert math.isclose(up["z"][0], full["z"][0] / 2, rel_tol=1e-12)
        # a field on v alone: fixing s_v = +1 adds h_v to every energy
        h = [0.0] * n
        h[v] = 2.0
        upf = oracle.spin_glass_brute_force(g, J, h, betas=[0.4], fixed={v: 1})
        assert upf["energy_min"] == up["energy_min"] + 2.0
        assert math.isclose(upf["z"][0], up["z"][0] * math.exp(-0.8), rel_tol=1e-12)


# ----------------------------------------------------------- SizeMax(k) ----

def test_topk_unit_weights_is_the_size_histogram_expanded():
    for t in range(20):
        g = gg.gnp(10 + t % 6, 0.3, 1000 + t)
        hist = oracle.brute_force(g)["poly"]
        expanded = [float(s) for s in range(len(hist) - 1, -1, -1) for _ in range(hist[s])]
        for k in (1, 3, 8):
            want = (expanded + [float("-inf")] * k)[:k]
            assert oracle.brute_force_topk(g, k) == want


def test_topk_petersen_matches_paper():
    assert oracle.brute_force_topk(gg.petersen(), 2) == [float(x) for x in GOLD["petersen"]["size_max_2"]["value"]]


def test_topk_weighted_empty_graph_is_the_largest_subset_sums():
    import itertools
    for t in range(6):
        n = 4 + t
        w = gg.integer_weights(n, 1100 + t, 1, 9)
        g = gg.empty(n).with_weights(w)
        sums = sorted((sum(float(w[i]) for i in c) for r in range(n + 1) for c in itertools.combinations(range(n), r)),
                      reverse=True)
        assert oracle.brute_force_topk(g, 8) == (sums + [float("-inf")] * 8)[:8]


def test_topk_antiferromagnetic_ring():
    """-H of the even ring with J = 1: two ground states at n, then the
    states with two domain walls at n - 4."""
    for n in (6, 8, 10):
        assert oracle.spin_glass_topk(gg.cycle(n), 3) == [float(n), float(n), float(n - 4)]


# --- CountingMax(k) by enumeration: counts at the k highest integer values ---

def test_count_top_petersen_matches_paper():
    want = {int(s): c for s, c in GOLD["petersen"]["counting_max_2"]["value"].items()}
    assert oracle.brute_force_counting_max_k(gg.petersen(), 2) == {"top": 4, "counts": want}


def test_count_top_unit_weights_is_the_eliminated_polynomial():
    """Unit weights: the top coefficients of the independence polynomial,
    which the oracle's elimination over polynomial tables computes
    independently of the enumeration."""
    for t in range(20):
        g = gg.gnp(8 + t % 10, 0.3, 1200 + t)
        poly = oracle.eliminate_polynomial(g)["poly"]
        alpha = len(poly) - 1
        for k in (1, 2, 4, 6):
            want = {alpha - d: (poly[alpha - d] if alpha - d >= 0 else 0) for d in range(k)}
            assert oracle.brute_force_counting_max_k(g, k) == {"top": alpha, "counts": want}


def test_count_top_weighted_graphs_by_plain_enumeration():
    """Integer weights on small graphs: every subset listed with itertools,
    independence checked edge by edge."""
    import itertools
    for t in range(12):
        n = 3 + t % 8
        g = gg.gnp(n, 0.35, 1300 + t).with_weights(gg.integer_weights(n, 1300 + t, 1, 6))
        edges = [tuple(e) for e in g.edges.tolist()]
        vals = [sum(int(g.weights[v]) for v in c) for r in range(n + 1) for c in itertools.combinations(range(n), r)
                if not any(u in c and v in c for u, v in edges)]
        top = max(vals)
        want = {top - d: vals.count(top - d) for d in range(4)}
        assert oracle.brute_force_counting_max_k(g, 4) == {"top": top, "counts": want}


def test_count_top_fixed_vertices_are_deletions():
    """n_v = 0 counts the sets of G - v; n_v = 1 those of G - N[v], each
    shifted by w_v."""
    for t in range(10):
        n = 6 + t % 8
        g = gg.gnp(n, 0.3, 1400 + t).with_weights(gg.integer_weights(n, 1400 + t, 1, 5))
        v = t % n
        adj = g.adjacency()
        out = oracle.brute_force_counting_max_k(g, 3, fixed={v: 0})
        assert out == oracle.brute_force_counting_max_k(gg.induced(g, [u for u in range(n) if u != v]), 3)
        rest = gg.induced(g, [u for u in range(n) if u != v and u not in adj[v]])
        sub = oracle.brute_force_counting_max_k(rest, 3)
        wv = int(g.weights[v])
        got = oracle.brute_force_counting_max_k(g, 3, fixed={v: 1})
        assert got == {"top": sub["top"] + wv, "counts": {s + wv: c for s, c in sub["counts"].items()}}


def test_count_top_spin_glass_closed_forms():
    """Fields only: -H = -sum h_v s_v, whose value counts are the
    coefficients of prod_v (x^h_v + x^-h_v); the ferromagnetic ring (J = -1)
    has its two ground states at -H = n and nothing until n - 4."""
    rng = np.random.default_rng(5)
    for t in range(6):
        n = 5 + t
        h = [float(x) for x in rng.integers(-3, 4, n)]
        coeff = {0: 1}
        for hv in h:
            nxt = {}
            for e, c in coeff.items():
                for s in (hv, -hv):
                    nxt[e + int(s)] = nxt.get(e + int(s), 0) + c
            coeff = nxt
        top = max(coeff)
        want = {top - d: coeff.get(top - d, 0) for d in range(4)}
        assert oracle.spin_glass_counting_max_k(gg.empty(n), 4, h=h) == {"top": top, "counts": want}
    for n in (6, 8):
        got = oracle.spin_glass_counting_max_k(gg.cycle(n), 4, J=[-1.0] * n)
        assert got == {"top": n, "counts": {n: 2, n - 1: 0, n - 2: 0, n - 3: 0}}
        got = oracle.spin_glass_counting_max_k(gg.cycle(n), 1, J=[-1.0] * n, fixed={0: 1, 3: 0})
        assert got["top"] == n - 4  # two domain walls forced


def test_count_top_rejects_fractional_weights_and_reports_infeasible():
    g = gg.path(3).with_weights(np.array([1.0, 0.5, 2.0]))
    with pytest.raises(oracle.OracleError):
        oracle.brute_force_counting_max_k(g, 2)
    assert oracle.brute_force_counting_max_k(gg.path(2), 2, fixed={0: 1, 1: 1}) == {"top": float("-inf"), "counts": {}}


def test_served_stream_stored_values_reproduce():
    """tests/golden/k4_jobs.json: the stream it names, every job with n <= 130
    present, the sample drawn only from the larger ones, and a few stored
    values recomputed by the oracle (a check of the file, not a pin of the
    oracle)."""
    rec = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "k4_jobs.json")))
    mix = gg.job_mix(rec["njobs"], rec["seed"], *rec["n_range"])
    small = {k for k, j in enumerate(mix) if j[0] <= rec["check_n"]}
    large = [k for k, j in enumerate(mix) if j[0] > rec["check_n"]]
    sample = set(rec["sample"]["jobs"])
    assert sample <= set(large) and len(sample) == round(rec["sample"]["fraction"] * len(large))
    assert {int(k) for k in rec["expected"]} == small | sample
    checked = 0
    for k in sorted(small, key=lambda k: mix[k][0])[:6]:
        n, gseed, sr = mix[k]
        g = gg.random_regular(n, 3, gseed)
        want = rec["expected"][str(k)]
        if sr == "tropical_i32":
            assert oracle.eliminate(g, "tropical")["size"] == want
        elif sr == "counting_tropical":
            r = oracle.eliminate(g, "counting_tropical")
            assert [r["size"], str(r["count"] % 2 ** 64)] == want
        else:
            assert abs(oracle.eliminate(g, "partition", 0.0)["log_z"] - want) <= 1e-12 * abs(want)
        checked += 1
    assert checked == 6
