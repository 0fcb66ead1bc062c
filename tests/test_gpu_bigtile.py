"""GPU parity of the 128 x 128 register-tiled VALU GEMM.

The per-node executor sends nodes of the 4-byte VALU algebras (max-plus
int32 and float32, counts mod p) with M, N >= 2^7 and K >= 2^4 to a 128 x 128
tile (halved to 128 x 64 or 64 x 128 when that gives at most 32 output
tiles), and nodes with one side >= 2^8 and the other 2^5 or 2^6 to the
256 x 32, 256 x 64 tiles (or their mirror images); counting-tropical nodes go
to 128 x 64, 64 x 128, 256 x 32 and 32 x 256 tiles.  Square lattices of side
14 and 16, a King's subgraph of side 15, a finely sliced plan of the
240-vertex 3-regular network and a hand-made tree whose middle node is a
1024 x 1024 x 16 product have such nodes (with and without batch indices,
with split K); each case asserts which tiles ran and compares the result with
the oracle.
"""
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


def _solve_profiled(ctx, net, plan, sr, **kw):
    ctx.set_profiling(True)
    try:
        r = ctx.solve(net, plan, sr, executor="stream", **kw)
        recs = ctx.profile()
    finally:
        ctx.set_profiling(False)
    return r, recs


def _plan(net, method, seed=0):
    if method == "greedy":
        return tn.Plan.create(net, seed=seed)
    return tn.Plan.create(net, method="treesa", ntrials=2, niters=5, seed=seed)


def _nbig(recs):
    return sum(1 for x in recs if x["kind"] == "gemm_big")


def _tile(shape):
    """(log2 TM, log2 TN) of the register-tiled kernel for a GEMM shape (b, i, j, k)."""
    b, i, j, k = shape
    if i >= 7 and j >= 7 and k >= 4:
        if b + (i - 7) + (j - 7) <= 5:  # at most 32 square tiles: half tiles
            return (7, 6) if j >= i else (6, 7)
        return (7, 7)
    if i >= 8 and j in (5, 6):
        return (8, j)
    if j >= 8 and i in (5, 6):
        return (i, 8)
    return None


def _ct_tile(shape):
    """(log2 TM, log2 TN) of the counting-tropical register-tiled kernel."""
    _, i, j, k = shape
    if k < 2:
        return None
    if i >= 7 and j >= 6:
        return (7, 6)
    if i >= 6 and j >= 7:
        return (6, 7)
    if i >= 8 and j == 5:
        return (8, 5)
    if j >= 8 and i == 5:
        return (5, 8)
    return None


# (graph, planner, planner seed, 4-byte tiles, counting-tropical tiles the plan must exercise)
CASES = [
    ("lattice14", "greedy", 0, {(7, 6), (8, 6), (8, 5), (6, 8)}, {(7, 6), (8, 5)}),
    ("lattice14", "treesa", 0, {(6, 7), (8, 6)}, {(7, 6)}),
    ("lattice16", "greedy", 0, {(6, 7), (7, 6), (6, 8)}, {(7, 6), (6, 7)}),
    ("ksg15", "treesa", 2, {(7, 6), (8, 6), (8, 5), (5, 8)}, {(7, 6), (6, 7), (8, 5), (5, 8)}),
]


def _graph(name):
    if name.startswith("lattice"):
        return gg.square_lattice(int(name[7:]))
    return gg.kings_subgraph(15, 0.8, 1)


@pytest.mark.parametrize("name,method,seed,tiles,ct_tiles", CASES)
def test_big_tiles_vs_oracle(ctx, name, method, seed, tiles, ct_tiles):
    gu = _graph(name)
    gw = gu.with_weights(gg.dyadic_weights(gu.nv, 7))
    net_u, net_w = tn.Net.from_graph(gu), tn.Net.from_graph(gw)
    plan_u, plan_w = _plan(net_u, method, seed), _plan(net_w, method, seed)
    print(f"{name} {method} complexity {plan_u.complexity()}", flush=True)
    cases = [("tropical_f32", net_w, plan_w, "size", oracle.eliminate(gw, "tropical")["size"]),
             ("tropical_i32", net_u, plan_u, "size", oracle.eliminate(gu, "tropical")["size"]),
             ("count_exact", net_u, plan_u, "count", oracle.eliminate(gu, "count")["count"])]
    for sr, net, plan, key, want in cases:
        r, recs = _solve_profiled(ctx, net, plan, sr)
        ran = {_tile(x["shape"]) for x in recs if x["kind"] == "gemm_big"}
        print(f"  {sr}: {r[key]} vs {want}, big-tile launches {_nbig(recs)}, tiles {sorted(ran)}", flush=True)
        assert tiles <= ran  # count_exact: the residue lanes mod p
        # dyadic weights: every partial sum is exact in float32
        assert r[key] == want
    want = oracle.eliminate(gu, "counting_tropical")
    r, recs = _solve_profiled(ctx, net_u, plan_u, "counting_tropical")
    ran = {_ct_tile(x["shape"]) for x in recs if x["kind"] == "gemm_big"}
    print(f"  counting_tropical: {r['size']}, {r['count_mod_2_64']} vs {want}, tiles {sorted(ran, key=str)}", flush=True)
    assert ct_tiles <= ran
    assert (r["size"], r["count_mod_2_64"]) == (want["size"], want["count"] % 2 ** 64)


def test_k5_slice_big_tiles_vs_plan_follower(ctx):
    g = gg.random_regular(240, 3, 0)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=4, niters=5, sc_target=18, nslices=40, seed=0)
    info = plan.info()
    print("k5 sc 18", plan.complexity(), info, flush=True)
    tree = plan.export()
    s = int(np.random.default_rng(1).integers(1, 2 ** info["nsliced"]))
    want = oracle.follow_plan(g, tree, "count", slices=(s, s + 1))["count"]
    r, recs = _solve_profiled(ctx, net, plan, "count_exact", slices=(s, s + 1))
    print(f"  slice {s}: oracle {want} gpu {r['count']}, big {_nbig(recs)}", flush=True)
    assert _nbig(recs) > 0
    assert r["count"] == want
    # the max-plus lanes on the same slice agree with each other and with the
    # counting-tropical size (which runs on the 4 x 4 kernel)
    kinds = {x["kind"] for x in recs}
    print("  kernel kinds", sorted(kinds), flush=True)
    assert {"gemm_thin", "gemm_dot"} <= kinds  # sliced plans have thin nodes (N * K <= 32, M >= 2^10)
    a, recs = _solve_profiled(ctx, net, plan, "tropical_i32", slices=(s, s + 1))
    assert _nbig(recs) > 0
    b = ctx.solve(net, plan, "tropical_f32", slices=(s, s + 1), executor="stream")
    z = oracle.follow_plan(g, tree, "partition", beta=0.25, slices=(s, s + 1))["log_z"]
    assert abs(ctx.solve(net, plan, "partition_f32", beta=0.25, slices=(s, s + 1), executor="stream")["log_z"] - z) <= 1e-5
    c = ctx.solve(net, plan, "counting_tropical", slices=(s, s + 1), executor="stream")
    assert a["size"] == b["size"] == c["size"]


@pytest.mark.parametrize("name,method,seed", [("lattice14", "greedy", 0), ("ksg15", "treesa", 2)])
def test_persistent_big_tiles_vs_oracle(ctx, name, method, seed):
    """The persistent kernel runs the same tile shapes (they depend on the
    node only), so the networks above cover its register-tiled paths too."""
    gu = _graph(name)
    gw = gu.with_weights(gg.dyadic_weights(gu.nv, 7))
    net_u, net_w = tn.Net.from_graph(gu), tn.Net.from_graph(gw)
    plan_u, plan_w = _plan(net_u, method, seed), _plan(net_w, method, seed)
    ct = oracle.eliminate(gu, "counting_tropical")
    r = ctx.solve(net_u, plan_u, "counting_tropical", executor="persistent")
    assert (r["size"], r["count_mod_2_64"]) == (ct["size"], ct["count"] % 2 ** 64)
    assert ctx.solve(net_u, plan_u, "tropical_i32", executor="persistent")["size"] == ct["size"]
    assert ctx.solve(net_u, plan_u, "count_exact", executor="persistent")["count"] == oracle.eliminate(gu, "count")["count"]
    want = oracle.eliminate(gw, "tropical")["size"]
    assert ctx.solve(net_w, plan_w, "tropical_f32", executor="persistent")["size"] == want


@pytest.mark.parametrize("side", [14, 16])
@pytest.mark.parametrize("executor", ["stream", "persistent"])
def test_thin_and_dot_modes_vs_oracle(ctx, side, executor):
    """The root of a lattice plan contracts two tensors over all their indices
    (M = N = 1, K >= 2^12) and runs as a long-K reduction; every algebra
    against the oracle.  (Thin nodes come with slicing: see the sliced
    240-vertex test.)"""
    gu = gg.square_lattice(side)
    gw = gu.with_weights(gg.dyadic_weights(gu.nv, 3))
    net_u, net_w = tn.Net.from_graph(gu), tn.Net.from_graph(gw)
    plan_u, plan_w = _plan(net_u, "greedy"), _plan(net_w, "greedy")
    ct = oracle.eliminate(gu, "counting_tropical")
    cnt = oracle.eliminate(gu, "count")["count"]
    trw = oracle.eliminate(gw, "tropical")["size"]
    kinds = set()

    def run(net, plan, sr, **kw):
        if executor == "stream":
            r, recs = _solve_profiled(ctx, net, plan, sr, **kw)
            kinds.update(x["kind"] for x in recs)
            return r
        return ctx.solve(net, plan, sr, executor="persistent", **kw)

    r = run(net_u, plan_u, "counting_tropical")
    assert (r["size"], r["count_mod_2_64"]) == (ct["size"], ct["count"] % 2 ** 64)
    assert run(net_u, plan_u, "tropical_i32")["size"] == ct["size"]
    assert run(net_w, plan_w, "tropical_f32")["size"] == trw
    assert run(net_u, plan_u, "count_exact")["count"] == cnt
    for beta in (0.5, 2.0):
        want = oracle.eliminate(gw, "partition", beta=beta)["log_z"]
        assert abs(run(net_w, plan_w, "partition_f32", beta=beta)["log_z"] - want) <= 1e-5
        assert abs(run(net_w, plan_w, "partition_bf16", beta=beta)["log_z"] - want) <= 0.05
    if executor == "stream":
        print("kernel kinds", sorted(kinds), flush=True)
        assert "gemm_dot" in kinds


def test_square_tile_on_a_hand_made_tree(ctx):
    """Vertex groups I, J (10 each) and K (4): I-K and J-K complete bipartite,
    I-J a perfect matching.  The tree contracts the I-K edges into A(I, K),
    the J-K edges into B(J, K), the matching into C(I, J), then A x B -> (I, J)
    (M = N = 2^10, K = 2^4: 64 tiles of 128 x 128) and finally with C.  The
    oracle is the brute force over the 24 vertices."""
    I, J, K = list(range(10)), list(range(10, 20)), list(range(20, 24))
    edges = [(i, k) for i in I for k in K] + [(j, k) for j in J for k in K] + [(i, i + 10) for i in I]
    g = gg.Graph(24, np.asarray(sorted(edges), np.int32), None, "ijk")
    eid = {tuple(e): n for n, e in enumerate(g.edges.tolist())}
    def chain(es, verts):
        leaves = []
        placed = set()
        for (u, v) in es:
            f = [eid[(u, v)]]
            for x in (u, v):
                if x in verts and x not in placed:
                    placed.add(x)
                    f.append(-x - 1)
            leaves.append(f)
        return leaves
    la = chain([(i, k) for i in I for k in K], set(I) | set(K))
    lb = chain([(j, k) for j in J for k in K], set(J))
    lc = chain([(i, i + 10) for i in I], set())
    leaves = la + lb + lc
    left, right = [], []
    nl = len(leaves)
    def fold(first, count):
        node = first
        for t in range(1, count):
            left.append(node)
            right.append(first + t)
            node = nl + len(left) - 1
        return node
    a = fold(0, len(la))
    b = fold(len(la), len(lb))
    c = fold(len(la) + len(lb), len(lc))
    left.append(a); right.append(b)
    ab = nl + len(left) - 1
    left.append(ab); right.append(c)
    gw = g.with_weights(gg.dyadic_weights(24, 11))
    bf_u = oracle.brute_force(g, betas=[0.5])
    bf_w = oracle.brute_force(gw, betas=[0.5])
    for graph, bf in ((g, bf_u), (gw, bf_w)):
        net = tn.Net.from_graph(graph)
        plan = tn.Plan.from_tree(net, leaves, left, right)
        sr = "tropical_i32" if graph is g else "tropical_f32"
        r, recs = _solve_profiled(ctx, net, plan, sr)
        ran = {(x["shape"][1], x["shape"][2]) for x in recs if x["kind"] == "gemm_big"}
        print(f"{sr}: big-tile shapes (log2 M, N) {sorted(ran)}", flush=True)
        assert (10, 10) in ran and _tile([0, 10, 10, 4]) == (7, 7)
        assert r["size"] == bf["size_max"]
        z, _ = _solve_profiled(ctx, net, plan, "partition_f32", beta=0.5)
        assert abs(z["log_z"] - bf["log_z"][0]) <= 1e-5
    net = tn.Net.from_graph(g)
    plan = tn.Plan.from_tree(net, leaves, left, right)
    r, recs = _solve_profiled(ctx, net, plan, "count_exact")
    assert (10, 10) in {(x["shape"][1], x["shape"][2]) for x in recs if x["kind"] == "gemm_big"}
    assert r["count"] == bf_u["count_all"]
    r = ctx.solve(net, plan, "counting_tropical", executor="stream")
    assert (r["size"], r["count_mod_2_64"]) == (bf_u["size_max"], bf_u["count_max"])
    r = ctx.solve(net, plan, "tropical_i32", executor="persistent")
    assert r["size"] == bf_u["size_max"]


def _with_pendant_paths(g, two, three):
    """g with a pendant path of two vertices hung on every vertex in `two`
    and one of three vertices on every vertex in `three`.  A path v-a-b adds
    one to any maximum set (b with v, else a or b: two ways when v is out); a
    path v-a-b-c adds two (one way when v is out, two when v is in), so the
    number of maximum sets is the sum over the base graph's maximum sets S of
    2^(|two \\ S| + |three & S|): counts of 2^40 and more, also in the large
    intermediate tensors."""
    e = [tuple(x) for x in g.edges.tolist()]
    nv = g.nv
    for v in two:
        e += [(v, nv), (nv, nv + 1)]
        nv += 2
    for v in three:
        e += [(v, nv), (nv, nv + 1), (nv + 1, nv + 2)]
        nv += 3
    es = sorted({(min(u, v), max(u, v)) for u, v in e})
    return gg.Graph(nv, np.array(es, np.int32).reshape(-1, 2), None, g.name + "+paths")


@pytest.mark.parametrize("base", ["lattice14", "rr120"])
def test_counting_tropical_big_tiles_with_counts_above_2_32(ctx, base):
    """The counting-tropical tiles take a 32-bit product path when every
    count of a K step is below 2^32 and the full 64-bit product otherwise;
    pendant paths make the counts of the large nodes exceed 2^32."""
    g0 = gg.square_lattice(14) if base == "lattice14" else gg.random_regular(120, 3, 5)
    rng = np.random.default_rng(3)
    perm = rng.permutation(g0.nv)
    two, three = sorted(perm[: g0.nv // 2].tolist()), sorted(perm[g0.nv // 2: g0.nv // 2 + g0.nv // 4].tolist())
    g = _with_pendant_paths(g0, two, three)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, seed=0)
    want = oracle.eliminate(g, "counting_tropical")
    print(f"{base}+paths: {g.nv} vertices, complexity {plan.complexity()}, size {want['size']}, "
          f"count 2^{float(np.log2(float(want['count']))):.1f}", flush=True)
    assert want["count"] > 2 ** 48
    r, recs = _solve_profiled(ctx, net, plan, "counting_tropical")
    ran = {_ct_tile(x["shape"]) for x in recs if x["kind"] == "gemm_big"}
    print(f"  tiles {sorted(ran, key=str)}: {r['size']}, {r['count_mod_2_64']}", flush=True)
    assert ran - {None}
    assert (r["size"], r["count_mod_2_64"]) == (want["size"], want["count"] % 2 ** 64)
    rp = ctx.solve(net, plan, "counting_tropical", executor="persistent")
    assert (rp["size"], rp["count_mod_2_64"]) == (want["size"], want["count"] % 2 ** 64)


@pytest.mark.parametrize("ntwo,nthree", [(8, 4), (12, 6), (16, 8)])
def test_counting_tropical_big_tiles_with_counts_around_2_14(ctx, ntwo, nthree):
    """Below 2^floor((32 - tk) / 2) (2^14 for the tiles' K step of 16) a K
    step's counts take the 24-bit path, up to 2^32 the 32-bit one: a few
    pendant paths on the 120-vertex graph put the number of maximum sets at
    2^13.9, 2^18.1 and 2^21.3, so the large nodes hold counts on both sides
    of the line and their tiles switch paths from step to step."""
    g0 = gg.random_regular(120, 3, 5)
    perm = np.random.default_rng(4).permutation(g0.nv)
    two, three = sorted(perm[:ntwo].tolist()), sorted(perm[ntwo:ntwo + nthree].tolist())
    g = _with_pendant_paths(g0, two, three)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, seed=0)
    want = oracle.eliminate(g, "counting_tropical")
    print(f"rr120+{ntwo}+{nthree}: complexity {plan.complexity()}, size {want['size']}, "
          f"count 2^{float(np.log2(float(want['count']))):.1f}", flush=True)
    assert 2 ** 13 < want["count"] < 2 ** 32
    r, recs = _solve_profiled(ctx, net, plan, "counting_tropical")
    assert {_ct_tile(x["shape"]) for x in recs if x["kind"] == "gemm_big"} - {None}
    assert (r["size"], r["count_mod_2_64"]) == (want["size"], want["count"])
    rp = ctx.solve(net, plan, "counting_tropical", executor="persistent")
    assert (rp["size"], rp["count_mod_2_64"]) == (want["size"], want["count"])


def test_thin_nodes_with_four_or_more_columns_every_algebra(ctx):
    """A sliced plan of the 120-vertex graph has thin nodes (M >= 2^10,
    N * K <= 32) with N >= 4, which store four consecutive outputs per lane:
    every algebra against the oracle (per-node launches: the persistent
    executor takes unsliced plans only)."""
    executor = "stream"
    g = gg.random_regular(120, 3, 0)
    gw = g.with_weights(gg.dyadic_weights(g.nv, 0))
    net, netw = tn.Net.from_graph(g), tn.Net.from_graph(gw)
    kw = dict(method="treesa", ntrials=4, niters=10, sc_target=14, nslices=20, seed=0)
    plan, planw = tn.Plan.create(net, **kw), tn.Plan.create(netw, **kw)
    for sr in ("tropical_f32", "counting_tropical"):
        thin = [d for d in plan.gemm_shapes(sr) if d["kind"] == "gemm_thin" and d["lj"] >= 2]
        print(sr, "thin nodes with N >= 4:", [(d["lb"], d["li"], d["lj"], d["lk"]) for d in thin], flush=True)
        assert thin
    ct = oracle.eliminate(g, "counting_tropical")
    kinds = set()

    def run(n, p, sr, **k):
        if executor == "stream":
            r, recs = _solve_profiled(ctx, n, p, sr, **k)
            kinds.update(x["kind"] for x in recs)
            return r
        return ctx.solve(n, p, sr, executor="persistent", **k)

    r = run(net, plan, "counting_tropical")
    assert (r["size"], r["count_mod_2_64"]) == (ct["size"], ct["count"] % 2 ** 64)
    assert run(net, plan, "tropical_i32")["size"] == ct["size"]
    assert run(netw, planw, "tropical_f32")["size"] == oracle.eliminate(gw, "tropical")["size"]
    assert run(net, plan, "count_exact")["count"] == oracle.eliminate(g, "count")["count"]
    want = oracle.eliminate(gw, "partition", beta=1.0)["log_z"]
    assert abs(run(netw, planw, "partition_f32", beta=1.0)["log_z"] - want) <= 1e-5
    assert abs(run(netw, planw, "partition_bf16", beta=1.0)["log_z"] - want) <= 0.05
    if executor == "stream":
        assert "gemm_thin" in kinds
