"""GPU parity at 2^30-entry intermediates against independent values.

* The 3 x 29 grid contracted along the explicit tree of tests/wide_trees.py:
  its largest node multiplies a 2^29-entry operand by a 2^11-entry one over
  five summed indices into a 2^30-entry result (2^35 semiring operations, on
  the register-tiled kernels, or matrix cores for Z), and the nodes around it
  permute and stream tensors of 2^29-2^30 entries (for counting tropical the
  8-byte count plane of a rank-30 tensor is 8 GiB, so byte offsets pass
  2^32).  The grid's treewidth is 3, so the oracle's variable elimination, an
  algorithm that shares nothing with a contraction tree, gives every expected
  value exactly.
* The 20 x 20 grid of the Sec. 5.1 example: Z(0) against the value printed
  there, and the exact count (about 2^239, which takes nine CRT primes and a
  check prime) against the oracle's 256-bit elimination
  (tests/golden/square20.json, written by make_golden_square20.py).
"""
import json
import math
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2501_00227_amd as tn
from wide_trees import three_row_gemm_tree

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(__file__), "golden")
W, M = 29, 5


@pytest.fixture(scope="module")
def ctx():
    tn.lib()
    c = tn.Context(0)
    yield c
    c.set_profiling(False)
    c.synchronize()


def _wide(weights=None):
    g = gg.grid(3, W)
    if weights == "int":
        g = g.with_weights(gg.integer_weights(g.nv, 7, 1, 4))
    elif weights == "dyadic":
        g = g.with_weights(gg.dyadic_weights(g.nv, 7))
    net = tn.Net.from_graph(g)
    leaves, left, right = three_row_gemm_tree(W, M, g.edges)
    plan = tn.Plan.from_tree(net, leaves, left, right)
    info = plan.info()
    assert info["max_rank"] == W + 1, info
    return g, net, plan, leaves, left, right


def _profiled(ctx, fn):
    ctx.set_profiling(True)
    ctx.profile(clear=True)
    try:
        out = fn()
        recs = ctx.profile(clear=True)
    finally:
        ctx.set_profiling(False)
    return out, recs


def _assert_full_size(recs, big_kind):
    """The run really went through 2^30-entry tensors: a rank-30 permute and
    the 2^35-operation GEMM on the expected kernel family."""
    perms = [r for r in recs if r["kind"] == "permute"]
    assert max(r["shape"][0] for r in perms) == W + 1, sorted({r["shape"][0] for r in perms})
    big = [r for r in recs if r["ops"] == 2.0 ** (W + 1 + M)]
    assert big and all(r["kind"] == big_kind for r in big), [(r["kind"], r["shape"]) for r in big]


def test_wide_tree_tropical_vs_elimination(ctx):
    g, net, plan, *_ = _wide("int")
    want = oracle.eliminate(g, "tropical")["size"]
    print(f"3x{W} grid, integer weights, plan {plan.complexity()}, oracle size {want}", flush=True)
    r, recs = _profiled(ctx, lambda: ctx.solve(net, plan, "tropical_i32", executor="stream"))
    assert r["size"] == want
    _assert_full_size(recs, "gemm_big")
    g, net, plan, *_ = _wide("dyadic")
    want = oracle.eliminate(g, "tropical")["size"]
    r, recs = _profiled(ctx, lambda: ctx.solve(net, plan, "tropical_f32"))
    print(f"  dyadic weights: gpu {r['size']!r} oracle {want!r}", flush=True)
    assert r["size"] == want  # weights k/2^14: every partial sum is exact in float32
    _assert_full_size(recs, "gemm_big")


def test_wide_tree_counting_tropical_vs_elimination(ctx):
    g, net, plan, *_ = _wide()
    want = oracle.eliminate(g, "counting_tropical")
    r, recs = _profiled(ctx, lambda: ctx.solve(net, plan, "counting_tropical"))
    print(f"3x{W} grid counting tropical: gpu ({r['size']}, {r['count_mod_2_64']}) oracle {want}", flush=True)
    assert (r["size"], r["count_mod_2_64"]) == (want["size"], want["count"] % 2 ** 64)
    _assert_full_size(recs, "gemm_big")
    # both planes of the rank-30 tensors were permuted (4-byte sizes, 8-byte counts)
    p30 = [r for r in recs if r["kind"] == "permute" and r["shape"][0] == W + 1]
    assert {round(r["alg_bytes"] / 2 ** (W + 2)) for r in p30} >= {4, 8}


def test_wide_tree_exact_count_vs_elimination(ctx):
    g, net, plan, *_ = _wide()
    want = oracle.eliminate(g, "count")["count"]
    r = ctx.solve(net, plan, "count_exact")
    print(f"3x{W} grid exact count: gpu {r['count']} oracle {want} ({len(r['primes'])} primes)", flush=True)
    assert r["count"] == want


def test_wide_tree_partition_function_vs_elimination(ctx):
    g, net, plan, *_ = _wide()
    for beta in (0.0, 1.0):
        want = oracle.eliminate(g, "partition", beta)["log_z"]
        r, recs = _profiled(ctx, lambda: ctx.solve(net, plan, "partition_f32", beta=beta))
        rb = ctx.solve(net, plan, "partition_bf16", beta=beta)
        print(f"  beta {beta}: ln Z fp32 err {r['log_z'] - want:+.3e}, bf16 inputs err {rb['log_z'] - want:+.3e}",
              flush=True)
        assert abs(r["log_z"] - want) <= 1e-5
        assert abs(rb["log_z"] - want) <= 5e-2
        _assert_full_size(recs, "gemm_mfma")


def test_wide_tree_sliced_vs_elimination(ctx):
    """The same tree with one of the big node's summed indices sliced: two
    slices of 2^34 operations, accumulated by the slice loop."""
    g, net, _, leaves, left, right = _wide("int")
    plan = tn.Plan.from_tree(net, leaves, left, right, sliced=[W + 2])  # vertex (1, 2)
    assert plan.info()["nsliced"] == 1 and plan.info()["max_rank"] == W + 1
    want = oracle.eliminate(g, "tropical")["size"]
    assert ctx.solve(net, plan, "tropical_i32")["size"] == want
    parts = [ctx.solve(net, plan, "tropical_i32", slices=(s, s + 1))["size"] for s in (0, 1)]
    assert max(parts) == want


def test_square20_paper_value_and_exact_count(ctx):
    gold = json.load(open(os.path.join(GOLD, "square20.json")))
    printed = json.load(open(os.path.join(GOLD, "paper_values.json")))["square20"]["partition_beta0"]["value"]
    g = gg.square_lattice(20)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net)
    print("20x20 grid plan", plan.complexity(), flush=True)
    r = ctx.solve(net, plan, "count_exact")
    print(f"  exact count {r['count']} with {len(r['primes'])} primes", flush=True)
    assert r["count"] == int(gold["count"])
    assert abs(r["count"] - printed) / printed < 1e-15
    z = ctx.solve(net, plan, "partition_f32", beta=0.0)
    print(f"  Z(0) = {z['z']!r}, printed {printed!r}", flush=True)
    assert abs(z["z"] - printed) / printed <= 1e-5
    for beta, want in gold["log_z"].items():
        r = ctx.solve(net, plan, "partition_f32", beta=float(beta))
        assert abs(r["log_z"] - want) <= 1e-5, (beta, r["log_z"], want)
    r = ctx.solve(net, plan, "counting_tropical")
    assert [r["size"], str(r["count_mod_2_64"])] == [gold["counting_tropical"][0],
                                                     str(int(gold["counting_tropical"][1]) % 2 ** 64)]
    assert ctx.solve(net, plan, "tropical_i32")["size"] == gold["counting_tropical"][0]
