"""Checkpoint and resume of a sliced contraction: a 32-slice plan of the
120-vertex graph contracted in three slice ranges, each result stored as
bytes and read back, then combined (tn_result_combine), equals the
contraction over all slices in every algebra (bit for bit where the algebra
is exact)."""
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


def test_three_slice_ranges_combine_to_the_whole(ctx):
    g = gg.random_regular(120, 3, 0)
    gw = g.with_weights(gg.dyadic_weights(g.nv, 0))
    kw = dict(method="treesa", ntrials=4, niters=10, sc_target=14, nslices=20, seed=0)
    net, netw = tn.Net.from_graph(g), tn.Net.from_graph(gw)
    plan, planw = tn.Plan.create(net, **kw), tn.Plan.create(netw, **kw)
    ns = 1 << plan.info()["nsliced"]
    assert ns == 1 << planw.info()["nsliced"] and ns >= 8
    cuts = [0, ns // 3, (2 * ns) // 3, ns]
    cases = [(net, plan, "tropical_i32", {}), (netw, planw, "tropical_f32", {}), (net, plan, "counting_tropical", {}),
             (net, plan, "count_exact", {}), (netw, planw, "partition_f32", {"beta": 1.0})]
    for n, p, sr, extra in cases:
        whole = ctx.solve(n, p, sr, **extra)
        acc = None
        for a, b in zip(cuts, cuts[1:]):
            r = ctx.solve_result(n, p, sr, slices=(a, b), **extra)
            stored = bytes(r)  # a checkpoint: the partial result and the next slice index b
            r = tn.tn_result.from_buffer_copy(stored)
            acc = r if acc is None else tn.result_combine(acc, r)
        got = tn.decode(acc)
        print(sr, {k: got.get(k) for k in ("size", "count_mod_2_64", "count", "log_z")}, flush=True)
        if sr == "partition_f32":
            assert abs(got["log_z"] - whole["log_z"]) <= 1e-12 * abs(whole["log_z"])
        else:
            for k in ("size", "count_mod_2_64", "count"):
                assert got.get(k) == whole.get(k), (sr, k, got, whole)
    # the oracle's value from a first slice and the rest
    ct = oracle.eliminate(g, "counting_tropical")
    first = ctx.solve_result(net, plan, "counting_tropical", slices=(0, 1))
    rest = ctx.solve_result(net, plan, "counting_tropical", slices=(1, ns))
    got = tn.decode(tn.result_combine(first, rest))
    assert (got["size"], got["count_mod_2_64"]) == (ct["size"], ct["count"] % 2 ** 64)
