"""The launch-shape autotuner on the GPU.

Tuning times every candidate shape of a node on seeded operands and rejects
any whose result differs from the heuristic shape's: on the n=120 network
every candidate of every tuned node must agree bit for bit in the exact
algebras (a consistency check of all tile families against each other).
With the tuned table, results still equal the oracle's, and a job's result
is the same alone and in a batch of other jobs.
"""
import pytest

import graphgen as gg
import oracle
import paper_2501_00227_amd as tn

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    tn.lib()
    c = tn.Context(0)
    tn.tune_clear()
    yield c
    tn.tune_clear()
    c.synchronize()


def test_tuned_shapes_agree_and_match_the_oracle(ctx, tmp_path):
    g = gg.random_regular(120, 3, 4)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=4, niters=10, seed=4)
    before = {sr: plan.gemm_shapes(sr) for sr in ("tropical_i32", "counting_tropical", "count_exact", "partition_f32")}
    for sr in before:
        n = ctx.tune_plan(plan, sr, min_log2_ops=16, reps=2)
        print(f"tuned {sr}: {n} node shapes", flush=True)
        assert n > 0
    recs = tn.tune_records()
    for r in recs:
        print({k: r[k] for k in ("dsr", "lb", "li", "lj", "lk", "ncand", "nrejected", "heuristic_ms", "best_ms")},
              r["shape"], flush=True)
        assert r["ncand"] >= 1 and r["best_ms"] <= r["heuristic_ms"] * 1.0001
        if r["dsr"] in (0, 1, 2, 3):  # exact algebras: every candidate reproduced the heuristic's bits
            assert r["nrejected"] == 0, r
    assert any(r["ncand"] > 5 for r in recs)
    changed = sum(a != b for sr in before for a, b in zip(before[sr], plan.gemm_shapes(sr)))
    print("node launch shapes changed by tuning:", changed, flush=True)
    ref = {s: oracle.eliminate(g, s) for s in ("tropical", "counting_tropical", "count")}
    refz = oracle.eliminate(g, "partition", 0.5)
    for ex in ("stream", "persistent"):
        assert ctx.solve(net, plan, "tropical_i32", executor=ex)["size"] == ref["tropical"]["size"]
        r = ctx.solve(net, plan, "counting_tropical", executor=ex)
        assert (r["size"], r["count_mod_2_64"]) == (ref["counting_tropical"]["size"],
                                                    ref["counting_tropical"]["count"] % 2 ** 64)
        assert ctx.solve(net, plan, "count_exact", executor=ex)["count"] == ref["count"]["count"]
        assert abs(ctx.solve(net, plan, "partition_f32", beta=0.5, executor=ex)["log_z"] - refz["log_z"]) <= 1e-5
    # alone vs in a batch with other jobs, tuned shapes
    others = [gg.random_regular(n, 3, 10 + n) for n in (40, 60, 80, 100)]
    onets = [tn.Net.from_graph(x) for x in others]
    oplans = [tn.Plan.create(x) for x in onets]
    for sr in ("counting_tropical", "partition_f32"):
        alone = ctx.solve_batch([net], [plan], sr)[0]
        mixed = ctx.solve_batch(onets + [net] + onets, oplans + [plan] + oplans, sr)[len(onets)]
        for k in ("size", "count_mod_2_64", "z_mant", "z_exp2"):
            assert alone.get(k) == mixed.get(k), (sr, k, alone, mixed)
    # save, clear, load: the same shapes again
    path = str(tmp_path / "t.tune")
    n = tn.tune_save(path)
    after = {sr: plan.gemm_shapes(sr) for sr in before}
    tn.tune_clear()
    assert {sr: plan.gemm_shapes(sr) for sr in before} == before
    assert tn.tune_load(path) == n
    assert {sr: plan.gemm_shapes(sr) for sr in before} == after
