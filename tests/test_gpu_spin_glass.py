"""GPU tests of the spin glass (Sec. 2 energy H = sum J s_u s_v + sum h s_v;
the Sec. 6.4 buckyball example): the same contraction path with spin-glass
leaf tensors, every algebra on both executors, against the paper's printed
buckyball values and the oracle (brute force, elimination)."""
import json
import os
import random

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


@pytest.mark.parametrize("executor", ["stream", "persistent"])
def test_buckyball_matches_paper(ctx, executor):
    g = gg.fullerene()
    net = tn.Net.spin_glass(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=4, niters=10, seed=0)
    fp = GOLD["fullerene"]
    r = ctx.solve(net, plan, "partition_f32", beta=1.0, executor=executor)
    print(f"{executor}: ln Z / N = {r['log_z'] / g.nv!r}", flush=True)
    assert abs(r["log_z"] - g.nv * fp["log_z_per_vertex_beta1"]["value"]) <= 1e-5
    rb = ctx.solve(net, plan, "partition_bf16", beta=1.0, executor=executor)
    assert abs(rb["log_z"] - g.nv * fp["log_z_per_vertex_beta1"]["value"]) <= 0.05
    ct = ctx.solve(net, plan, "counting_tropical", executor=executor)
    assert [-ct["size"], ct["count_mod_2_64"]] == fp["counting_min"]["value"]
    assert ctx.solve(net, plan, "tropical_i32", executor=executor)["size"] == 66
    assert ctx.solve(net, plan, "tropical_f32", executor=executor)["size"] == 66
    assert ctx.solve(net, plan, "count_exact", executor=executor)["count"] == 2 ** 60


def test_random_spin_glasses_match_brute_force(ctx):
    rng = random.Random(3)
    for t in range(16):
        n = rng.randint(2, 18)
        g = gg.gnp(n, rng.uniform(0.15, 0.6), 200 + t)
        J = [float(rng.randint(-3, 3)) for _ in range(g.ne)]
        h = [float(rng.randint(-2, 2)) for _ in range(n)]
        beta = rng.choice([0.2, 0.5, 1.0])
        bf = oracle.spin_glass_brute_force(g, J, h, betas=[beta])
        net = tn.Net.spin_glass(g, J, h)
        plan = tn.Plan.create(net, seed=t)
        for ex in ("stream", "persistent"):
            ct = ctx.solve(net, plan, "counting_tropical", executor=ex)
            assert (-ct["size"], ct["count_mod_2_64"]) == (bf["energy_min"], bf["count_min"]), (t, ex)
            assert ctx.solve(net, plan, "tropical_i32", executor=ex)["size"] == -bf["energy_min"]
            assert ctx.solve(net, plan, "tropical_f32", executor=ex)["size"] == -bf["energy_min"]
            z = ctx.solve(net, plan, "partition_f32", beta=beta, executor=ex)["log_z"]
            assert abs(z - bf["log_z"][0]) <= 1e-5, (t, ex, z, bf["log_z"][0])
            assert ctx.solve(net, plan, "count_exact", executor=ex)["count"] == 2 ** n


@pytest.mark.parametrize("n,seed", [(60, 0), (100, 1)])
def test_regular_spin_glass_matches_elimination(ctx, n, seed):
    g = gg.random_regular(n, 3, seed)
    rng = random.Random(seed)
    J = [rng.choice([-1.0, 1.0]) for _ in range(g.ne)]  # +-J glass
    net = tn.Net.spin_glass(g, J)
    plan = tn.Plan.create(net, method="treesa", ntrials=2, niters=5, seed=seed)
    ct_ref = oracle.spin_glass_eliminate(g, "counting_tropical", J=J)
    z_ref = oracle.spin_glass_eliminate(g, "partition", J=J, beta=0.7)["log_z"]
    ct = ctx.solve(net, plan, "counting_tropical")
    print(f"n={n}: ground state {-ct['size']} x {ct['count_mod_2_64']}", flush=True)
    assert (ct["size"], ct["count_mod_2_64"]) == (ct_ref["size"], ct_ref["count"] % 2 ** 64)
    assert abs(ctx.solve(net, plan, "partition_f32", beta=0.7)["log_z"] - z_ref) <= 1e-5


def test_spin_glass_rejections(ctx):
    g = gg.petersen()
    net = tn.Net.spin_glass(g, J=[0.5] * g.ne)
    plan = tn.Plan.create(net)
    with pytest.raises(tn.TnError) as ei:  # non-integer couplings in int32 max-plus
        ctx.solve(net, plan, "tropical_i32")
    assert ei.value.code == tn.TN_EINVAL
    assert ctx.solve(net, plan, "tropical_f32")["size"] == -oracle.spin_glass_brute_force(g, [0.5] * g.ne)["energy_min"]
    with pytest.raises(tn.TnError) as ei:
        ctx.solve_polynomial(net, plan)
    assert ei.value.code == tn.TN_EINVAL
    inet = tn.Net.from_graph(g)  # a plan of the IS network does not fit the spin glass
    with pytest.raises(tn.TnError) as ei:
        ctx.solve(net, tn.Plan.create(inet), "tropical_f32")
    assert ei.value.code == tn.TN_EINVAL
