"""The scratch-free entry point (tn_solve_noalloc) through the C ABI.

It must give tn_solve's results (per-node launches, executor 1): bit-exact in
the integer algebras, and the partition function within 1e-5 relative (the
same kernels in the same order, so in practice identical), on two calls in
a row, the second with a smaller network, for every algebra; make no call
of the context's device allocator; and refuse a solve larger than its
scratch array with TN_ETOOBIG before touching the device.
"""
import ctypes
import math

import pytest

import graphgen as gg
import paper_2501_00227_amd as tn

pytestmark = pytest.mark.gpu
SEMIRINGS = ["tropical_i32", "tropical_f32", "counting_tropical", "count_exact", "partition_f32", "partition_bf16"]


@pytest.fixture(scope="module")
def counted():
    """A context whose device allocator counts its calls (then hands them to
    torch's caching allocator)."""
    import torch

    tn.lib()
    torch.cuda.set_device(0)
    calls = {"alloc": 0, "free": 0}
    t_alloc, t_free = torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete

    def _alloc(nbytes, user, stream):
        calls["alloc"] += 1
        try:
            return t_alloc(int(nbytes), 0, int(stream or 0))
        except Exception:
            return None

    def _free(ptr, nbytes, user, stream):
        calls["free"] += 1
        t_free(int(ptr))

    a_cb, f_cb = tn.ALLOC_FN(_alloc), tn.FREE_FN(_free)
    alloc = tn.tn_allocator(ctypes.cast(a_cb, ctypes.c_void_p), ctypes.cast(f_cb, ctypes.c_void_p), None)
    h = ctypes.c_void_p()
    stream = torch.cuda.current_stream(0).cuda_stream
    tn._check(tn.lib().tn_ctx_create(0, ctypes.c_void_p(stream), ctypes.byref(alloc), ctypes.byref(h)))
    ctx = tn.Context.__new__(tn.Context)
    ctx._cb = (a_cb, f_cb)
    ctx.h = h
    tn._live.add(ctx)
    yield ctx, calls
    ctx.synchronize()
    ctx.close()


def _same(sr, a, b):
    if sr.startswith("partition"):
        assert math.isfinite(b["log_z"]) and abs(a["log_z"] - b["log_z"]) <= 1e-5, (sr, a, b)
    else:
        keys = {"tropical_i32": ["size"], "tropical_f32": ["size"], "counting_tropical": ["size", "count_mod_2_64"],
                "count_exact": ["count", "residues", "primes"]}[sr]
        assert {k: a[k] for k in keys} == {k: b[k] for k in keys}, (sr, a, b)


def _case(g, **plan_kw):
    net = tn.Net.from_graph(g)
    return net, tn.Plan.create(net, **plan_kw)


def test_noalloc_matches_solve_on_two_calls_in_a_row(counted):
    ctx, calls = counted
    big = _case(gg.random_regular(120, 3, 1))
    small = _case(gg.random_regular(40, 3, 2))
    for sr in SEMIRINGS:
        beta = 0.7 if sr.startswith("partition") else 0.0
        for name, (net, plan) in (("n=120", big), ("n=40", small)):
            print(f"noalloc {sr} {name}", flush=True)
            want = ctx.solve(net, plan, sr, beta=beta, executor="stream")
            before = dict(calls)
            got = ctx.solve_noalloc(net, plan, sr, beta=beta)
            assert calls == before, "the scratch-free entry point called the device allocator"
            _same(sr, got, want)


def test_noalloc_weighted_and_sliced(counted):
    ctx, calls = counted
    g = gg.kings_subgraph(8, 0.8, 3)
    g = g.with_weights(gg.dyadic_weights(g.nv, 3))
    net, plan = _case(g, method="treesa", ntrials=2, niters=5, sc_target=6, nslices=4, seed=3)
    assert plan.info()["nsliced"] > 0
    for sr, beta in (("tropical_f32", 0.0), ("partition_f32", 1.5), ("count_exact", 0.0)):
        for sl in (None, (1, 3)):
            print(f"noalloc sliced {sr} slices={sl}", flush=True)
            want = ctx.solve(net, plan, sr, beta=beta, slices=sl, executor="stream")
            before = dict(calls)
            got = ctx.solve_noalloc(net, plan, sr, beta=beta, slices=sl)
            assert calls == before
            _same(sr, got, want)
    # an empty network (no leaves) and a second small call after it
    net0, plan0 = _case(gg.empty(0))
    assert ctx.solve_noalloc(net0, plan0, "count_exact")["count"] == 1
    net1, plan1 = _case(gg.cycle(7))
    assert ctx.solve_noalloc(net1, plan1, "count_exact")["count"] == 29  # Lucas L_7


def test_noalloc_refuses_solves_above_its_scratch(counted):
    ctx, _ = counted
    net, plan = _case(gg.random_regular(200, 3, 0), sc_target=30)
    need = plan.peak_bytes("tropical_i32")
    print("n=200 plan needs", need, flush=True)
    assert need > 256 << 20
    with pytest.raises(tn.TnError) as ei:
        ctx.solve_noalloc(net, plan, "tropical_i32")
    assert ei.value.code == tn.TN_ETOOBIG
    o = tn.solve_opts("tropical_i32", executor="persistent")
    assert tn.lib().tn_solve_noalloc(ctx.h, net.h, plan.h, ctypes.byref(o), ctypes.byref(tn.tn_result())) \
        == tn.TN_EINVAL
