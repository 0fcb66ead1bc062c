"""Served stream and failure handling on the GPU.

* Admission binds: a burst of jobs whose device bytes far exceed the HBM
  budget is served in several admission rounds, the admitted bytes never
  pass the budget, the server's device pool high-water mark stays within
  the budget plus the task-table reserve, and every result equals the job's
  result alone and the oracle's.
* Launches overlap: jobs admitted while a long launch runs go out at once on
  another stream (two launches in flight together).
* Jobs still queued can be cancelled; a job above the budget is refused.
* Failures forced from the host end cleanly: a dependency-wait limit so small
  that the persistent launch gives up (every workgroup leaves, TN_EDEVICE),
  an allocator that returns NULL (TN_ENOMEM); the same context then solves
  correctly again.
"""
import ctypes

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
    c.set_wait_limit(10.0)
    c.synchronize()


def _key(r):
    return tuple(r.get(k) for k in ("size", "count_mod_2_64", "count", "z_mant", "z_exp2"))


def _jobs(n, seed, n_lo, n_hi):
    import random

    rng = random.Random(seed)
    out = []
    for k in range(n):
        nv = rng.randrange(n_lo, n_hi + 1, 2)
        g = gg.random_regular(nv, 3, 1000 * seed + k)
        net = tn.Net.from_graph(g)
        plan = tn.Plan.create(net, seed=k)
        sr = ["tropical_i32", "counting_tropical", "partition_f32"][k % 3]
        out.append((g, net, plan, sr))
    return out


def test_admission_binds(ctx):
    jobs = _jobs(48, seed=7, n_lo=60, n_hi=110)
    sizes = sorted(p.peak_bytes(sr) for _, _, p, sr in jobs)
    budget = max(4 * sizes[len(sizes) // 2], (3 * sizes[-1]) // 2)  # a few jobs at a time, any job fits
    total = sum(sizes)
    print(f"budget {budget} bytes, the burst needs {total} ({total / budget:.1f} x)", flush=True)
    assert total > 3 * budget
    alone = [ctx.solve(net, plan, sr, executor="persistent") for _, net, plan, sr in jobs]
    srv = tn.Server(ctx, budget, max_slots=64)
    ids = [srv.submit(net, plan, sr) for _, net, plan, sr in jobs]  # one burst
    srv.drain()
    res = [srv.poll(i) for i in ids]
    st = srv.stats()
    srv.close()
    print("server stats", st, flush=True)
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["launches"] >= 3                      # the budget split the burst
    assert st["peak_admitted_bytes"] <= budget
    assert st["peak_pool_bytes"] <= budget + (64 << 20)
    for (g, _, _, sr), r, a in zip(jobs, res, alone):
        assert r is not None and _key(r) == _key(a)
    # every tropical / counting result against the oracle (n <= 110: elimination)
    for (g, _, _, sr), r in zip(jobs, res):
        if sr == "tropical_i32":
            assert r["size"] == oracle.eliminate(g, "tropical")["size"]
        elif sr == "counting_tropical":
            ref = oracle.eliminate(g, "counting_tropical")
            assert (r["size"], r["count_mod_2_64"]) == (ref["size"], ref["count"] % 2 ** 64)


def test_launches_overlap_on_the_device(ctx):
    """A job admitted while an earlier launch still runs goes out at once on
    another stream: a long per-node job (counting tropical on n=170, some
    2^35 ops) is submitted, and once it is on the device small jobs follow;
    at least two launches are then in flight together."""
    import time

    g = gg.random_regular(170, 3, 170)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, seed=1)
    assert plan.complexity()[0] > 33
    small = _jobs(8, seed=11, n_lo=40, n_hi=80)
    want = ctx.solve(net, plan, "counting_tropical")
    alone = [ctx.solve(n2, p2, sr) for _, n2, p2, sr in small]
    srv = tn.Server(ctx, 32 << 30, max_slots=64)
    big = srv.submit(net, plan, "counting_tropical")
    t0 = time.perf_counter()
    while srv.stats()["launches"] < 1 and time.perf_counter() - t0 < 5.0:
        time.sleep(1e-4)
    ids = [srv.submit(n2, p2, sr) for _, n2, p2, sr in small]
    srv.drain()
    r = srv.poll(big)
    assert (r["size"], r["count_mod_2_64"]) == (want["size"], want["count_mod_2_64"])
    for jid, a in zip(ids, alone):
        assert _key(srv.poll(jid)) == _key(a)
    st = srv.stats()
    srv.close()
    print("server stats", st, flush=True)
    assert st["peak_inflight"] >= 2


def test_cancel_queued_jobs_and_refuse_oversized(ctx):
    g = gg.random_regular(150, 3, 3)
    net = tn.Net.from_graph(g)
    big = tn.Plan.create(net, method="treesa", ntrials=2, niters=5, sc_target=24, seed=3)
    small = _jobs(6, seed=8, n_lo=20, n_hi=30)
    srv = tn.Server(ctx, 32 << 30, max_slots=1)
    first = srv.submit(net, big, "counting_tropical")
    queued = [srv.submit(n2, p2, sr) for _, n2, p2, sr in small]
    cancelled = []
    for jid in queued[2:]:
        try:
            srv.cancel(jid)
            cancelled.append(jid)
        except tn.TnError as e:
            assert e.code == tn.TN_EBUSY
    srv.drain()
    r = srv.poll(first)  # a large tree: served alone on per-node launches
    want = ctx.solve(net, big, "counting_tropical")
    assert (r["size"], r["count_mod_2_64"]) == (want["size"], want["count_mod_2_64"])
    for jid in queued:
        if jid in cancelled:
            with pytest.raises(tn.TnError) as ei:
                srv.poll(jid)
            assert ei.value.code == tn.TN_ECANCELED
        else:
            assert srv.poll(jid) is not None
    st = srv.stats()
    assert st["canceled"] == len(cancelled) >= 1
    srv.close()
    tiny = tn.Server(ctx, 1 << 16, max_slots=1)
    with pytest.raises(tn.TnError) as ei:  # a job far above the budget
        tiny.submit(net, big, "counting_tropical")
    assert ei.value.code == tn.TN_ETOOBIG
    assert tiny.stats()["rejected"] == 1
    tiny.close()


def _kinds(ctx, fn):
    ctx.set_profiling(True)
    try:
        ctx.profile(clear=True)
        out = fn()
        kinds = {r["kind"] for r in ctx.profile(clear=True)}
    finally:
        ctx.set_profiling(False)
    return out, kinds


def test_routes_of_large_trees(ctx):
    """Alone, trees with more than 2^27 ops per pass run on per-node launches.
    Launched together (a batch, the server), mid-size trees of the exact
    algebras (2^27 to 2^31 ops, intermediates up to 2^24 entries) share the
    persistent launch; the real algebra's large trees and trees above 2^31
    ops go out on per-node launches.  Every route gives the job's result
    alone."""
    small = _jobs(6, seed=9, n_lo=30, n_hi=60)
    nets = {}
    for n in (140, 150):
        g = gg.random_regular(n, 3, n)
        net = tn.Net.from_graph(g)
        nets[n] = (g, net, tn.Plan.create(net, seed=1))
    tc140, tc150 = nets[140][2].complexity()[0], nets[150][2].complexity()[0]
    assert 27 < tc140 <= 31 and nets[140][2].info()["max_rank"] <= 24 and tc150 > 31
    mids = [nets[140] + ("tropical_i32",), nets[140] + ("counting_tropical",)]
    bigs = [nets[150] + ("tropical_i32",), nets[140] + ("partition_f32",)]
    for _, net, plan, sr in mids:
        _, kinds = _kinds(ctx, lambda: ctx.solve(net, plan, sr))
        assert "batch" not in kinds  # alone: per-node launches
        _, kinds = _kinds(ctx, lambda: ctx.solve_batch([net], [plan], [sr]))
        assert kinds == {"batch"}  # launched together: the shared persistent launch
    for _, net, plan, sr in bigs:
        _, kinds = _kinds(ctx, lambda: ctx.solve_batch([net], [plan], [sr]))
        assert "batch" not in kinds
    jobs = small[:3] + mids[:1] + bigs[:1] + small[3:] + mids[1:] + bigs[1:]
    alone = [ctx.solve(net, plan, sr) for _, net, plan, sr in jobs]
    mixed = ctx.solve_batch([j[1] for j in jobs], [j[2] for j in jobs], [j[3] for j in jobs])
    for a, m in zip(alone, mixed):
        assert _key(a) == _key(m)
    srv = tn.Server(ctx, 8 << 30, max_slots=16)
    ids = [srv.submit(net, plan, sr) for _, net, plan, sr in jobs]
    srv.drain()
    for jid, a in zip(ids, alone):
        assert _key(srv.poll(jid)) == _key(a)
    st = srv.stats()
    srv.close()
    assert st["launches"] >= 3  # the per-node jobs went out alone
    want140 = oracle.eliminate(nets[140][0], "counting_tropical", max_width=26)
    want150 = oracle.eliminate(nets[150][0], "tropical", max_width=26)
    assert alone[3]["size"] == want140["size"]
    assert (alone[8]["size"], alone[8]["count_mod_2_64"]) == (want140["size"], want140["count"] % 2 ** 64)
    assert alone[4]["size"] == want150["size"]


def test_wait_limit_abandons_the_launch_and_the_context_recovers(ctx):
    g = gg.random_regular(120, 3, 0)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=2, niters=5, seed=0)
    want = oracle.eliminate(g, "counting_tropical")
    ctx.set_wait_limit(1e-8)  # one tick of the wall clock: every dependency wait gives up
    with pytest.raises(tn.TnError) as ei:
        ctx.solve_batch([net, net], [plan, plan], ["counting_tropical", "tropical_i32"])
    assert ei.value.code == tn.TN_EDEVICE
    ctx.set_wait_limit(10.0)
    r = ctx.solve_batch([net, net], [plan, plan], ["counting_tropical", "tropical_i32"])
    assert (r[0]["size"], r[0]["count_mod_2_64"]) == (want["size"], want["count"] % 2 ** 64)
    assert r[1]["size"] == want["size"]
    with pytest.raises(tn.TnError):
        ctx.set_wait_limit(0.0)


def test_allocator_failure_is_reported_and_the_next_solve_succeeds():
    import torch

    torch.cuda.set_device(0)
    state = {"fail": False, "calls": 0}
    t_alloc, t_free = torch.cuda.caching_allocator_alloc, torch.cuda.caching_allocator_delete

    def _alloc(nbytes, user, stream):
        state["calls"] += 1
        if state["fail"]:
            return None
        return t_alloc(int(nbytes), 0, int(stream or 0))

    def _free(ptr, nbytes, user, stream):
        t_free(int(ptr))

    a_cb, f_cb = tn.ALLOC_FN(_alloc), tn.FREE_FN(_free)
    alloc = tn.tn_allocator(ctypes.cast(a_cb, ctypes.c_void_p), ctypes.cast(f_cb, ctypes.c_void_p), None)
    h = ctypes.c_void_p()
    tn._check(tn.lib().tn_ctx_create(0, ctypes.c_void_p(torch.cuda.current_stream(0).cuda_stream),
                                     ctypes.byref(alloc), ctypes.byref(h)))
    c = tn.Context.__new__(tn.Context)
    c._cb = (a_cb, f_cb)
    c.h = h
    tn._live.add(c)
    g = gg.random_regular(60, 3, 1)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net)
    want = oracle.eliminate(g, "count")["count"]
    state["fail"] = True
    for ex in ("stream", "persistent"):
        with pytest.raises(tn.TnError) as ei:
            c.solve(net, plan, "count_exact", executor=ex)
        assert ei.value.code == tn.TN_ENOMEM
    with pytest.raises(tn.TnError) as ei:
        tn.Server(c, 1 << 20)
    assert ei.value.code == tn.TN_ENOMEM
    state["fail"] = False
    for ex in ("stream", "persistent"):
        assert c.solve(net, plan, "count_exact", executor=ex)["count"] == want
    c.synchronize()
    c.close()
