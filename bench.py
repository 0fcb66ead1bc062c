"""Benchmark of the hot path on one MI355X.

Headline (``value``): one step = the 240-vertex 3-regular network (seed 0,
unit weights) contracted over all its slices in two algebras, tropical
float32 (SizeMax) and counting tropical (CountingMax: int32 size, uint64
count), on per-node launches.  The contraction order is TreeSA with
sc_target 30 and slicing, so the largest intermediates hold 2^30 entries.
value = 2 x 2^tc semiring ops / seconds per step (tc: the plan's total time
complexity over all slices, Sec. 4.1).  Planning is host-side and untimed;
the network's leaves are built on the device inside the step.

In the same JSON line:
  roofline       the kernel with the most device time in the timed steps
                 (HIP events around every launch, on the context stream):
                 semiring ops (or algorithmic bytes) per launch over its
                 average launch time, against the engine peak of its algebra
                 (VALU instruction rate / instructions per op, matrix cores)
                 or HBM; plus the time-weighted fraction of every launch of
                 the step against its own roofline min(P_engine, I x B)
  per_node       the step's longest launches with their bound and fraction
  tuned          the step with the committed launch-shape table and with the
                 heuristic shapes only; the same for the 120-vertex step
  k2_step        the 120-vertex network's three contractions (max-plus int32,
                 exact count, Z at x = 1) as one persistent launch
  k3             King's subgraph 24 x 24 at 0.8, weights k/2^14: tropical
                 float32 and Z(beta) for beta in {0.5, 1, 2, 4} on matrix
                 cores (float32 and bfloat16 inputs), error against the
                 oracle's extended-precision values (tests/golden/k3.json)
  batched        a job stream: plain, batched and served solves/s, p50/p99
  widened rows   polynomial, spin glass, SingleConfigMax, SizeMax(8),
                 CountingMax(4), conditioning
  cpu_baseline   the oracle's plan follower on the same network and
                 algebras (a finer-sliced plan, a bounded sample of slices,
                 one process per host core)
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import math
import multiprocessing as mp
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM = 8000e9  # bytes / s
# VALU issue, 256 CUs x 2.4 GHz: FP32 instructions 128 lanes per CU-clock
# (the published 157.3 TFLOP/s = 78.65 T lane FMAs / s); integer instructions
# (adds, three-input max, compares, selects, multiply-adds) one wave of 64
# lanes per CU-clock, 39.3 T lane instructions / s, the rate the integer
# kernels' VALU counters saturate at.
LANE_F32 = 78.65e12
LANE_INT = 256 * 2.4e9 * 64
# Fewest VALU instructions per semiring op: max-plus one add per product plus
# one three-input max per two products (1.5); counting tropical in two
# passes, 1.5 for the sizes plus add, compare, select and multiply-add for the
# counts (5.5); counts mod p a 32x32->64 multiply-add per product plus one
# Montgomery reduction (two multiplies, an add, a min) per four (2.5).
ENGINE = {"tropical_i32": LANE_INT / 1.5, "tropical_f32": LANE_F32 / 1.5, "counting_tropical": LANE_INT / 5.5,
          "count_exact": LANE_INT / 2.5,
          # the real algebra on matrix cores: one multiply-add per op;
          # 157.3 TFLOP/s float32, 2.5 PFLOP/s bfloat16 inputs (dense)
          "partition_f32": 157.3e12 / 2, "partition_bf16": 2.5e15 / 2}
ENGINE_BOUND = {"partition_f32": "mfma", "partition_bf16": "mfma"}
SR_NAME = {0: "tropical_i32", 1: "tropical_f32", 2: "counting_tropical", 3: "count_exact", 4: "partition_f32",
           5: "partition_bf16", -1: "mixed"}
TABLE = os.path.join(ROOT, "paper_2501_00227_amd", "mi355x_tiles.tune")

K5_PLAN = dict(method="treesa", ntrials=16, niters=50, rw_weight=0.5, sc_target=30, nslices=30, seed=0)
K5_STEP = ("tropical_f32", "counting_tropical")
K2_STEP = (("tropical_i32", 0.0), ("count_exact", 0.0), ("partition_f32", 0.0))
CPU_PLAN = dict(method="treesa", ntrials=4, niters=5, sc_target=16, nslices=40, seed=0)


def build_k5(seed=0):
    import graphgen as gg
    import paper_2501_00227_amd as tn

    g = gg.random_regular(240, 3, seed)
    net = tn.Net.from_graph(g)
    return g, net, tn.Plan.create(net, **K5_PLAN)


def build_k2(seed=0):
    import graphgen as gg
    import paper_2501_00227_amd as tn

    g = gg.random_regular(120, 3, seed)
    net = tn.Net.from_graph(g)
    return g, net, tn.Plan.create(net, method="treesa", ntrials=8, niters=20, seed=seed)


def build_k3(seed=0):
    import graphgen as gg
    import paper_2501_00227_amd as tn

    g = gg.kings_subgraph(24, 0.8, seed)
    g = g.with_weights(gg.dyadic_weights(g.nv, seed))
    net = tn.Net.from_graph(g)
    return g, net, tn.Plan.create(net, seed=seed)


def k5_step(ctx, net, plan):
    return [ctx.solve(net, plan, sr, executor="stream") for sr in K5_STEP]


def k2_step(ctx, net, plan):
    return ctx.solve_batch([net] * len(K2_STEP), [plan] * len(K2_STEP), [s for s, _ in K2_STEP],
                           [b for _, b in K2_STEP])


# ------------------------------------------------------------- roofline --
def launch_roofline(r):
    """One launch against its own roofline: GEMMs against min(P_engine,
    I x B_HBM), I = ops / algorithmic bytes; every other kernel against HBM."""
    t = r["ms"] * 1e-3
    sr = SR_NAME.get(r["semiring"], "mixed")
    if r["ops"] > 0 and sr in ENGINE and t > 0:
        intensity = r["ops"] / r["alg_bytes"]
        pe = ENGINE[sr]
        roof = min(pe, intensity * HBM)
        bound = ENGINE_BOUND.get(sr, "alu") if pe <= intensity * HBM else "hbm"
        return {"bound": bound, "achieved_ops": r["ops"] / t, "roof_ops": roof, "frac": r["ops"] / t / roof}
    gbs = r["alg_bytes"] / t if t > 0 else 0.0
    return {"bound": "hbm", "achieved_bytes": gbs, "frac": gbs / HBM}


def profile_traffic(kernel):
    """HBM bytes per launch of a kernel from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE scaled by a plain copy's readings), if
    the kernel sources are unchanged since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k.get("traffic_bytes_per_launch")


def kernel_source_hash():
    srcs = ["paper_2501_00227_amd/csrc/kernels.hip", "paper_2501_00227_amd/csrc/kernels_dev.h",
            "paper_2501_00227_amd/csrc/batch_kernels.hip"]
    return hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in srcs)).hexdigest()[:16]


def dominant_roofline(recs):
    """Roofline of the kernel with the most device time, and the
    time-weighted fraction of all launches against their own rooflines."""
    by = {}
    tw_num = tw_den = 0.0
    for r in recs:
        b = by.setdefault(r["kernel"] or r["kind"], {"ms": 0.0, "n": 0, "ops": 0.0, "bytes": 0.0, "sr": set()})
        b["ms"] += r["ms"]
        b["n"] += 1
        b["ops"] += r["ops"]
        b["bytes"] += r["alg_bytes"]
        b["sr"].add(SR_NAME.get(r["semiring"], "mixed"))
        lr = launch_roofline(r)
        tw_num += r["ms"] * lr["frac"]
        tw_den += r["ms"]
    name = max(by, key=lambda k: by[k]["ms"])
    b = by[name]
    avg_s = b["ms"] / b["n"] * 1e-3
    sr = sorted(b["sr"])[0]
    per_launch_ops, per_launch_bytes = b["ops"] / b["n"], b["bytes"] / b["n"]
    intensity = per_launch_ops / per_launch_bytes if per_launch_bytes else 0.0
    if per_launch_ops > 0 and sr in ENGINE and ENGINE[sr] <= intensity * HBM:
        bound, achieved, peak, unit = ENGINE_BOUND.get(sr, "alu"), per_launch_ops / avg_s / 1e12, ENGINE[sr] / 1e12, \
            "TOP/s"
    else:
        bound, achieved, peak, unit = "hbm", per_launch_bytes / avg_s / 1e9, HBM / 1e9, "GB/s"
    total_ms = sum(x["ms"] for x in by.values())
    kernels = sorted(((k, v["ms"], v["n"]) for k, v in by.items()), key=lambda x: -x[1])
    return {"bound": bound, "achieved": achieved, "peak": peak, "unit": unit, "frac": achieved / peak,
            "traffic": profile_traffic(name), "kernel": name, "semiring": sr, "launches": b["n"],
            "avg_launch_ms": b["ms"] / b["n"], "ops_per_launch": per_launch_ops,
            "alg_bytes_per_launch": per_launch_bytes, "share_of_device_time": b["ms"] / total_ms,
            "time_weighted_frac_all_launches": tw_num / tw_den,
            "device_time_by_kernel_ms": {k: round(ms, 3) for k, ms, n in kernels[:12]}}


def per_node_table(recs, top=16):
    """The step's nodes with the most device time (launches of one node,
    kernel and algebra summed over the slices), each against its roofline."""
    groups = {}
    for r in recs:
        key = (r["kernel"], r["semiring"], r["node"], tuple(r["shape"]))
        g = groups.setdefault(key, dict(r, ms=0.0, ops=0.0, alg_bytes=0.0, launches=0))
        g["ms"] += r["ms"]
        g["ops"] += r["ops"]
        g["alg_bytes"] += r["alg_bytes"]
        g["launches"] += 1
    rows = []
    for r in sorted(groups.values(), key=lambda r: -r["ms"])[:top]:
        lr = launch_roofline(r)
        row = {"kernel": r["kernel"], "semiring": SR_NAME.get(r["semiring"], "mixed"), "node": r["node"],
               "shape_log2": r["shape"], "launches": r["launches"], "ms": round(r["ms"], 3), "bound": lr["bound"],
               "frac": round(lr["frac"], 4)}
        if "achieved_ops" in lr:
            row["TOP_per_s"] = round(lr["achieved_ops"] / 1e12, 3)
            row["roof_TOP_per_s"] = round(lr["roof_ops"] / 1e12, 3)
        else:
            row["GB_per_s"] = round(lr["achieved_bytes"] / 1e9, 1)
        rows.append(row)
    return rows


# ------------------------------------------------------------ measurement --
def timed_steps(step, steps, warmup, ctx, profile=True):
    import torch

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.synchronize()
    if profile:
        ctx.profile(clear=True)
        ctx.set_profiling(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
    ctx.synchronize()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    recs = []
    if profile:
        recs = ctx.profile(clear=True)
        ctx.set_profiling(False)
    return dt, res, recs


def tuned_vs_heuristic(ctx, step, reps=1):
    import paper_2501_00227_amd as tn

    out = {}
    for mode in ("heuristic", "tuned"):
        tn.tune_clear()
        if mode == "tuned" and os.path.exists(TABLE):
            tn.tune_load(TABLE)
        step()
        ctx.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            step()
        ctx.synchronize()
        out[mode + "_ms"] = (time.perf_counter() - t0) / reps * 1e3
    return out


def k3_record(ctx):
    """King's subgraph 24 x 24 at 0.8: tropical f32 and Z(beta) on matrix
    cores against the oracle's stored values, with the Z nodes' rooflines."""
    g, net, plan = build_k3(0)
    gold = next(c for c in json.load(open(os.path.join(ROOT, "tests", "golden", "k3.json")))["cases"]
                if c["seed"] == 0)
    tc, sc, rwc = plan.complexity()
    out = {"workload": "King's subgraph 24x24 p=0.8 seed 0 (%d vertices, %d edges), weights k/2^14" % (g.nv, g.ne),
           "tc_log2": tc, "sc_log2": sc}
    ctx.solve(net, plan, "tropical_f32")
    t0 = time.perf_counter()
    r = ctx.solve(net, plan, "tropical_f32")
    out["tropical_f32"] = {"ms": (time.perf_counter() - t0) * 1e3, "size": r["size"],
                           "exact": r["size"] == gold["size_max"]}
    out["partition"] = []
    for beta, want in gold["log_z"].items():
        row = {"beta": float(beta)}
        for sr in ("partition_f32", "partition_bf16"):
            ctx.solve(net, plan, sr, beta=float(beta))
            t0 = time.perf_counter()
            r = ctx.solve(net, plan, sr, beta=float(beta))
            dt = time.perf_counter() - t0
            # the node records from a separate solve: events on every launch
            # would lengthen the timed one (some 5000 launches)
            ctx.set_profiling(True)
            ctx.solve(net, plan, sr, beta=float(beta))
            recs = ctx.profile(clear=True)
            ctx.set_profiling(False)
            mf = [x for x in recs if x["kind"] == "gemm_mfma"]
            key = sr.split("_")[1]
            row[key] = {"ms": dt * 1e3, "log_z": r["log_z"], "abs_err_log_z": abs(r["log_z"] - want),
                        "rel_err_z": abs(math.expm1(r["log_z"] - want)), "GOP_per_s": 2.0 ** tc / dt / 1e9,
                        "z_range_log2": r["z_range_log2"]}
            if mf:
                big = max(mf, key=lambda x: x["ops"])
                lr = launch_roofline(big)
                row[key]["largest_mfma_node"] = {"shape_log2": big["shape"], "ms": big["ms"],
                                                 "TFLOP_per_s": 2 * big["ops"] / big["ms"] / 1e9,
                                                 "bound": lr["bound"], "frac": lr["frac"]}
                row[key]["mfma_share_of_device_time"] = sum(x["ms"] for x in mf) / sum(x["ms"] for x in recs)
        out["partition"].append(row)
    out["fp32_max_rel_err_z"] = max(x["f32"]["rel_err_z"] for x in out["partition"])
    out["bf16_max_rel_err_z"] = max(x["bf16"]["rel_err_z"] for x in out["partition"])
    return out


def k1_graphs():
    import graphgen as gg

    gold = json.load(open(os.path.join(ROOT, "tests", "golden", "k1.json")))["cases"]
    return [gg.random_regular(20, 3, c["seed"]) for c in gold], gold


def k1_record(ctx, reps=20):
    """Twenty 3-regular 20-vertex graphs (seeds 0..19), counting tropical:
    solves per second one at a time (both executors) and as one batch, every
    result against the oracle's stored values.  Intermediates of a few KB:
    launch latency, not a roofline, sets the rate."""
    import paper_2501_00227_amd as tn

    graphs, gold = k1_graphs()
    nets = [tn.Net.from_graph(g) for g in graphs]
    plans = [tn.Plan.create(n, seed=c["seed"]) for n, c in zip(nets, gold)]
    want = [(c["size_max"], c["count_max"]) for c in gold]
    out = {"workload": "K1: 3-regular n=20 seeds 0..19, unit weights, counting tropical (int32 size, uint64 count), "
                       "greedy plans", "jobs": len(nets),
           "sc_log2_max": max(p.complexity()[1] for p in plans)}

    def check(rs):
        return all((r["size"], r["count_mod_2_64"]) == w for r, w in zip(rs, want))

    for ex in ("stream", "persistent"):
        one = lambda: [ctx.solve(n, p, "counting_tropical", executor=ex) for n, p in zip(nets, plans)]  # noqa: E731
        ok = check(one())
        t0 = time.perf_counter()
        for _ in range(reps):
            ok = check(one()) and ok
        dt = time.perf_counter() - t0
        out["one_at_a_time_" + ex] = {"solves_per_s": reps * len(nets) / dt, "exact": ok}
    batch = lambda: ctx.solve_batch(nets, plans, "counting_tropical")  # noqa: E731
    ok = check(batch())
    t0 = time.perf_counter()
    for _ in range(reps):
        ok = check(batch()) and ok
    dt = time.perf_counter() - t0
    out["batched"] = {"solves_per_s": reps * len(nets) / dt, "exact": ok, "launches_per_batch": 1}
    return out


# ---------------------------------------------------------- cpu baseline --
def _o3_slice(args):
    import graphgen as gg
    import oracle

    tree, s = args
    g = gg.random_regular(240, 3, 0)
    t0 = time.perf_counter()
    a = oracle.follow_plan(g, tree, "tropical", slices=(s, s + 1))
    b = oracle.follow_plan(g, tree, "counting_tropical", slices=(s, s + 1))
    return time.perf_counter() - t0, a, b


def cpu_baseline():
    """The oracle's plan follower (O3) on the headline network and algebras:
    the same graph planned to 2^16-entry intermediates, one slice per host
    core, tropical then counting tropical, all cores in parallel."""
    import graphgen as gg
    import paper_2501_00227_amd as tn

    g = gg.random_regular(240, 3, 0)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, **CPU_PLAN)
    info = plan.info()
    tree = plan.export()
    tc_slice = info["tc_log2"] - info["nsliced"]
    cores = min(16, len(os.sched_getaffinity(0)))
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_o3_slice, [(tree, s) for s in range(cores)])
    wall = time.perf_counter() - t0
    ops = cores * 2 * 2.0 ** tc_slice
    # beside K1: the oracle's brute force over all 2^20 subsets, one core
    import oracle

    graphs, _ = k1_graphs()
    t1 = time.perf_counter()
    for g1 in graphs:
        oracle.brute_force(g1)
    k1 = {"solves_per_s": len(graphs) / (time.perf_counter() - t1), "cores": 1,
          "sample": "the twenty K1 graphs (3-regular n=20), brute force over all 2^20 subsets"}
    return {"value": ops / wall / 1e9, "unit": "GOP/s", "cores": cores, "kind": "oracle",
            "sample": "3-regular n=240 seed 0 (the headline network), tropical + counting tropical by the oracle's plan "
                      "follower on a TreeSA plan sliced to 2^%d-entry intermediates (%d slices of 2^%.2f ops each): "
                      "slices 0..%d, one process per core" % (info["max_rank"], 1 << info["nsliced"], tc_slice,
                                                              cores - 1),
            "seconds": wall, "per_slice_seconds_mean": sum(r[0] for r in res) / len(res),
            "nproc": os.cpu_count(), "cpu_model": model, "k1_brute_force": k1}


def independence_polynomial(ctx, net, plan, tc):
    """The n=120 network's independence polynomial (finite-field method): one
    max-plus and one exact-count contraction, then (alpha + 1) x (#primes)
    mod-p evaluations in persistent launches, interpolation and CRT."""
    p = ctx.solve_polynomial(net, plan)  # warm (device programs, scratch)
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        p = ctx.solve_polynomial(net, plan)
    dt = (time.perf_counter() - t0) / reps
    # the library's choice: CRT primes (between 2^29 and 2^30) until 29 bits
    # per prime cover the total count's bits + 1 (at least two), plus one
    # check prime; the first two contractions are one max-plus pass and the
    # exact count (3 + 1 primes for this network's count bound)
    nprimes = max(2, -(-(sum(p).bit_length() + 1) // 29)) + 1
    passes = 1 + 4 + len(p) * nprimes
    return {"workload": "3-regular n=120 seed 0: independence polynomial, Sec. 6.2 finite-field method",
            "seconds": dt, "degree": len(p) - 1, "evaluation_passes": passes,
            "GOP_per_s": passes * 2.0 ** tc / dt / 1e9, "max_coefficient_bits": max(c.bit_length() for c in p)}


def single_config(ctx, net, plan):
    """One maximum independent set of the n=120 network (SingleConfigMax):
    one float32 max-plus pass kept on the device, then the back-trace
    kernel; and SizeMax(k)/CountingMax(k) at k = 4 (read off the
    independence polynomial)."""
    r = ctx.solve_single_config_max(net, plan)  # warm
    t0 = time.perf_counter()
    reps = 20
    for _ in range(reps):
        r = ctx.solve_single_config_max(net, plan)
    dt = (time.perf_counter() - t0) / reps
    mk = ctx.solve_max_k(net, plan, 4)
    return {"workload": "3-regular n=120 seed 0: one maximum independent set (Sec. 5 SingleConfigMax)",
            "ms": dt * 1e3, "value": r["value"], "set_size": sum(r["config"]),
            "size_max_4": mk["size_max_k"], "counting_max_4": {str(k): v for k, v in mk["counting_max_k"].items()}}


def size_max_8_weighted(ctx, g, plan, tc):
    """SizeMax(8) of the n=120 network with weights k/2^14 (Sec. 5 table, any
    weights): max-plus over sorted eight-lists, as one persistent launch and
    as per-node launches."""
    import graphgen as gg
    import paper_2501_00227_amd as tn

    net = tn.Net.from_graph(g.with_weights(gg.dyadic_weights(g.nv, 0)))
    out = {"workload": "3-regular n=120 seed 0, weights k/2^14: SizeMax(8) (eight-list max-plus)"}
    for ex in ("persistent", "stream"):
        top = ctx.solve_size_max_k(net, plan, 8, ex)  # warm
        t0 = time.perf_counter()
        reps = 20
        for _ in range(reps):
            top = ctx.solve_size_max_k(net, plan, 8, ex)
        dt = (time.perf_counter() - t0) / reps
        out[ex] = {"ms": dt * 1e3, "GOP_per_s": 2.0 ** tc / dt / 1e9}
        out["size_max_8"] = top
    return out


def counting_max_4(ctx, net, plan, tc):
    """CountingMax(4) of the n=120 network in one contraction over truncated
    polynomials (one persistent launch and per-node launches), against the
    same counts read off the independence polynomial."""
    out = {"workload": "3-regular n=120 seed 0: CountingMax(4) (truncated-polynomial algebra)"}
    for ex in ("persistent", "stream"):
        r = ctx.solve_counting_max_k(net, plan, 4, ex)  # warm
        t0 = time.perf_counter()
        reps = 20
        for _ in range(reps):
            r = ctx.solve_counting_max_k(net, plan, 4, ex)
        dt = (time.perf_counter() - t0) / reps
        out[ex] = {"ms": dt * 1e3, "GOP_per_s": 2.0 ** tc / dt / 1e9}
    via_poly = ctx.solve_max_k(net, plan, 4)["counting_max_k"]
    out.update({"top": r["top"], "counts": {str(k): v for k, v in r["counts"].items()},
                "equals_polynomial_path": r["counts"] == {k: v % 2 ** 64 for k, v in via_poly.items()}})
    return out


def conditioned_batch(ctx, g, plan, nfix=8, njobs=64, seed=0):
    """Conditioning: njobs copies of the network, each with nfix random
    vertices fixed, counted (counting tropical) in one persistent launch."""
    import random

    import paper_2501_00227_amd as tn

    base = tn.Net.from_graph(g)
    rng = random.Random(seed)
    adj = g.adjacency()
    nets = []
    for _ in range(njobs):
        fixed = {}
        for v in rng.sample(range(g.nv), nfix):
            fixed[v] = 0 if any(fixed.get(u) == 1 for u in adj[v]) else rng.randint(0, 1)
        nets.append(base.condition(fixed))
    ctx.solve_batch(nets, [plan] * njobs, "counting_tropical")  # warm
    t0 = time.perf_counter()
    reps = 5
    for _ in range(reps):
        ctx.solve_batch(nets, [plan] * njobs, "counting_tropical")
    dt = (time.perf_counter() - t0) / reps
    return {"workload": "3-regular n=120 seed 0: %d conditionings (%d fixed vertices each), counting tropical, "
                        "one persistent launch" % (njobs, nfix), "ms": dt * 1e3, "solves_per_s": njobs / dt}


def buckyball(ctx):
    """The Sec. 6.4 example: antiferromagnetic unit-coupling spin glass on
    the C60 graph, ln Z / N at beta = 1 (float32 on matrix cores) and the
    ground-state energy and degeneracy (counting tropical)."""
    import graphgen as gg
    import paper_2501_00227_amd as tn

    g = gg.fullerene()
    net = tn.Net.spin_glass(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=4, niters=10, seed=0)
    out = {"workload": "C60 spin glass, J = 1, h = 0 (Sec. 6.4)", "tc_log2": plan.complexity()[0]}
    for sr, beta in (("partition_f32", 1.0), ("counting_tropical", 0.0)):
        ctx.solve(net, plan, sr, beta=beta)
        t0 = time.perf_counter()
        for _ in range(20):
            r = ctx.solve(net, plan, sr, beta=beta)
        out[sr + "_ms"] = (time.perf_counter() - t0) / 20 * 1e3
        if sr == "partition_f32":
            out["log_z_per_vertex"] = r["log_z"] / g.nv
        else:
            out["ground_state"] = [-r["size"], r["count_mod_2_64"]]
    return out


K4_N = (40, 200)
K4_BUDGET = 2 << 30


def k4_expected(njobs, seed):
    """Expected results of the served jobs with n <= 130 among the first
    stored ones (the oracle's elimination, stored by
    tests/golden/make_golden_k4.py for the first 2000 jobs of the stream), or
    None when the stream does not start with the stored one."""
    path = os.path.join(ROOT, "tests", "golden", "k4_jobs.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    # job_mix draws job after job, so a longer stream starts with the stored one
    if rec["njobs"] > njobs or rec["seed"] != seed or rec["n_range"] != list(K4_N):
        return None
    out = {}
    for k, v in rec["expected"].items():
        if v is None:
            continue
        out[int(k)] = [v[0], int(v[1])] if isinstance(v, list) else v
    return out


def _k4_matches(sr, r, want):
    if sr == "tropical_i32":
        return r["size"] == want
    if sr == "counting_tropical":
        return [r["size"], r["count_mod_2_64"]] == want
    return abs(r["log_z"] - want) <= 1e-5


def job_stream(ctx, njobs, seed=0, expected=None):
    """The served workload: 3-regular jobs with n uniform over even values in
    [40, 200], algebra uniform over tropical int32, counting tropical and
    float32 Z at x = 1; jobs above the 2 GiB device budget are refused
    (TN_ETOOBIG) and counted.  Plain one-at-a-time, batched (persistent
    launches of 256 jobs) and served (Poisson arrivals at 0.5, 1, 2 and 4 x
    the plain rate, p50/p99 latency submit -> result on the host), every job
    with n <= 130 among the first 2000 checked against the oracle's stored
    values."""
    import numpy as np

    import graphgen as gg
    import paper_2501_00227_amd as tn

    mix = gg.job_mix(njobs, seed, *K4_N)

    def mk(j):
        n, gseed, sr = j
        net = tn.Net.from_graph(gg.random_regular(n, 3, gseed))
        return net, tn.Plan.create(net, seed=gseed), sr

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(8) as ex:
        jobs = list(ex.map(mk, mix))
    plan_s = time.perf_counter() - t0
    # the jobs that fit the budget (the server refuses the others)
    keep = [k for k, (net, plan, sr) in enumerate(jobs) if tn.server_job_bytes(net, plan, sr) <= K4_BUDGET]
    res = {"workload": "K4: %d 3-regular jobs, n uniform over even values in [%d, %d], algebra uniform over tropical "
                       "int32 / counting tropical / Z(x=1) fp32, device budget %d GiB" %
                       (njobs, K4_N[0], K4_N[1], K4_BUDGET >> 30),
           "jobs": njobs, "admissible": len(keep), "planning_seconds_8_threads": plan_s,
           "largest_admissible_n": max(mix[k][0] for k in keep)}
    mism = 0
    checked = 0

    def check(k, r):
        nonlocal mism, checked
        if expected is not None and k in expected:
            checked += 1
            if not _k4_matches(mix[k][2], r, expected[k]):
                mism += 1

    # one at a time (a sample of the admissible jobs), each tn_solve synchronous
    sample = keep[: min(300, len(keep))]
    for k in sample[:20]:
        ctx.solve(*jobs[k])
    t0 = time.perf_counter()
    for k in sample:
        ctx.solve(*jobs[k])
    plain = len(sample) / (time.perf_counter() - t0)
    res["plain_solves_per_s"] = plain
    # batched: persistent launches of 256 jobs
    t0 = time.perf_counter()
    for q in range(0, len(keep), 256):
        chunk = keep[q:q + 256]
        out = ctx.solve_batch([jobs[k][0] for k in chunk], [jobs[k][1] for k in chunk], [jobs[k][2] for k in chunk])
        for k, r in zip(chunk, out):
            check(k, r)
    res["batched_solves_per_s"] = len(keep) / (time.perf_counter() - t0)
    # served: Poisson arrivals at 0.5, 1, 2 and 4 x the one-at-a-time rate;
    # every job is submitted, the ones above the budget are refused
    res["served"] = []
    for mult in (0.5, 1.0, 2.0, 4.0):
        rate = mult * plain
        arrivals = gg.poisson_arrivals(njobs, rate, seed + 1)
        srv = tn.Server(ctx, K4_BUDGET, max_slots=512)
        ids = [None] * njobs
        t_start = time.perf_counter()

        def producer():
            for i, (net, plan, sr) in enumerate(jobs):
                dt = arrivals[i] - (time.perf_counter() - t_start)
                if dt > 0:
                    time.sleep(dt)
                try:
                    ids[i] = srv.submit(net, plan, sr)
                except tn.TnError as e:
                    if e.code != tn.TN_ETOOBIG:
                        raise

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        srv.drain()
        t_end = time.perf_counter()
        lat = []
        for k, jid in enumerate(ids):
            if jid is None:
                continue
            r = srv.poll(jid)
            lat.append(r["latency_s"])
            if mult == 1.0:
                check(k, r)
        lat = np.array(lat)
        st = srv.stats()
        srv.close()
        res["served"].append({"arrival_rate_per_s": rate, "rate_over_plain": mult,
                              "solves_per_s": len(lat) / (t_end - t_start),
                              "p50_ms": float(np.percentile(lat, 50) * 1e3),
                              "p99_ms": float(np.percentile(lat, 99) * 1e3),
                              "launches": st["launches"], "peak_running": st["peak_running"],
                              "peak_inflight": st["peak_inflight"], "rejected": st["rejected"],
                              "requeued": st["requeued"], "peak_admitted_bytes": st["peak_admitted_bytes"],
                              "peak_pool_bytes": st["peak_pool_bytes"], "budget_bytes": K4_BUDGET})
    res["oracle_checked"] = checked
    res["oracle_mismatches"] = mism
    res["oracle_stored_jobs"] = len(expected) if expected else 0
    return res


def tune_workloads(ctx, path):
    """Tune the launch shapes of the benchmark workloads' large nodes and
    write the table (the committed table is made this way)."""
    import paper_2501_00227_amd as tn

    tn.tune_clear()
    _, _, p5 = build_k5()
    _, _, p2 = build_k2()
    _, _, p3 = build_k3()
    work = [(p5, "tropical_f32", 28), (p5, "counting_tropical", 28),
            (p2, "tropical_i32", 16), (p2, "count_exact", 16), (p2, "partition_f32", 16),
            (p3, "tropical_f32", 20), (p3, "partition_f32", 20), (p3, "partition_bf16", 20)]
    for plan, sr, lo in work:
        t0 = time.perf_counter()
        n = ctx.tune_plan(plan, sr, min_log2_ops=lo, reps=2)
        print(json.dumps({"tuned": sr, "min_log2_ops": lo, "keys": n, "seconds": time.perf_counter() - t0}),
              flush=True)
    n = tn.tune_save(path)
    recs = tn.tune_records()
    print(json.dumps({"table": path, "entries": n, "records": recs}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--jobs", type=int, default=10000, help="jobs in the batched / served stream")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline step only")
    ap.add_argument("--heuristic", action="store_true", help="heuristic launch shapes only (no tuning table)")
    ap.add_argument("--tune-out", help="tune the workloads' large nodes, write the table to this path, exit")
    ap.add_argument("--widened", action="store_true",
                    help="only the polynomial, spin-glass, maximum-configuration, SizeMax(8), CountingMax(4) and "
                         "conditioning lines")
    ap.add_argument("--k3", action="store_true", help="only the King's-subgraph partition-function line")
    ap.add_argument("--k2", action="store_true", help="only the 120-vertex persistent step")
    ap.add_argument("--k4", action="store_true", help="only the served workload")
    ap.add_argument("--k1", action="store_true", help="only the twenty 20-vertex graphs")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 256 MiB device copy (for scaling hardware byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: several GPUs would share slices and jobs with one final "
              "(+)-reduction of a scalar root, which is not implemented; use --gpus 1", file=sys.stderr)
        sys.exit(2)
    # the oracle runs first, in forked processes, before anything touches the GPU
    cpu = None
    only = args.tune_out or args.widened or args.calibrate_copy or args.k3 or args.k2 or args.k4 or args.k1
    if not (args.no_cpu or only):
        cpu = cpu_baseline()

    import torch
    import paper_2501_00227_amd as tn

    torch.cuda.set_device(0)
    if args.calibrate_copy:
        x = torch.empty(64 << 20, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        for _ in range(3):
            y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4, "copies": 3}))
        return
    ctx = tn.Context(0)
    if args.tune_out:
        tune_workloads(ctx, args.tune_out)
        return
    tn.tune_clear()
    if not args.heuristic and os.path.exists(TABLE):
        tn.tune_load(TABLE)
    if args.k3:
        print(json.dumps({"k3": k3_record(ctx)}))
        return
    if args.k1:
        print(json.dumps({"k1": k1_record(ctx)}))
        return
    if args.k4:
        print(json.dumps({"batched": job_stream(ctx, args.jobs, args.seed, k4_expected(args.jobs, args.seed))}))
        return
    if args.k2:
        g2, net2, plan2 = build_k2(args.seed)
        tc2 = plan2.complexity()[0]
        dt2, _, _ = timed_steps(lambda: k2_step(ctx, net2, plan2), args.steps, args.warmup, ctx, profile=False)
        dtp, res2, recs2 = timed_steps(lambda: k2_step(ctx, net2, plan2), args.steps, 0, ctx)
        print(json.dumps({"k2_step": {"ms_per_step": dt2 * 1e3, "ms_per_step_profiled": dtp * 1e3,
                                      "GOP_per_s": len(K2_STEP) * 2.0 ** tc2 / dt2 / 1e9,
                                      "roofline": dominant_roofline(recs2)}}))
        return
    if args.widened:
        g, net, plan = build_k2(args.seed)
        tc = plan.complexity()[0]
        print(json.dumps({"independence_polynomial": independence_polynomial(ctx, net, plan, tc),
                          "spin_glass_buckyball": buckyball(ctx), "single_config_max": single_config(ctx, net, plan),
                          "size_max_8_weighted": size_max_8_weighted(ctx, g, plan, tc),
                          "counting_max_4": counting_max_4(ctx, net, plan, tc),
                          "conditioned": conditioned_batch(ctx, g, plan)}))
        return

    g5, net5, plan5 = build_k5(args.seed)
    info5 = plan5.info()
    tc5, sc5, rwc5 = plan5.complexity()
    step5 = lambda: k5_step(ctx, net5, plan5)  # noqa: E731
    dt, res, recs = timed_steps(step5, args.steps, args.warmup, ctx)
    ops_per_step = len(K5_STEP) * 2.0 ** tc5
    per_step = len(recs) // max(args.steps, 1)
    roof = dominant_roofline(recs)
    out = {
        "metric": "semiring GOP/s & % roofline at largest intermediate; batched solves/s + p50/p99",
        "value": ops_per_step / dt / 1e9,
        "unit": "GOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+i32+u64",
        "data": "synthetic",
        "config": {"workload": "K5: 3-regular n=240 seed %d, unit weights; tropical float32 + counting tropical "
                               "(int32 size, uint64 count), each over all %d slices of a TreeSA plan with sc_target 30 "
                               "(largest intermediate 2^%d entries), per-node launches" %
                               (args.seed, 1 << info5["nsliced"], info5["max_rank"]),
                   "tc_log2": tc5, "sc_log2": sc5, "rwc_log2": rwc5, "nsliced": info5["nsliced"],
                   "launch_shapes": "heuristic" if args.heuristic or not os.path.exists(TABLE)
                   else "tuned table " + os.path.relpath(TABLE, ROOT)},
        "roofline": roof,
        "per_node": per_node_table(recs[-per_step:]),
        "results": {"size_max": res[0]["size"], "counting_max": [res[1]["size"], res[1]["count_mod_2_64"]],
                    "seconds_per_algebra": [r["seconds"] for r in res]},
    }
    if not args.quick:
        g2, net2, plan2 = build_k2(args.seed)
        tc2, sc2, rwc2 = plan2.complexity()
        step2 = lambda: k2_step(ctx, net2, plan2)  # noqa: E731
        if not args.heuristic and os.path.exists(TABLE):
            out["tuned"] = {"table": os.path.relpath(TABLE, ROOT),
                            "k5_step": tuned_vs_heuristic(ctx, step5),
                            "k2_step": tuned_vs_heuristic(ctx, step2, reps=200)}
        # wall time per step without profiling (HIP events on every launch
        # cost more than this step's device time), then the launch's
        # roofline from a profiled run
        dt2, res2, _ = timed_steps(step2, 1000, 200, ctx, profile=False)
        dtp, _, recs2 = timed_steps(step2, 200, 20, ctx)
        out["k2_step"] = {"workload": "3-regular n=120 seed %d, unit weights: tropical int32 + exact count (3 + 1 "
                                      "primes below 2^30, CRT) + Z(x=1) fp32, one persistent launch per step" % args.seed,
                          "tc_log2": tc2, "sc_log2": sc2, "ms_per_step": dt2 * 1e3, "ms_per_step_profiled": dtp * 1e3,
                          "GOP_per_s": len(K2_STEP) * 2.0 ** tc2 / dt2 / 1e9, "roofline": dominant_roofline(recs2),
                          "results": {"size_max": res2[0]["size"], "count_all": str(res2[1]["count"]),
                                      "log_z": res2[2]["log_z"]}}
        out["k3"] = k3_record(ctx)
        out["k1"] = k1_record(ctx)
        g, net, plan = g2, net2, plan2
        out["independence_polynomial"] = independence_polynomial(ctx, net, plan, tc2)
        out["spin_glass_buckyball"] = buckyball(ctx)
        out["single_config_max"] = single_config(ctx, net, plan)
        out["size_max_8_weighted"] = size_max_8_weighted(ctx, g, plan, tc2)
        out["counting_max_4"] = counting_max_4(ctx, net, plan, tc2)
        out["conditioned"] = conditioned_batch(ctx, g, plan)
        out["batched"] = job_stream(ctx, args.jobs, args.seed, k4_expected(args.jobs, args.seed))
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out))


if __name__ == "__main__":
    main()
