"""Benchmark of the hot path on one MI355X.

Headline (``value``): one step = the three contractions of the seeded
3-regular n=120 network (unit weights, TreeSA order), run as one persistent
launch: max independent-set size (int32 max-plus), exact independent-set
count (residues mod primes below 2^30, as many as a bound on the count
needs (3 at n = 120), + a check prime, CRT) and the
partition function at x = 1 (float32, per-tensor power-of-two exponents).
Leaf data and plan tables are resident on the device before timing; planning
is host-side and untimed.  value = 3 x 2^tc semiring ops / seconds per step,
tc the plan's time complexity (Sec. 4.1).

Also reported in the same JSON line:
  roofline              the dominant kernel of the timed step (HIP events on
                        the context stream), algorithmic bytes per launch over
                        its average launch duration, against HBM peak
  largest_intermediate  one slice of the 240-vertex 3-regular network planned
                        to a largest intermediate of 2^30 entries: the GEMM
                        node with the most semiring ops and the largest permute,
                        against the VALU peak of their algebra / HBM peak
  batched / served      a stream of 3-regular jobs (n even in [40, 120],
                        algebra uniform over tropical int32, counting tropical,
                        float32 partition function): one-at-a-time, batched
                        (persistent launches of 256 jobs) and served
                        (Poisson arrivals at 0.5, 1, 2 and 4 x the one-at-a-time
                        rate; p50/p99 latency submit -> result on the host)
  cpu_baseline          the CPU oracle producing the step's three results
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import threading
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_GBS = 8000.0
# VALU peak from the published FP32 vector rate: 157.3 TFLOP/s = 78.6 T lane
# FMAs / s, i.e. 78.6 T 32-bit lane instructions / s (256 CUs x 2.4 GHz x 128
# lanes per clock).
LANE_TOPS = 157.3 / 2.0
# Fewest VALU instructions one semiring op can take on gfx950: max-plus is one
# add per product plus one three-input max per two products; counting
# tropical is a saturating add, a 64-bit product (one 32x32->64 multiply-add,
# two 32-bit multiplies, one three-input add), two compares, four selects, a
# 64-bit add and a max.
INSTR_PER_OP = {"tropical_i32": 1.5, "tropical_f32": 1.5, "counting_tropical": 13.0}
SR_NAME = {0: "tropical_i32", 1: "tropical_f32", 2: "counting_tropical", 3: "count_exact", 4: "partition_f32",
           5: "partition_bf16", -1: "mixed"}
MFMA_F32_TFLOPS = 157.3

STEP = (("tropical_i32", 0.0), ("count_exact", 0.0), ("partition_f32", 0.0))


def build_k2(seed):
    import graphgen as gg
    import paper_2501_00227_amd as tn

    g = gg.random_regular(120, 3, seed)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=8, niters=20, seed=seed)
    return g, net, plan


def run_step(ctx, net, plan, executor="persistent"):
    """The three contractions of one step: one persistent launch, or (for
    comparison) per-node stream launches, one contraction after the other."""
    if executor == "stream":
        return [ctx.solve(net, plan, s, beta=b, executor="stream") for s, b in STEP]
    return ctx.solve_batch([net] * len(STEP), [plan] * len(STEP), [s for s, _ in STEP], [b for _, b in STEP])


def measured_traffic():
    """HBM bytes per launch of the persistent kernel from the committed
    rocprofv3 FETCH_SIZE / WRITE_SIZE runs, if the kernel is unchanged since."""
    import hashlib

    path = os.path.join(ROOT, "profiles", "k2_step_persistent_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    srcs = ["paper_2501_00227_amd/csrc/batch_kernels.hip", "paper_2501_00227_amd/csrc/kernels_dev.h"]
    h = hashlib.sha256(b"".join(open(os.path.join(ROOT, f), "rb").read() for f in srcs)).hexdigest()[:16]
    if h != rec.get("kernel_source_sha256_16"):
        return None
    return rec["batch_kernel"]["traffic_bytes_per_launch"]


def group(recs):
    groups = {}
    for r in recs:
        key = (r["kind"], r["semiring"])
        g = groups.setdefault(key, {"ms": 0.0, "n": 0, "ops": 0.0, "bytes": 0.0})
        g["ms"] += r["ms"]
        g["n"] += 1
        g["ops"] += r["ops"]
        g["bytes"] += r["alg_bytes"]
    return groups


def cpu_baseline(g, ops_per_step):
    import oracle

    t0 = time.perf_counter()
    oracle.eliminate(g, "tropical")
    oracle.eliminate(g, "count")
    oracle.eliminate(g, "partition", 0.0)
    dt = time.perf_counter() - t0
    return {"value": ops_per_step / dt / 1e9, "unit": "GOP/s", "cores": 1, "kind": "oracle",
            "sample": "one full step (the same three results) by the oracle's variable elimination, "
                      "single-threaded; work counted as the GPU plan's 3 x 2^tc semiring ops",
            "seconds": dt}


def largest_intermediate(ctx):
    """One slice of the n=240 network planned to sc = 30, per-node timings."""
    import graphgen as gg
    import paper_2501_00227_amd as tn

    g = gg.random_regular(240, 3, 0)
    net = tn.Net.from_graph(g)
    plan = tn.Plan.create(net, method="treesa", ntrials=8, niters=10, sc_target=30, nslices=30, seed=0)
    tc, sc, rwc = plan.complexity()
    info = plan.info()
    out = {"workload": "3-regular n=240 seed 0, TreeSA sc_target 30: slice 0 of %d" % (1 << info["nsliced"]),
           "tc_log2_per_slice": tc - info["nsliced"], "sc_log2": sc, "nsliced": info["nsliced"]}
    for sr in ("tropical_f32", "counting_tropical"):
        ctx.solve(net, plan, sr, slices=(0, 1))  # warm
        ctx.set_profiling(True)
        t0 = time.perf_counter()
        ctx.solve(net, plan, sr, slices=(0, 1))
        dt = time.perf_counter() - t0
        recs = ctx.profile()
        ctx.set_profiling(False)
        gem = max((r for r in recs if r["kind"].startswith("gemm")), key=lambda r: r["ops"])
        perm = max((r for r in recs if r["kind"] == "permute"), key=lambda r: r["alg_bytes"])
        peak = LANE_TOPS / INSTR_PER_OP[sr]
        tops = gem["ops"] / gem["ms"] / 1e9
        gbs = perm["alg_bytes"] / perm["ms"] / 1e6
        out[sr] = {
            "slice_seconds": dt,
            "slice_GOPs": 2.0 ** (tc - info["nsliced"]) / dt / 1e9,
            "largest_gemm": {"shape_log2_bikj": gem["shape"], "ms": gem["ms"], "achieved": tops, "unit": "TOP/s",
                             "peak": peak, "bound": "alu", "frac": tops / peak},
            "largest_permute": {"rank": perm["shape"][0], "ms": perm["ms"], "achieved": gbs, "unit": "GB/s",
                                "peak": HBM_GBS, "bound": "hbm", "frac": gbs / HBM_GBS},
        }
    return out


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


def job_stream(ctx, njobs, seed=0):
    """Batched and served throughput on a stream of small 3-regular jobs."""
    import numpy as np

    import graphgen as gg
    import paper_2501_00227_amd as tn

    mix = gg.job_mix(njobs, seed, 40, 120)

    def mk(j):
        n, gseed, sr = j
        net = tn.Net.from_graph(gg.random_regular(n, 3, gseed))
        return net, tn.Plan.create(net, seed=gseed), sr

    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(8) as ex:
        jobs = list(ex.map(mk, mix))
    plan_s = time.perf_counter() - t0
    res = {"jobs": njobs, "n_range": [40, 120], "planning_seconds_8_threads": plan_s}
    # one at a time (a sample), each tn_solve synchronous
    sample = jobs[: min(300, njobs)]
    for net, plan, sr in sample[:20]:
        ctx.solve(net, plan, sr)
    t0 = time.perf_counter()
    for net, plan, sr in sample:
        ctx.solve(net, plan, sr)
    plain = len(sample) / (time.perf_counter() - t0)
    res["plain_solves_per_s"] = plain
    # batched: persistent launches of 256 jobs
    t0 = time.perf_counter()
    for k in range(0, njobs, 256):
        chunk = jobs[k:k + 256]
        ctx.solve_batch([c[0] for c in chunk], [c[1] for c in chunk], [c[2] for c in chunk])
    res["batched_solves_per_s"] = njobs / (time.perf_counter() - t0)
    # served: Poisson arrivals at 0.5, 1, 2 and 4 x the one-at-a-time rate
    res["served"] = []
    for mult in (0.5, 1.0, 2.0, 4.0):
        rate = mult * plain
        arrivals = gg.poisson_arrivals(njobs, rate, seed + 1)
        srv = tn.Server(ctx, 16 << 30, max_slots=512)
        ids = [None] * njobs
        t_start = time.perf_counter()

        def producer():
            for i, (net, plan, sr) in enumerate(jobs):
                dt = arrivals[i] - (time.perf_counter() - t_start)
                if dt > 0:
                    time.sleep(dt)
                ids[i] = srv.submit(net, plan, sr)

        th = threading.Thread(target=producer)
        th.start()
        th.join()
        srv.drain()
        t_end = time.perf_counter()
        lat = np.array([srv.poll(i)["latency_s"] for i in ids])
        st = srv.stats()
        srv.close()
        res["served"].append({"arrival_rate_per_s": rate, "rate_over_plain": mult,
                              "solves_per_s": njobs / (t_end - t_start),
                              "p50_ms": float(np.percentile(lat, 50) * 1e3),
                              "p99_ms": float(np.percentile(lat, 99) * 1e3),
                              "launches": st["launches"], "peak_running": st["peak_running"],
                              "peak_admitted_bytes": st["peak_admitted_bytes"], "budget_bytes": 16 << 30})
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--jobs", type=int, default=2000, help="jobs in the batched / served stream")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--quick", action="store_true", help="headline step only")
    ap.add_argument("--executor", default="persistent", choices=["persistent", "stream"],
                    help="persistent launch per step (default) or per-node stream launches")
    ap.add_argument("--widened", action="store_true",
                    help="only the polynomial, spin-glass, maximum-configuration, SizeMax(8), CountingMax(4) and "
                         "conditioning lines")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 256 MiB device copy (for scaling hardware byte counters) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: several GPUs would share slices and jobs with one final "
              "(+)-reduction of a scalar root, which is not implemented; use --gpus 1", file=sys.stderr)
        sys.exit(2)

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
    g, net, plan = build_k2(args.seed)
    tc, sc, rwc = plan.complexity()
    ctx = tn.Context(0)
    if args.widened:
        print(json.dumps({"independence_polynomial": independence_polynomial(ctx, net, plan, tc),
                          "spin_glass_buckyball": buckyball(ctx), "single_config_max": single_config(ctx, net, plan),
                          "size_max_8_weighted": size_max_8_weighted(ctx, g, plan, tc),
                          "counting_max_4": counting_max_4(ctx, net, plan, tc),
                          "conditioned": conditioned_batch(ctx, g, plan)}))
        return
    for _ in range(args.warmup):
        run_step(ctx, net, plan, args.executor)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        res = run_step(ctx, net, plan, args.executor)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / args.steps
    ops_per_step = len(STEP) * 2.0 ** tc
    value = ops_per_step / dt / 1e9

    # profiled steps: HIP events around every launch on the context stream
    ctx.set_profiling(True)
    for _ in range(5):
        run_step(ctx, net, plan, args.executor)
    recs = ctx.profile(clear=True)
    ctx.set_profiling(False)
    groups = group(recs)
    (kind, sr) = max(groups, key=lambda k: groups[k]["ms"])
    grp = groups[(kind, sr)]
    avg_ms = grp["ms"] / grp["n"]
    achieved = grp["bytes"] / grp["n"] / (avg_ms * 1e-3) / 1e9
    kname = "batch_kernel (persistent: %s)" % SR_NAME.get(sr, sr) if kind == "batch" else "%s/%s" % (kind, SR_NAME.get(sr, sr))
    roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_GBS, "unit": "GB/s", "frac": achieved / HBM_GBS,
            "traffic": measured_traffic() if kind == "batch" else None, "kernel": kname,
            "avg_launch_ms": avg_ms, "launches": grp["n"],
            "alg_bytes_per_launch": grp["bytes"] / grp["n"], "ops_per_launch": grp["ops"] / grp["n"],
            "share_of_device_time": grp["ms"] / sum(x["ms"] for x in groups.values())}

    out = {
        "metric": "semiring GOP/s & % roofline at largest intermediate; batched solves/s + p50/p99",
        "value": value,
        "unit": "GOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32+u32+f32",
        "data": "synthetic",
        "config": {"workload": "3-regular n=120 seed %d, unit weights: tropical int32 + exact count (3 + 1 "
                               "primes below 2^30, CRT) + Z(x=1) fp32, %s" % (args.seed, "one persistent launch per step"
                                                                   if args.executor == "persistent"
                                                                   else "per-node stream launches"),
                   "tc_log2": tc, "sc_log2": sc, "rwc_log2": rwc},
        "roofline": roof,
        "results": {"size_max": res[0]["size"], "count_all": str(res[1]["count"]), "log_z": res[2]["log_z"]},
    }
    if not args.quick:
        out["largest_intermediate"] = largest_intermediate(ctx)
        out["independence_polynomial"] = independence_polynomial(ctx, net, plan, tc)
        out["spin_glass_buckyball"] = buckyball(ctx)
        out["single_config_max"] = single_config(ctx, net, plan)
        out["size_max_8_weighted"] = size_max_8_weighted(ctx, g, plan, tc)
        out["counting_max_4"] = counting_max_4(ctx, net, plan, tc)
        out["conditioned"] = conditioned_batch(ctx, g, plan)
        out["batched"] = job_stream(ctx, args.jobs, args.seed)
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, ops_per_step)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
