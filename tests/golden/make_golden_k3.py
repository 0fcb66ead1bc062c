"""Stored expected values for the King's-subgraph workload (24x24, p = 0.8,
weights k/2^14): the oracle's variable elimination, one process per value.

Calls only the CPU oracle; run from the repository root:
    python tests/golden/make_golden_k3.py [seed]
"""
import json
import multiprocessing as mp
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

BETAS = (0.5, 1.0, 2.0, 4.0)


def _graph(seed):
    g = gg.kings_subgraph(24, 0.8, seed)
    return g.with_weights(gg.dyadic_weights(g.nv, seed))


def _one(args):
    seed, what = args
    g = _graph(seed)
    t0 = time.time()
    if what == "tropical":
        r = oracle.eliminate(g, "tropical", max_width=25)
        val = r["size"]
    else:
        r = oracle.eliminate(g, "partition", float(what), max_width=25)
        val = r["log_z"]
    return what, val, time.time() - t0, r["width"]


if __name__ == "__main__":
    seed = int(sys.argv[1]) if len(sys.argv) > 1 else 0
    g = _graph(seed)
    tasks = [(seed, "tropical")] + [(seed, b) for b in BETAS]
    with mp.Pool(len(tasks)) as pool:
        res = pool.map(_one, tasks)
    rec = {"seed": seed, "nv": g.nv, "ne": g.ne, "log_z": {}}
    for what, val, dt, width in res:
        if what == "tropical":
            rec["size_max"] = val
        else:
            rec["log_z"][str(what)] = val
        rec["width"] = width
        print(what, val, "%.1fs" % dt, flush=True)
    path = os.path.join(HERE, "k3.json")
    data = json.load(open(path)) if os.path.exists(path) else {
        "about": "King's subgraph 24x24 p=0.8, weights k/2^14; oracle variable elimination", "cases": []}
    data["cases"] = [c for c in data["cases"] if c["seed"] != seed] + [rec]
    json.dump(data, open(path, "w"), indent=1)
    print("wrote k3 seed", seed)
