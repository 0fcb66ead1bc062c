"""Write the stored expected values used by the GPU parity tests.

Calls only the CPU oracle (``oracle/``) on inputs from ``graphgen``; nothing
here touches the GPU library.  Run from the repository root:

    python tests/golden/make_golden.py [k1|k2|k3|all]
"""
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402


def k1():
    """3-regular n=20, seeds 0..19, unit weights: brute force (O1)."""
    out = []
    for s in range(20):
        g = gg.random_regular(20, 3, s)
        r = oracle.brute_force(g, [0.0, 1.0])
        out.append({"seed": s, "size_max": r["size_max"], "count_max": r["count_max"],
                    "count_all": r["count_all"], "log_z_beta1": r["log_z"][1]})
    return {"about": "3-regular n=20 unit weights; oracle brute force", "cases": out}


def k2():
    """3-regular n=120, seeds 0..4, unit weights: elimination (O2)."""
    out = []
    for s in range(5):
        g = gg.random_regular(120, 3, s)
        t = oracle.eliminate(g, "tropical")
        c = oracle.eliminate(g, "count")
        ct = oracle.eliminate(g, "counting_tropical")
        z = oracle.eliminate(g, "partition", 0.0)
        out.append({"seed": s, "size_max": t["size"], "count_all": str(c["count"]),
                    "count_max": str(ct["count"]), "log_z_beta0": z["log_z"], "width": t["width"]})
    return {"about": "3-regular n=120 unit weights; oracle variable elimination", "cases": out}


def k3(seeds=(0,), betas=(0.5, 1.0, 2.0, 4.0)):
    """King's subgraph 24x24 @0.8, dyadic weights: elimination (O2)."""
    out = []
    for s in seeds:
        g = gg.kings_subgraph(24, 0.8, s)
        g = g.with_weights(gg.dyadic_weights(g.nv, s))
        t0 = time.time()
        rec = {"seed": s, "nv": g.nv, "ne": g.ne}
        rec["size_max"] = oracle.eliminate(g, "tropical", max_width=25)["size"]
        rec["log_z"] = {str(b): oracle.eliminate(g, "partition", b, max_width=25)["log_z"] for b in betas}
        rec["seconds"] = time.time() - t0
        out.append(rec)
        print("k3 seed", s, rec, flush=True)
    return {"about": "King's subgraph 24x24 p=0.8, weights k/2^14; oracle variable elimination", "cases": out}


if __name__ == "__main__":
    which = sys.argv[1] if len(sys.argv) > 1 else "all"
    for name, fn in (("k1", k1), ("k2", k2), ("k3", k3)):
        if which in (name, "all"):
            data = fn()
            with open(os.path.join(HERE, name + ".json"), "w") as f:
                json.dump(data, f, indent=1)
            print("wrote", name)
