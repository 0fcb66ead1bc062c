"""Stored expected values for the full 20 x 20 grid (the Sec. 5.1 example):
the exact number of independent sets and ln Z(beta) from the oracle's
variable elimination (256-bit counts, long double Z).

Calls only the CPU oracle; run from the repository root:
    python tests/golden/make_golden_square20.py
"""
import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

BETAS = (0.0, 0.5, 1.0)


def _one(what):
    g = gg.square_lattice(20)
    if what == "count":
        return what, str(oracle.eliminate(g, "count", max_width=21)["count"])
    if what == "counting_tropical":
        r = oracle.eliminate(g, "counting_tropical", max_width=21)
        return what, [r["size"], str(r["count"])]
    return what, oracle.eliminate(g, "partition", float(what), max_width=21)["log_z"]


if __name__ == "__main__":
    with mp.Pool(2 + len(BETAS)) as pool:
        res = dict(pool.map(_one, ["count", "counting_tropical"] + list(BETAS)))
    rec = {
        "about": "20x20 grid (square(20) of Sec. 5.1); oracle variable elimination. count: exact number of "
                 "independent sets (decimal); counting_tropical: [largest size, number of largest sets]; "
                 "log_z: ln Z(beta) for unit weights",
        "count": res["count"],
        "counting_tropical": res["counting_tropical"],
        "log_z": {str(b): res[b] for b in BETAS},
    }
    json.dump(rec, open(os.path.join(HERE, "square20.json"), "w"), indent=1)
    print(rec)
