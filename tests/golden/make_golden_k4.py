"""Stored expected values for the served stream (2000 jobs of
graphgen.job_mix(2000, seed 0, n in [40, 200]): every job with n <= 130 and
a seeded 2% sample of the larger ones, by the oracle's variable elimination
(tropical size, counting-tropical size and count mod 2^64, ln Z at x = 1).
Jobs whose elimination width exceeds 26 are stored as null (not checked).

Calls only the CPU oracle; run from the repository root:
    python tests/golden/make_golden_k4.py
"""
import json
import multiprocessing as mp

import numpy as np
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import graphgen as gg  # noqa: E402
import oracle  # noqa: E402

NJOBS, SEED, N_LO, N_HI, CHECK_N = 2000, 0, 40, 200, 130
SAMPLE_FRAC, SAMPLE_SEED = 0.02, 1  # of the jobs with n > CHECK_N


def _one(job):
    n, gseed, sr = job
    g = gg.random_regular(n, 3, gseed)
    try:
        if sr == "tropical_i32":
            return oracle.eliminate(g, "tropical", max_width=26)["size"]
        if sr == "counting_tropical":
            r = oracle.eliminate(g, "counting_tropical", max_width=26)
            return [r["size"], str(r["count"] % 2 ** 64)]
        return oracle.eliminate(g, "partition", 0.0, max_width=26)["log_z"]
    except oracle.OracleError:
        return None


if __name__ == "__main__":
    mix = gg.job_mix(NJOBS, SEED, N_LO, N_HI)
    idx = [k for k, j in enumerate(mix) if j[0] <= CHECK_N]
    large = [k for k, j in enumerate(mix) if j[0] > CHECK_N]
    rng = np.random.default_rng(SAMPLE_SEED)
    sample = sorted(rng.choice(large, size=round(SAMPLE_FRAC * len(large)), replace=False).tolist())
    idx += sample
    # largest first, so the long eliminations overlap
    order = sorted(idx, key=lambda k: -mix[k][0])
    with mp.Pool(int(sys.argv[1]) if len(sys.argv) > 1 else 8) as pool:
        vals = pool.map(_one, [mix[k] for k in order], chunksize=1)
    got = dict(zip(order, vals))
    rec = {"about": "served-stream jobs graphgen.job_mix(%d, %d, %d, %d) with n <= %d, and a %g sample (numpy "
                    "default_rng(%d).choice without replacement) of the larger ones: oracle elimination (tropical: "
                    "size; counting_tropical: [size, count mod 2^64 as decimal]; partition_f32: ln Z at x = 1); null "
                    "= elimination width above 26, not checked" % (NJOBS, SEED, N_LO, N_HI, CHECK_N, SAMPLE_FRAC,
                                                                  SAMPLE_SEED),
           "njobs": NJOBS, "seed": SEED, "n_range": [N_LO, N_HI], "check_n": CHECK_N,
           "sample": {"fraction": SAMPLE_FRAC, "seed": SAMPLE_SEED, "jobs": sample},
           "expected": {str(k): got[k] for k in sorted(got)}}
    json.dump(rec, open(os.path.join(HERE, "k4_jobs.json"), "w"))
    print(len(got), "jobs,", sum(v is None for v in got.values()), "unchecked")
