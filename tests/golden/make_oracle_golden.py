"""Writes oracle_runs.json: the oracle's full result on the named workloads.

Calls only the seeded generators and oracle/ (never the HIP path).  Stores tau,
the per-boundary decisions, the work counters, the sha256 of the counters and
a fixed sample of (vertex, counter) pairs.  A name with the suffix
"_balanced" runs the workload with balanced delta_L(v), delta_U(v) (the
default first phase) and also stores t*, the first-phase counters' sha256 and
the constants at the sampled vertices.  Besides the named workloads:
    batch64         every query of the 64-graph batched pool (its own eps,
                    seed and check interval), as a list in pool order;
    rmat22_eps0.05, rmat22_eps0.01
                    the served R-MAT scale-22 graph (edge factor 16, seed 1)
                    at the serving settings: delta 0.1, checks every 16384
                    samples, run seed 1.
Run from the repository root:
    python tests/golden/make_oracle_golden.py [name ...]
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1903_09422_amd import graphs as G  # noqa: E402

SEED = 1
BAL = "_balanced"
OUT = os.path.join(HERE, "oracle_runs.json")
RMAT22 = {"rmat22_eps0.05": 0.05, "rmat22_eps0.01": 0.01}


def entry(g, r, eps, delta, n_check, seed, dt, samples=256):
    rng = np.random.default_rng(12345)
    idx = np.sort(rng.choice(g.n, size=min(g.n, samples), replace=False))
    return {
        "graph_sha256": g.sha256(), "seed": seed, "eps": eps, "delta": delta,
        "check_interval": n_check, "tau": r.tau, "decisions": r.decisions.tolist(),
        "stats": {k: (float(v) if isinstance(v, float) else int(v)) for k, v in r.stats.items()},
        "counts_sha256": hashlib.sha256(r.counts.astype("<i4").tobytes()).hexdigest(),
        "counts_sum": int(r.counts.sum()), "counts_max": int(r.counts.max()),
        "sample_idx": idx.tolist(), "sample_counts": r.counts[idx].tolist(),
        "oracle_seconds": round(dt, 1),
    }


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        if name == "batch64":
            rows = []
            t0 = time.time()
            for g, eps, delta, n_check, seed in G.batch_pool():
                t1 = time.time()
                r = oracle.run(g, eps, delta, seed, n_check)
                rows.append(entry(g, r, eps, delta, n_check, seed, time.time() - t1, samples=64))
            data[name] = rows
            print(name, len(rows), f"{time.time() - t0:.1f}s")
            continue
        if name in RMAT22:
            g, eps, delta, n_check = G.rmat(22, 16, seed=1), RMAT22[name], 0.1, 16384
            t0 = time.time()
            r = oracle.run(g, eps, delta, SEED, n_check)
            data[name] = entry(g, r, eps, delta, n_check, SEED, time.time() - t0)
            print(name, r.tau, f"{time.time() - t0:.1f}s")
            continue
        balanced = name.endswith(BAL)
        g, eps, delta, n_check = G.workload(name[:-len(BAL)] if balanced else name)
        t0 = time.time()
        r = oracle.run(g, eps, delta, SEED, n_check, first_samples=-1 if balanced else 0)
        dt = time.time() - t0
        data[name] = entry(g, r, eps, delta, n_check, SEED, dt)
        if balanced:
            idx = np.asarray(data[name]["sample_idx"])
            data[name].update({
                "c1_sha256": hashlib.sha256(r.c1.astype("<i4").tobytes()).hexdigest(),
                "sample_LL": r.LL[idx].tolist(), "sample_LU": r.LU[idx].tolist(),
            })
        print(name, r.tau, f"{dt:.1f}s")
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or sorted(G.WORKLOADS) + [w + BAL for w in sorted(G.WORKLOADS)]
         + ["batch64"] + sorted(RMAT22))
