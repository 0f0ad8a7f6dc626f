"""Writes oracle_runs.json: the oracle's full result on the named workloads.

Calls only the seeded generators and oracle/ (never the HIP path).  Stores tau,
the per-boundary decisions, the work counters, the sha256 of the counters and
a fixed sample of (vertex, counter) pairs.  A name with the suffix
"_balanced" runs the workload with balanced delta_L(v), delta_U(v) (the
default first phase) and also stores t*, the first-phase counters' sha256 and
the constants at the sampled vertices.  Run from the repository root:
    python tests/golden/make_oracle_golden.py [workload ...]
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


def main(names):
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in names:
        balanced = name.endswith(BAL)
        g, eps, delta, n_check = G.workload(name[:-len(BAL)] if balanced else name)
        t0 = time.time()
        r = oracle.run(g, eps, delta, SEED, n_check, first_samples=-1 if balanced else 0)
        dt = time.time() - t0
        rng = np.random.default_rng(12345)
        idx = np.sort(rng.choice(g.n, size=min(g.n, 256), replace=False))
        data[name] = {
            "graph_sha256": g.sha256(), "seed": SEED, "eps": eps, "delta": delta,
            "check_interval": n_check, "tau": r.tau, "decisions": r.decisions.tolist(),
            "stats": {k: (float(v) if isinstance(v, float) else int(v)) for k, v in r.stats.items()},
            "counts_sha256": hashlib.sha256(r.counts.astype("<i4").tobytes()).hexdigest(),
            "counts_sum": int(r.counts.sum()), "counts_max": int(r.counts.max()),
            "sample_idx": idx.tolist(), "sample_counts": r.counts[idx].tolist(),
            "oracle_seconds": round(dt, 1),
        }
        if balanced:
            data[name].update({
                "c1_sha256": hashlib.sha256(r.c1.astype("<i4").tobytes()).hexdigest(),
                "sample_LL": r.LL[idx].tolist(), "sample_LU": r.LU[idx].tolist(),
            })
        print(name, r.tau, f"{dt:.1f}s")
    with open(OUT, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:] or sorted(G.WORKLOADS) + [w + BAL for w in sorted(G.WORKLOADS)])
