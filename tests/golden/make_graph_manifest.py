"""Writes graphs_manifest.json: size and sha256 of each named synthetic workload.

Inputs only: it calls the seeded generators, nothing of the method.
Run from the repository root:  python tests/golden/make_graph_manifest.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from paper_1903_09422_amd import graphs as G  # noqa: E402


def main():
    out = {}
    for name in sorted(G.WORKLOADS):
        g, eps, delta, n_check = G.workload(name)
        out[name] = {"n": g.n, "arcs": g.num_arcs, "max_degree": int(g.degrees().max()),
                     "sha256": g.sha256(), "eps": eps, "delta": delta, "check_interval": n_check}
    with open(os.path.join(HERE, "graphs_manifest.json"), "w") as f:
        json.dump(out, f, indent=1, sort_keys=True)
        f.write("\n")


if __name__ == "__main__":
    main()
