"""Benchmark: KADABRA adaptive-sampling betweenness on one MI355X.

One step = one complete adaptive run (every step of the sampling path: pair
draws, bidirectional BFS, path draws, counter increments, frame merges and
FP64 stop checks at every boundary, and the scores c/tau written to device
memory) on the R-MAT scale-18 workload with eps = 0.01, delta = 0.1 and a
check every 16384 samples.  The graph is resident in HBM before timing.

Prints one JSON line.  `value` is samples/s over the timed steps; the line also
carries traversed edges/s, per-query latency percentiles, the roofline of the
dominant kernel (the sampler) and the CPU oracle's rate on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E

# Algorithmic bytes per unit of work counted by the sampler (a lower bound:
# what any implementation of the method must read per unit):
BYTES_PER = {
    "v_exp": 28,          # expanded frontier vertex: row_ptr pair 8 + sigma 16 + list entry 4
    "e_scan": 12,         # scanned arc: column index 4 + the neighbour's distance pair 8
    "e_bt": 12,           # arc scanned when backtracking: column index 4 + distance pair 8
    "path_interior": 4,   # counter increment
}


def algorithmic_bytes(stats: dict) -> int:
    return sum(BYTES_PER[k] * int(stats[k]) for k in BYTES_PER)


def cpu_baseline(g, eps, delta, seed, n_check, repeats):
    import oracle

    oracle.lib()
    t0 = time.perf_counter()
    samples = 0
    for _ in range(repeats):
        r = oracle.run(g, eps, delta, seed, n_check)
        samples += r.tau
    dt = time.perf_counter() - t0
    return {"value": samples / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{repeats} complete oracle run(s) of the same workload and seed "
                      f"(tau={r.tau} each), single-threaded, {dt:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat18", choices=["rmat18", "pgrid1024", "er4096"])
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--team", type=int, default=0)
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--frames", type=int, default=1)
    ap.add_argument("--overlap", type=int, default=1)
    ap.add_argument("--probe-min", type=int, default=-1)
    ap.add_argument("--cpu-repeats", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--traffic-json", default=os.path.join(ROOT, "profiles", "traffic.json"),
                    help="HBM bytes per sampler launch from rocprofv3 counters, if measured")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES device-to-device once (profiler calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch

        src = torch.ones(args.calibrate_copy // 4, dtype=torch.int32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": src.numel() * 4}))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): the sampling "
              "path here is single-device; see DESIGN.md for how it would shard.", file=sys.stderr)
        return 2

    import torch

    from paper_1903_09422_amd import Graph, graphs

    g, eps, delta, n_check = graphs.workload(args.workload)
    dev = Graph.from_csr(g)  # uploads the CSR: inputs resident before timing
    dev.set_param("check_interval", n_check)
    dev.set_param("team", args.team)
    dev.set_param("slots", args.slots)
    dev.set_param("frames", args.frames)
    dev.set_param("overlap", args.overlap)
    dev.set_param("probe_min", args.probe_min)
    stream = torch.cuda.Stream()
    dev.set_stream(stream)
    scores = torch.empty(g.n, dtype=torch.float64, device="cuda")

    def step():
        dev.run(eps, delta, args.seed)
        dev.result_device(scores=scores)
        return dev.stats()

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    lat, samples, escan, kern_ms, kern_bytes, launches = [], 0, 0, 0.0, 0, 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        st = step()
        stream.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
        samples += st["tau"]
        escan += st["e_scan"]
        kern_ms += st["ms_sample_kernels"]
        launches += st["sample_launches"]
        kern_bytes += algorithmic_bytes(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    achieved = kern_bytes / (kern_ms * 1e-3) / 1e9  # GB/s over the sampler launches
    traffic = None
    if os.path.exists(args.traffic_json):
        with open(args.traffic_json) as f:
            tj = json.load(f)
        if tj.get("workload") == args.workload and tj.get("kernel_source_sha") == _kernel_sha():
            traffic = tj.get("hbm_bytes_per_launch")
    out = {
        "metric": "samples/s (KADABRA adaptive sampling, eps=0.01)",
        "value": samples / dt,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": _describe(args.workload, g, eps, delta, n_check, args.seed),
            "tau": int(st["tau"]),
            "omega": int(st["omega"]),
            "mapping": {"team": dev.get_param("last_team"), "slots": dev.get_param("last_slots"),
                        "frames": args.frames, "overlap": args.overlap,
                        "probe_min": args.probe_min},
        },
        "traversed_edges_per_s": escan / dt,
        "query_latency_ms": {"p50": float(np.percentile(lat, 50)),
                             "p99": float(np.percentile(lat, 99))},
        "roofline": {
            "bound": "hbm",
            "kernel": "sample_kernel",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": traffic,
            "avg_launch_ms": kern_ms / max(launches, 1),
            "algorithmic_bytes_per_launch": kern_bytes / max(launches, 1),
        },
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(g, eps, delta, args.seed, n_check, args.cpu_repeats)
    dev.close()
    print(json.dumps(out))
    return 0


def _kernel_sha() -> str:
    import hashlib

    p = os.path.join(ROOT, "paper_1903_09422_amd", "csrc", "kadabra_kernels.hip")
    with open(p, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _describe(name, g, eps, delta, n_check, seed):
    shapes = {
        "rmat18": "R-MAT scale 18 (a,b,c,d = 0.57,0.19,0.19,0.05), edge factor 16, symmetrised, "
                  "dedup, LCC",
        "pgrid1024": "1024x1024 4-neighbour grid, 5% edges deleted, 0.1% random shortcuts, LCC",
        "er4096": "Erdos-Renyi G(4096, mean degree 8), LCC",
    }
    return (f"{name}: {shapes[name]}; n={g.n}, arcs={g.num_arcs}; eps={eps}, delta={delta}, "
            f"check every {n_check} samples, seed {seed}")


if __name__ == "__main__":
    sys.exit(main())
