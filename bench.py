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

# Algorithmic bytes per unit of work.  The roofline's `achieved` uses the
# per-unit figures of the method's traffic model over the oracle's counters of
# the same samples (the oracle counts every unit; its counters for the stored
# workloads are in tests/golden/oracle_runs.json):
#   8 V_exp   row_ptr pair of an expanded frontier vertex
#   8 E_scan  column index 4 + the target's distance from the expanding side 4
#   16 V_new  the other side's distance (meeting test) 4 + distance and sigma
#             written 12, for every newly reached vertex
#   8 E_pred  sigma read per predecessor arc
#   12 E_bt   column index and distance per arc of a backtracked row
#   12 per path interior vertex: its row_ptr pair 8 (|backtracked| taken as
#             the interior count) + the counter increment 4
MODEL_BYTES = {"v_exp": 8, "e_scan": 8, "v_new": 16, "e_pred": 8, "e_bt": 12, "path_interior": 12}
# The same terms for this sampler, from its own counters: sigma is read once
# per frontier vertex (the push form, 8 per V_exp instead of 8 per E_pred),
# and only the new vertices actually written are charged 16 -- a meeting
# level expanded with the meeting probe writes only the meeting set.
PROBE_MODEL_BYTES = {"v_exp": 16, "e_scan": 8, "v_written": 16, "e_bt": 12, "path_interior": 12}


def model_bytes(stats: dict, per_unit: dict) -> int:
    return sum(per_unit[k] * int(stats[k]) for k in per_unit)


def stored_oracle(name: str):
    """The oracle's stored result for a named workload (or the list of the
    batched pool's), written by tests/golden/make_oracle_golden.py."""
    path = os.path.join(ROOT, "tests", "golden", "oracle_runs.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f).get(name)


def copy_bandwidth_gbs(nbytes: int = 1 << 30, reps: int = 10) -> float:
    """Device-to-device copy rate on this GPU (bytes read + written per s)."""
    import torch

    src = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    e1.synchronize()
    ms = e0.elapsed_time(e1)
    del src, dst
    torch.cuda.empty_cache()
    return 2.0 * nbytes * reps / (ms * 1e-3) / 1e9


def cpu_baseline(g, eps, delta, seed, n_check, min_seconds, max_repeats):
    """Complete oracle runs of the same query, repeated until min_seconds of
    CPU work have been timed (at least one run, at most max_repeats)."""
    import oracle

    oracle.lib()
    t0 = time.perf_counter()
    samples = repeats = 0
    while True:
        r = oracle.run(g, eps, delta, seed, n_check)
        samples += r.tau
        repeats += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or repeats >= max_repeats:
            break
    return {"value": samples / dt, "unit": "samples/s", "cores": 1, "kind": "oracle",
            "sample": f"{repeats} complete oracle run(s) of the same workload and seed "
                      f"(tau={r.tau} each), single-threaded, {dt:.1f} s"}


def host_threads() -> int:
    """Host threads this process may use (its CPU affinity), at most 16 (the
    host share of one GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def cpu_baseline_threads(g, eps, delta, seed, n_check, min_seconds, max_repeats):
    """The oracle's adaptive loop on all usable host threads (per-thread
    counter frames of each epoch's samples, added at every boundary; the
    result equals the single-threaded oracle's), repeated as cpu_baseline."""
    import oracle

    threads = host_threads()
    t0 = time.perf_counter()
    samples = repeats = 0
    while True:
        r = oracle.run_threads(g, eps, delta, seed, n_check, threads)
        samples += r.tau
        repeats += 1
        dt = time.perf_counter() - t0
        if dt >= min_seconds or repeats >= max_repeats:
            break
    return {"value": samples / dt, "unit": "samples/s", "cores": threads, "kind": "oracle-threads",
            "sample": f"{repeats} complete threaded oracle run(s) of the same workload and seed "
                      f"(tau={r.tau} each), {threads} threads, {dt:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat18",
                    choices=["rmat18", "pgrid1024", "er4096", "batch64", "serve"])
    ap.add_argument("--serve-queries", type=int, default=256)
    ap.add_argument("--serve-loads", default="0.5,0.8,1.0",
                    help="serve: Poisson arrival rates as multiples of the one-at-a-time capacity")
    ap.add_argument("--round-us", default="",
                    help="serve: comma-separated round work caps (microseconds, 0 = none) of "
                         "extra batching servers to compare with the default one")
    ap.add_argument("--no-rmat22", action="store_true",
                    help="serve: leave R-MAT scale 22 out of the graph pool")
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--team", type=int, default=0,
                    help="lanes per sample; 0: the workload's mapping (WORKLOAD_TEAM, else the "
                         "library's automatic choice)")
    ap.add_argument("--slots", type=int, default=0)
    ap.add_argument("--frames", type=int, default=1)
    ap.add_argument("--overlap", type=int, default=1)
    ap.add_argument("--epochs-per-launch", type=int, default=2)
    ap.add_argument("--probe-min", type=int, default=-1)
    ap.add_argument("--probe-pull", type=int, default=0,
                    help="1: meeting probes in the pull form (scan the other side's frontier rows)")
    ap.add_argument("--balanced-steps", type=int, default=10,
                    help="queries of the balanced leg (per-vertex delta_L, delta_U); 0: skip it")
    ap.add_argument("--cpu-seconds", type=float, default=10.0,
                    help="CPU oracle leg: repeat complete runs until this much time is timed")
    ap.add_argument("--cpu-repeats", type=int, default=50, help="CPU oracle leg: at most this many runs")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--legs", default="pgrid1024,er4096,batch64,serve",
                    help="with the default workload: the other workloads measured in the same run "
                         "(comma-separated; empty: none), reported under `workloads`")
    ap.add_argument("--traffic-json", default=None,
                    help="HBM bytes per sampler launch from rocprofv3 counters (default: "
                         "profiles/sample_kernel_<workload>_traffic.json)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only copy BYTES device-to-device once (profiler calibration) and exit")
    ap.add_argument("--ingest-pmc", metavar="DIR",
                    help="read rocprofv3 outputs under DIR (kernel trace and FETCH_SIZE / "
                         "WRITE_SIZE passes of this bench and of --calibrate-copy) and write the "
                         "sampler's traffic summary under profiles/, then exit")
    args = ap.parse_args()
    if args.ingest_pmc:
        return ingest_pmc(args.ingest_pmc, args.workload)
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
              "path here runs on a single device.", file=sys.stderr)
        return 2

    if args.workload == "batch64":
        out = bench_batch(args, args.steps, args.warmup, autotune=True)
        print(json.dumps(out))
        return 0
    if args.workload == "serve":
        out = bench_serve(args, tuple(float(x) for x in args.serve_loads.split(",") if x))
        print(json.dumps(out))
        return 0

    copy_gbs = copy_bandwidth_gbs()
    out = measure_single(args.workload, args, args.steps, args.warmup, args.balanced_steps,
                         not args.no_cpu, copy_gbs)
    legs = [w for w in args.legs.split(",") if w] if args.workload == "rmat18" else []
    if legs:
        out["workloads"] = {}
    for w in legs:
        print(f"bench: leg {w}", file=sys.stderr, flush=True)
        if w == "batch64":
            leg = bench_batch(args, 3, 1, autotune=True)
        elif w == "serve":
            leg = bench_serve(args, (1.0,))
        else:
            leg = measure_single(w, args, 5 if w == "pgrid1024" else args.steps, 1, 0, False, copy_gbs)
        out["workloads"][w] = _leg_summary(leg)
    print(json.dumps(out))
    return 0


def _leg_summary(leg: dict) -> dict:
    keep = ("value", "unit", "ms_per_step", "config", "traversed_edges_per_s", "query_latency_ms",
            "roofline", "serial_samples_per_s", "speedup_vs_serial", "autotuned", "saturated",
            "speedup_vs_one_at_a_time", "poisson", "dtype")
    return {k: leg[k] for k in keep if k in leg}


# Mapping per single-query workload (no result depends on it): 128-lane teams,
# eight per CU, were measured faster than the library's automatic choice
# (256-lane teams, four per CU) on R-MAT-18 (+3 to +7%) and ER-4096 (+5%), and
# level on the grid.  The library keeps 256 lanes by default because 128-lane
# teams double the slot pool, and a process that holds many graph handles (the
# 64-graph batch leg) then runs out of device memory.
WORKLOAD_TEAM = {"rmat18": 128, "er4096": 128}


def measure_single(workload, args, steps, warmup, balanced_steps, with_cpu, copy_gbs) -> dict:
    """One query of a named workload, run `steps` times (one step = one
    complete adaptive run plus the device scores)."""
    import torch

    from paper_1903_09422_amd import Graph, graphs

    g, eps, delta, n_check = graphs.workload(workload)
    dev = Graph.from_csr(g)  # uploads the CSR: inputs resident before timing
    dev.set_param("check_interval", n_check)
    dev.set_param("team", args.team if args.team else WORKLOAD_TEAM.get(workload, 0))
    dev.set_param("slots", args.slots)
    dev.set_param("frames", args.frames)
    dev.set_param("overlap", args.overlap)
    dev.set_param("epochs_per_launch", args.epochs_per_launch)
    dev.set_param("probe_min", args.probe_min)
    dev.set_param("probe_pull", args.probe_pull)
    stream = torch.cuda.Stream()
    dev.set_stream(stream)
    scores = torch.empty(g.n, dtype=torch.float64, device="cuda")

    def step():
        dev.run(eps, delta, args.seed)
        dev.result_device(scores=scores)
        return dev.stats()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    lat, samples, escan, kern_ms, probe_bytes, launches = [], 0, 0, 0.0, 0, 0
    t0 = time.perf_counter()
    for _ in range(steps):
        ts = time.perf_counter()
        st = step()
        stream.synchronize()
        lat.append((time.perf_counter() - ts) * 1e3)
        samples += st["tau"]
        escan += st["e_scan"]
        kern_ms += st["ms_sample_kernels"]
        launches += st["sample_launches"]
        probe_bytes += model_bytes(st, PROBE_MODEL_BYTES)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0

    avg_launch_ms = kern_ms / max(launches, 1)
    # the method's bytes for these samples, from the oracle's counters of the
    # same query (stored for seed 1; every shared counter equals the GPU's)
    ref = stored_oracle(workload)
    model = None
    if ref and ref["seed"] == args.seed and ref["graph_sha256"] == g.sha256() and ref["tau"] == st["tau"] \
            and all(int(ref["stats"][k]) == int(st[k]) for k in ("v_exp", "e_scan", "e_bt", "path_interior")):
        model = model_bytes(ref["stats"], MODEL_BYTES) / max(st["sample_launches"], 1)
    probe_per_launch = probe_bytes / max(launches, 1)
    per_launch = model if model is not None else probe_per_launch
    achieved = per_launch / (avg_launch_ms * 1e-3) / 1e9
    probe_achieved = probe_per_launch / (avg_launch_ms * 1e-3) / 1e9
    traffic = None
    tj_path = args.traffic_json or os.path.join(ROOT, "profiles", f"sample_kernel_{workload}_traffic.json")
    if os.path.exists(tj_path):
        with open(tj_path) as f:
            tj = json.load(f)
        if tj.get("workload") == workload and tj.get("kernel_source_sha") == _kernel_sha():
            traffic = tj.get("hbm_bytes_per_launch")
    traffic_gbs = None if traffic is None else traffic / (avg_launch_ms * 1e-3) / 1e9
    out = {
        "metric": "samples/s (KADABRA adaptive sampling, eps=0.01)" if eps == 0.01 else
                  f"samples/s (KADABRA adaptive sampling, eps={eps})",
        "value": samples / dt,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": dt * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {
            "workload": _describe(workload, g, eps, delta, n_check, args.seed),
            "tau": int(st["tau"]),
            "omega": int(st["omega"]),
            "mapping": {"team": dev.get_param("last_team"), "slots": dev.get_param("last_slots"),
                        "frames": args.frames, "overlap": args.overlap,
                        "epochs_per_launch": args.epochs_per_launch,
                        "probe_min": args.probe_min, "probe_pull": args.probe_pull},
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
            "traffic_gbs": traffic_gbs,
            "avg_launch_ms": avg_launch_ms,
            "algorithmic_bytes_per_launch": per_launch,
            "model": ("8 V_exp + 8 E_scan + 16 V_new + 8 E_pred + 12 E_bt + 12 interior, oracle counters"
                      if model is not None else "push-form model (no stored oracle counters for this query)"),
            "probe_model": {"bytes_per_launch": probe_per_launch, "achieved": probe_achieved,
                            "frac": probe_achieved / HBM_PEAK_GBS,
                            "terms": "16 V_exp + 8 E_scan + 16 V_written + 12 E_bt + 12 interior"},
            "copy_gbs": copy_gbs,
            "frac_of_copy": achieved / copy_gbs,
        },
    }
    if balanced_steps > 0:
        out["balanced"] = balanced_leg(dev, step, stream, balanced_steps, dt * 1e3 / steps)
    if with_cpu:
        out["cpu_baseline"] = cpu_baseline(g, eps, delta, args.seed, n_check, args.cpu_seconds,
                                           args.cpu_repeats)
        out["cpu_baseline_threads"] = cpu_baseline_threads(g, eps, delta, args.seed, n_check,
                                                           args.cpu_seconds / 2, args.cpu_repeats)
    dev.close()
    return out


def balanced_leg(dev, step, stream, nsteps, uniform_ms):
    """The same query with balanced delta_L(v), delta_U(v): time per query
    (first phase, plan and adaptive loop) beside the uniform constants'."""
    dev.set_param("balance", 1)
    step()
    stream.synchronize()
    t0 = time.perf_counter()
    for _ in range(nsteps):
        st = step()
        stream.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / nsteps
    dev.set_param("balance", 0)
    drawn = int(st["tau"] + st["first_samples"])
    return {"ms_per_query": ms, "uniform_ms_per_query": uniform_ms, "speedup": uniform_ms / ms,
            "tau": int(st["tau"]), "first_samples": int(st["first_samples"]),
            "plan_tau": int(st["plan_tau"]), "samples_per_s": drawn / (ms * 1e-3)}


def bench_batch(args, steps, warmup, autotune=False) -> dict:
    """The batched workload: 64 queries (32 R-MAT of scales 12-16, 32 random
    hyperbolic graphs of 2^14-2^17 vertices; eps from {0.05, 0.02, 0.01}),
    run one after another through Graph.run and together through one Batch,
    on the same GPU (with autotune, the batch's mapping is picked by the
    library's autotuner first).  value = samples/s of the batched form."""
    import torch

    from paper_1903_09422_amd import Batch, Graph, graphs

    pool = graphs.batch_pool()
    handles = [Graph.from_csr(g) for g, *_ in pool]
    for h, (g, eps, delta, n_check, seed) in zip(handles, pool):
        h.set_param("check_interval", n_check)
        h.set_param("epochs_per_launch", args.epochs_per_launch)
    batch = Batch()
    batch.set_param("team", args.team)
    batch.set_param("slots", args.slots)
    batch.set_param("probe_min", args.probe_min)
    batch.set_param("epochs_per_launch", args.epochs_per_launch)
    for h, (g, eps, delta, n_check, seed) in zip(handles, pool):
        batch.add(h, eps, delta, seed, n_check)
    tuned = batch.autotune(2048) if autotune else None

    def serial():
        tot = 0
        for h, (g, eps, delta, n_check, seed) in zip(handles, pool):
            h.run(eps, delta, seed)
            tot += h.stats()["tau"]
        return tot

    def batched():
        batch.run()
        return sum(batch.stats(k)["tau"] for k in range(len(pool)))

    for _ in range(max(warmup, 1)):
        serial()
        batched()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    s_serial = sum(serial() for _ in range(steps))
    t_serial = time.perf_counter() - t0
    lat = []
    t0 = time.perf_counter()
    s_batch = 0
    for _ in range(steps):
        ts = time.perf_counter()
        s_batch += batched()
        lat.append((time.perf_counter() - ts) * 1e3)
    t_batch = time.perf_counter() - t0
    assert s_serial == s_batch
    balanced = None
    if args.balanced_steps > 0:
        # the same batch with balanced per-vertex delta_L, delta_U: time per batch
        batch.set_param("balance", 1)
        batched()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            s_bal = batched()
        t_bal = (time.perf_counter() - t0) / steps
        first = sum(batch.stats(k)["first_samples"] for k in range(len(pool)))
        batch.set_param("balance", 0)
        balanced = {"ms_per_batch": t_bal * 1e3, "uniform_ms_per_batch": t_batch * 1e3 / steps,
                    "speedup": (t_batch / steps) / t_bal, "samples": s_bal,
                    "first_phase_samples": first, "uniform_samples": s_batch // steps}
    out = {
        "metric": "samples/s (KADABRA adaptive sampling, 64-query batch)",
        "value": s_batch / t_batch,
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": t_batch * 1e3 / steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "batch64: 32 R-MAT (scale 12 + k mod 5, edge factor 16) + 32 "
                               "threshold random hyperbolic graphs (n = 2^(14 + k mod 4), mean "
                               "degree 10, exponent 2.8); eps from {0.05, 0.02, 0.01}, delta 0.1, "
                               "checks every 1024 samples",
                   "queries": len(pool), "samples_per_step": s_batch // steps,
                   "mapping": {"team": batch.get_param("last_team"),
                               "slots": batch.get_param("last_slots"),
                               "epochs_per_launch": batch.get_param("epochs_per_launch"),
                               "probe_min": batch.get_param("probe_min")}},
        "autotuned": tuned is not None,
        "serial_samples_per_s": s_serial / t_serial,
        "serial_ms_per_step": t_serial * 1e3 / steps,
        "speedup_vs_serial": (s_batch / t_batch) / (s_serial / t_serial),
        "batch_latency_ms": {"p50": float(np.percentile(lat, 50)), "p99": float(np.percentile(lat, 99))},
    }
    if balanced:
        out["balanced"] = balanced
    batch.close()
    for h in handles:
        h.close()
    return out


def bench_serve(args, loads) -> dict:
    """Serving: a seeded stream of queries (graph drawn uniformly from the
    64-graph pool, the perturbed 1024 x 1024 grid and R-MAT scale 22; eps from
    {0.05, 0.01}, delta 0.1, checks every 16384 samples) against resident
    graphs.  Two servers answer the same stream: one that runs a query at a
    time (max_active 1, first come first served) and the continuous-batching
    one; with --balanced-steps > 0 also a continuous-batching server whose
    queries use balanced per-vertex delta_L, delta_U (fewer samples per query,
    so its figures to compare are queries/s and latency).  Each first takes
    the whole stream at once (saturation: its capacity), then Poisson arrivals
    at 0.5, 0.8 and 1.0 times the one-at-a-time capacity.  value = the
    (uniform) batching server's samples/s at saturation."""
    import torch

    from paper_1903_09422_amd import Graph, Server, graphs

    print("serve: building graphs", file=sys.stderr, flush=True)
    pool = graphs.serve_pool(with_rmat22=not args.no_rmat22)
    handles = [Graph.from_csr(g) for g in pool]
    queries, gaps = graphs.serve_trace(len(pool), args.serve_queries, seed=7 + args.seed)
    print(f"serve: {len(pool)} graphs, {len(queries)} queries", file=sys.stderr, flush=True)

    def replay(srv, rate):
        """Submit the stream (all at once if rate is None), wait for all;
        returns (total samples, makespan s, server info)."""
        srv.info(reset=True)
        offsets = np.zeros(len(queries)) if rate is None else np.cumsum(gaps) / rate
        t0 = time.perf_counter()
        tickets = []
        for (gi, eps, delta, n_check, seed), off in zip(queries, offsets):
            now = time.perf_counter() - t0
            if off > now:
                time.sleep(off - now)
            tickets.append((srv.submit(gi, eps, delta, seed, n_check), time.perf_counter() - t0))
        tot, first, end = 0, 0, 0.0
        for (t, ts), (gi, *_rest) in zip(tickets, queries):
            srv.wait(t)
            res, lat = srv.result(t, gi, scores=False)
            tot += res.tau
            first += res.stats["first_samples"]
            end = max(end, ts + lat / 1e3)
            srv.release(t)
        info = srv.info()
        info["first_samples"] = first
        return tot, end, info

    out_rates = {}
    legs = {}
    servers = [("one_at_a_time", 1, 0, None), ("batching", 0, 0, None)]
    if args.balanced_steps > 0:
        servers.append(("batching_balanced", 0, 1, None))
    for cap in (int(x) for x in args.round_us.split(",") if x):
        servers.append((f"batching_round_us_{cap}", 0, 0, cap))
    for name, max_active, balance, round_us in servers:
        srv = Server(handles, max_active=max_active)
        for k, v in (("team", args.team), ("slots", args.slots), ("probe_min", args.probe_min),
                     ("epochs_per_launch", args.epochs_per_launch), ("balance", balance)):
            srv.set_param(k, v)
        if round_us is not None:
            srv.set_param("round_us", round_us)
        replay(srv, None)  # warm-up: pool, buffers, code
        torch.cuda.synchronize()
        tot, span, info = replay(srv, None)
        legs[name] = {"samples_per_s": tot / span, "queries_per_s": len(queries) / span,
                      "makespan_s": span, "samples": tot, "first_phase_samples": info["first_samples"],
                      "p50_ms": info["p50_ms"], "p99_ms": info["p99_ms"],
                      "peak_active": info["peak_active"]}
        print(f"serve: {name} saturated {tot / span:.4g} samples/s", file=sys.stderr, flush=True)
        cap = legs["one_at_a_time"]["queries_per_s"]
        for f in loads:
            t2, span2, inf2 = replay(srv, f * cap)
            assert t2 == tot
            out_rates.setdefault(f"{f:.1f}x", {"arrivals_per_s": f * cap})[name] = {
                "p50_ms": inf2["p50_ms"], "p99_ms": inf2["p99_ms"], "max_ms": inf2["max_ms"],
                "mean_queue_ms": inf2["mean_queue_ms"], "samples_per_s": t2 / span2,
                "peak_active": inf2["peak_active"]}
            print(f"serve: {name} at {f}x p50 {inf2['p50_ms']:.3g} ms p99 {inf2['p99_ms']:.3g} ms",
                  file=sys.stderr, flush=True)
        srv.close()
    assert legs["one_at_a_time"]["samples"] == legs["batching"]["samples"]
    b, o = legs["batching"], legs["one_at_a_time"]
    out = {
        "metric": "samples/s (KADABRA adaptive sampling, served stream at saturation)",
        "value": b["samples_per_s"],
        "unit": "samples/s",
        "n_gpus": 1,
        "steps": 1,
        "warmup": 1,
        "ms_per_step": b["makespan_s"] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"serve: {len(queries)} queries over {len(pool)} resident graphs "
                               "(64-graph pool + perturbed grid 1024^2"
                               + ("" if args.no_rmat22 else " + R-MAT scale 22") +
                               "), eps from {0.05, 0.01}, delta 0.1, checks every 16384 samples"},
        "saturated": legs,
        "speedup_vs_one_at_a_time": b["samples_per_s"] / o["samples_per_s"],
        "poisson": out_rates,
    }
    for h in handles:
        h.close()
    return out


COPY_BYTES = 1 << 30
PMC_CMDS = {
    "trace": "rocprofv3 --kernel-trace --stats -f csv -d DIR/ktrace -o bench -- "
             "python3 bench.py --workload {w} --steps 5 --warmup 1 --no-cpu --balanced-steps 0 --legs ''",
    "fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d DIR/pmc_FETCH_SIZE -o bench -- "
             "python3 bench.py --workload {w} --steps 2 --warmup 0 --no-cpu --balanced-steps 0 --legs ''",
    "write": "rocprofv3 --pmc WRITE_SIZE -f csv -d DIR/pmc_WRITE_SIZE -o bench -- "
             "python3 bench.py --workload {w} --steps 2 --warmup 0 --no-cpu --balanced-steps 0 --legs ''",
    "copy_fetch": "rocprofv3 --pmc FETCH_SIZE -f csv -d DIR/pmc_copy_FETCH_SIZE -o copy -- "
                  "python3 bench.py --calibrate-copy 1073741824",
    "copy_write": "rocprofv3 --pmc WRITE_SIZE -f csv -d DIR/pmc_copy_WRITE_SIZE -o copy -- "
                  "python3 bench.py --calibrate-copy 1073741824",
    "l2": "rocprofv3 --pmc TCC_HIT_sum TCC_MISS_sum -f csv -d DIR/pmc_tcc -o bench -- "
          "python3 bench.py --workload {w} --steps 2 --warmup 0 --no-cpu --balanced-steps 0 --legs ''",
    "wrreq": "rocprofv3 --pmc TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum TCC_EA0_RDREQ_sum "
             "TCC_EA0_RDREQ_DRAM_sum -f csv -d DIR/pmc_ea -o bench -- "
             "python3 bench.py --workload {w} --steps 2 --warmup 0 --no-cpu --balanced-steps 0 --legs ''",
}


def ingest_pmc(d: str, workload: str) -> int:
    """Turn rocprofv3 CSVs into the committed summary of the sampler kernel:
    average duration, and HBM bytes per launch = FETCH_SIZE and WRITE_SIZE
    (KiB per dispatch) each scaled by the factor that maps the same counter,
    read on a plain 1 GiB device copy, onto the bytes that copy moves."""
    import csv

    def rows(path):
        with open(path) as f:
            return list(csv.DictReader(f))

    def kib(sub, prefix, name):
        out = []
        for r in rows(os.path.join(d, sub, f"{prefix}_counter_collection.csv")):
            if name in r["Kernel_Name"]:
                out.append(float(r["Counter_Value"]))
        return out

    fetch_factor = COPY_BYTES / (kib("pmc_copy_FETCH_SIZE", "copy", "copyBuffer")[0] * 1024)
    write_factor = COPY_BYTES / (kib("pmc_copy_WRITE_SIZE", "copy", "copyBuffer")[0] * 1024)
    # launches that sampled (the gated speculative launch exits at once)
    fetch = [x for x in kib("pmc_FETCH_SIZE", "bench", "sample_kernel") if x > 1024]
    write = [x for x in kib("pmc_WRITE_SIZE", "bench", "sample_kernel") if x > 1024]
    hbm = (np.mean(fetch) * 1024 * fetch_factor) + (np.mean(write) * 1024 * write_factor)
    stats = rows(os.path.join(d, "ktrace", "bench_kernel_stats.csv"))
    trace = rows(os.path.join(d, "ktrace", "bench_kernel_trace.csv"))
    durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-6 for r in trace
            if "sample_kernel" in r["Kernel_Name"]]
    full = [x for x in durs if x > 0.05 * max(durs)]
    l2 = None
    if os.path.isdir(os.path.join(d, "pmc_tcc")):
        hits = kib("pmc_tcc", "bench", "sample_kernel")  # both counters, by row
        by = {}
        for r in rows(os.path.join(d, "pmc_tcc", "bench_counter_collection.csv")):
            if "sample_kernel" in r["Kernel_Name"]:
                by.setdefault(r["Dispatch_Id"], {})[r["Counter_Name"]] = float(r["Counter_Value"])
        full_l2 = [v for v in by.values() if v.get("TCC_HIT_sum", 0) + v.get("TCC_MISS_sum", 0) > 1e5]
        if full_l2 and hits:
            h = float(np.mean([v["TCC_HIT_sum"] for v in full_l2]))
            m = float(np.mean([v["TCC_MISS_sum"] for v in full_l2]))
            l2 = {"hits_per_launch": h, "misses_per_launch": m, "hit_rate": h / (h + m)}
    # the write bytes again from the L2-to-memory write requests (32 or 64
    # bytes each), beside WRITE_SIZE, and the share of L2 read misses that
    # went to DRAM
    ea = None
    if os.path.isdir(os.path.join(d, "pmc_ea")):
        by = {}
        for r in rows(os.path.join(d, "pmc_ea", "bench_counter_collection.csv")):
            if "sample_kernel" in r["Kernel_Name"]:
                by.setdefault(r["Dispatch_Id"], {})[r["Counter_Name"]] = float(r["Counter_Value"])
        full_ea = [v for v in by.values() if v.get("TCC_EA0_RDREQ_sum", 0) > 1e5]
        if full_ea:
            wr = float(np.mean([v["TCC_EA0_WRREQ_sum"] for v in full_ea]))
            w64 = float(np.mean([v["TCC_EA0_WRREQ_64B_sum"] for v in full_ea]))
            rd = float(np.mean([v["TCC_EA0_RDREQ_sum"] for v in full_ea]))
            rdd = float(np.mean([v["TCC_EA0_RDREQ_DRAM_sum"] for v in full_ea]))
            ea = {"write_requests": wr, "write_requests_64B": w64,
                  "write_bytes": 64.0 * w64 + 32.0 * (wr - w64), "read_requests": rd,
                  "read_requests_dram": rdd, "dram_share_of_reads": rdd / rd if rd else None}
    summary = {
        "kernel": "sample_kernel", "workload": workload, "kernel_source_sha": _kernel_sha(),
        "l2": l2, "ea": ea,
        "hbm_bytes_per_launch": hbm,
        "fetch_kib_per_launch": float(np.mean(fetch)), "write_kib_per_launch": float(np.mean(write)),
        "fetch_factor": fetch_factor, "write_factor": write_factor,
        "avg_launch_ms_sampling_launches": float(np.mean(full)),
        "commands": {k: v.format(w=workload) for k, v in PMC_CMDS.items()},
    }
    base = os.path.join(ROOT, "profiles", f"sample_kernel_{workload}")
    with open(base + "_traffic.json", "w") as f:
        json.dump(summary, f, indent=1)
        f.write("\n")
    with open(base + ".md", "w") as f:
        f.write(f"# sample_kernel on {workload}: rocprofv3 summary\n\n")
        f.write("Commands (run from the repository root; DIR = output folder):\n\n")
        for k, v in summary["commands"].items():
            f.write(f"- {k}: `{v}`\n")
        f.write("\n## Kernel statistics (--kernel-trace --stats)\n\n")
        f.write("| kernel | calls | total ms | average ms | % |\n|---|---|---|---|---|\n")
        for r in stats:
            f.write(f"| {r['Name'][:60]} | {r['Calls']} | {float(r['TotalDurationNs']) * 1e-6:.3f} | "
                    f"{float(r['AverageNs']) * 1e-6:.3f} | {float(r['Percentage']):.1f} |\n")
        f.write(f"\nSampling launches of the sampler (speculative launches that exit at once "
                f"excluded): {len(full)}, average {np.mean(full):.3f} ms.\n")
        f.write("\n## HBM traffic (--pmc, one pass per counter)\n\n")
        f.write(f"- FETCH_SIZE per sampling launch: {np.mean(fetch):.0f} KiB; copy calibration "
                f"factor {fetch_factor:.3f} (a 1 GiB device copy reads "
                f"{COPY_BYTES / fetch_factor / 1024:.0f} KiB)\n")
        f.write(f"- WRITE_SIZE per sampling launch: {np.mean(write):.0f} KiB; calibration factor "
                f"{write_factor:.3f}\n")
        f.write(f"- HBM bytes per launch: {hbm / 1e9:.3f} GB\n")
        if ea:
            f.write("\n## L2 to memory requests (--pmc TCC_EA0_WRREQ_sum TCC_EA0_WRREQ_64B_sum "
                    "TCC_EA0_RDREQ_sum TCC_EA0_RDREQ_DRAM_sum)\n\n")
            f.write(f"- write requests per sampling launch: {ea['write_requests']:.4g} "
                    f"({ea['write_requests_64B']:.4g} of 64 bytes, the rest 32): "
                    f"{ea['write_bytes'] / 1e9:.3f} GB written, against WRITE_SIZE's "
                    f"{np.mean(write) * 1024 * write_factor / 1e9:.3f} GB\n")
            f.write(f"- read requests: {ea['read_requests']:.4g}, of which to DRAM "
                    f"{ea['read_requests_dram']:.4g}\n")
        if l2:
            f.write("\n## L2 (--pmc TCC_HIT_sum TCC_MISS_sum)\n\n")
            f.write(f"- per sampling launch: {l2['hits_per_launch']:.4g} hits, "
                    f"{l2['misses_per_launch']:.4g} misses, hit rate {l2['hit_rate']:.3f}\n")
    print(json.dumps(summary))
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
