"""Serving with continuous batching: queries submitted at any time join the
running launches at the next round boundary; each result equals the oracle's
and the query's own single run, bit for bit, whatever else was in flight.
Admission respects the device-memory budget."""
import hashlib
import json
import os
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1903_09422_amd import Graph, KadabraError, Server, _lib
from paper_1903_09422_amd import graphs as G

pytestmark = pytest.mark.gpu

WORK_KEYS = ("v_exp", "e_scan", "e_bt", "path_interior", "disconnected")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

MIX = [
    (G.erdos_renyi(600, 6.0, seed=11), 0.05, 128),
    (G.rmat(10, 16, seed=5), 0.04, 256),
    (G.rhg(1 << 11, 10.0, 2.8, seed=7), 0.05, 200),
    (G.grid_graph(20, 20), 0.05, 64),
    (G.star_graph(30), 0.1, 33),
    (G.disjoint_union(G.grid_graph(6, 6), G.cycle_graph(9)), 0.05, 77),
]


def _same(got, want):
    assert got.tau == want.tau
    assert np.array_equal(got.counts, want.counts)
    for k in WORK_KEYS:
        assert got.stats[k] == want.stats[k], k


def _charge(n, frames=1, epochs=2):
    # counters 4n + scores 8n + one frame set per epoch in flight (2 per launched epoch)
    return n * (4 + 8 + 8 * epochs * frames)


@pytest.mark.parametrize("round_us", [None, 0, 1, 300])
def test_serve_staggered_equals_oracle(round_us):
    """Queries arrive while others run (two submitting threads, random gaps);
    every result equals the oracle's, whatever the round work cap (the
    default, none, one that admits a query only when none runs, and a small
    one)."""
    print(f"case serve staggered mix, round_us={round_us}", flush=True)
    handles = [Graph.from_csr(g) for g, *_ in MIX]
    jobs = [(k, seed) for seed in (3, 4) for k in range(len(MIX))]
    tickets = {}
    lock = threading.Lock()
    with Server(handles) as srv:
        if round_us is not None:
            srv.set_param("round_us", round_us)
        assert srv.get_param("round_us") == (16000 if round_us is None else round_us)
        def submitter(part, rng_seed):
            rng = np.random.default_rng(rng_seed)
            for k, seed in part:
                time.sleep(float(rng.uniform(0, 0.004)))
                g, eps, n_check = MIX[k]
                t = srv.submit(k, eps, 0.1, seed, n_check)
                with lock:
                    tickets[(k, seed)] = t

        th = [threading.Thread(target=submitter, args=(jobs[i::2], i)) for i in range(2)]
        for t in th:
            t.start()
        for t in th:
            t.join()
        for (k, seed), t in sorted(tickets.items()):
            assert srv.wait(t, timeout=60.0)
            g, eps, n_check = MIX[k]
            got, lat = srv.result(t, k)
            _same(got, oracle.run(g, eps, 0.1, seed, n_check))
            np.testing.assert_array_equal(got.scores, got.counts / float(got.tau))
            assert lat > 0 and got.stats["ms_total"] == lat
            srv.release(t)
        info = srv.info()
        assert info["completed"] == len(jobs) and info["failed"] == 0
        assert info["active"] == 0 and info["pending"] == 0 and info["bytes_in_use"] == 0
        assert info["p50_ms"] <= info["p99_ms"] <= info["max_ms"]
    for h in handles:
        h.close()


def test_serve_budget_gates_admission():
    """With a budget of one query's memory, a second query waits (not final,
    its result and release refused) until the first is released; then it runs
    and equals its own single run."""
    g, eps, n_check = MIX[1]
    print("case serve budget gate", flush=True)
    with Graph.from_csr(g) as h:
        with Server([h], hbm_budget_bytes=_charge(g.n)) as srv:
            a = srv.submit(0, eps, 0.1, 21, n_check)
            b = srv.submit(0, eps, 0.1, 22, n_check)
            assert srv.wait(a, timeout=60.0)
            # a's counters and score buffer stay charged until release: b waits
            assert not srv.wait(b, timeout=0.2)
            inf = srv.info()
            assert inf["pending"] == 1 and inf["active"] == 0
            assert inf["bytes_in_use"] == g.n * 12 <= inf["budget_bytes"]
            for call in (lambda: srv.result(b, 0), lambda: srv.release(b)):
                with pytest.raises(KadabraError) as e:
                    call()
                assert e.value.status == _lib.ESTATE
            got_a, _ = srv.result(a, 0)
            srv.release(a)
            assert srv.wait(b, timeout=60.0)
            got_b, _ = srv.result(b, 0)
            srv.release(b)
            assert srv.info()["peak_active"] == 1
        for seed, got in ((21, got_a), (22, got_b)):
            h.set_param("check_interval", n_check)
            h.run(eps, 0.1, seed)
            _same(got, h.result())


def test_serve_many_in_flight_and_buffer_reuse():
    """A burst of 24 queries over three graphs runs in shared launches
    (peak > 1), reusing released buffers; every result equals its single run."""
    graphs = [MIX[0][0], MIX[2][0], MIX[3][0]]
    handles = [Graph.from_csr(g) for g in graphs]
    print("case serve burst", flush=True)
    want = {}
    for k, h in enumerate(handles):
        h.set_param("check_interval", 96)
        for seed in range(8):
            h.run(0.05, 0.1, 100 + seed)
            want[(k, seed)] = h.result()
    with Server(handles, max_active=16) as srv:
        for rnd in range(2):  # a second round reuses the binned buffers
            tk = {(k, s): srv.submit(k, 0.05, 0.1, 100 + s, 96) for k in range(3) for s in range(8)}
            for (k, s), t in tk.items():
                assert srv.wait(t, timeout=60.0)
                got, _ = srv.result(t, k, scores=(rnd == 0))
                _same(got, want[(k, s)])
                srv.release(t)
        inf = srv.info()
        assert 1 < inf["peak_active"] <= 16
        assert inf["completed"] == 48 and inf["bytes_in_use"] == 0
    for h in handles:
        h.close()


def test_serve_errors_and_shutdown():
    g, eps, n_check = MIX[3]
    print("case serve errors", flush=True)
    with Graph.from_csr(g) as h:
        srv = Server([h], hbm_budget_bytes=_charge(g.n))
        for call, status in ((lambda: srv.submit(1, eps, 0.1, 1, n_check), _lib.EINVAL),
                             (lambda: srv.submit(0, 1.5, 0.1, 1, n_check), _lib.EINVAL),
                             (lambda: srv.wait(12345, 0.0), _lib.EINVAL),
                             (lambda: srv.result(12345, 0), _lib.EINVAL),
                             (lambda: srv.release(12345), _lib.EINVAL)):
            with pytest.raises(KadabraError) as e:
                call()
            assert e.value.status == status
        srv.set_param("frames", 2)  # before the first submit: allowed, doubles the frames
        with pytest.raises(KadabraError) as e:
            srv.submit(0, eps, 0.1, 1, n_check)  # now needs more than the budget
        assert e.value.status == _lib.ERANGE
        srv.close()
        srv = Server([h])
        assert srv.get_param("graphs") == 1 and srv.get_param("max_active") == 256
        t = srv.submit(0, eps, 0.1, 5, n_check)
        with pytest.raises(KadabraError) as e:
            srv.set_param("team", 64)
        assert e.value.status == _lib.ESTATE
        srv.wait(t, timeout=60.0)
        # destroy with work queued: pending queries are canceled, running ones
        # stop at their next boundary, and the call returns
        for s in range(20):
            srv.submit(0, 0.01, 0.1, 1000 + s, 8)
        t0 = time.time()
        srv.close()
        assert time.time() - t0 < 30.0


def test_serve_device_failure_stops_server():
    """A device-side check failure (forced: room for 3 BFS levels) fails the
    queries in flight with EDEVICE, and the server then refuses new work."""
    g = G.path_graph(60)
    print("case serve device failure", flush=True)
    with Graph.from_csr(g) as h:
        with Server([h]) as srv:
            srv.set_param("test_level_cap", 3)
            t = srv.submit(0, 0.1, 0.1, 1, 32)
            assert srv.wait(t, timeout=60.0)
            with pytest.raises(KadabraError) as e:
                srv.result(t, 0)
            assert e.value.status == _lib.EDEVICE
            assert srv.info()["failed"] == 1
            with pytest.raises(KadabraError) as e:
                srv.submit(0, 0.1, 0.1, 2, 32)
            assert e.value.status == _lib.EDEVICE
            srv.release(t)


def test_serve_concurrent_reads_and_release():
    """Result reads of one ticket from several threads race with its release:
    a read returns the same counters or, once released, EINVAL; a release
    during a read is refused with ESTATE and succeeds afterwards."""
    g, eps, n_check = MIX[0]
    print("case serve concurrent reads", flush=True)
    with Graph.from_csr(g) as h, Server([h]) as srv:
        t = srv.submit(0, eps, 0.1, 9, n_check)
        assert srv.wait(t, timeout=60.0)
        want, _ = srv.result(t)
        errors = []

        def reader():
            for _ in range(40):
                try:
                    got, _ = srv.result(t)
                    if not np.array_equal(got.counts, want.counts):
                        errors.append("counters differ")
                except KadabraError as e:
                    if e.status != _lib.EINVAL:
                        errors.append(e)
                    return

        ths = [threading.Thread(target=reader) for _ in range(3)]
        for x in ths:
            x.start()
        refused = 0
        while True:
            try:
                srv.release(t)
                break
            except KadabraError as e:
                assert e.status == _lib.ESTATE
                refused += 1
        for x in ths:
            x.join()
        assert not errors, errors
        with pytest.raises(KadabraError) as e:
            srv.result(t)
        assert e.value.status == _lib.EINVAL


def test_serve_workload_graphs_equal_oracle():
    """The served workload's graphs at their serving settings, submitted
    together: R-MAT scale 22 at eps 0.05 and 0.01, the perturbed 1024 x 1024
    grid and R-MAT scale 18 at eps 0.01, and eight queries of the 64-graph
    pool.  Every result equals the oracle's stored result (tau, every counter
    by sha256 and sampled values, every work counter)."""
    with open(os.path.join(GOLDEN, "oracle_runs.json")) as f:
        stored = json.load(f)
    print("case serve workload graphs: building R-MAT scale 22", flush=True)
    rmat22 = G.rmat(22, 16, seed=1)
    assert rmat22.sha256() == stored["rmat22_eps0.01"]["graph_sha256"]
    print("case serve workload graphs: building the pool, grid and R-MAT scale 18", flush=True)
    pool = G.batch_pool()
    grid, _, _, _ = G.workload("pgrid1024")
    r18, _, _, _ = G.workload("rmat18")
    picks = [3, 11, 24, 30, 33, 42, 50, 63]
    graphs = [rmat22, grid, r18] + [pool[k][0] for k in picks]
    handles = [Graph.from_csr(g) for g in graphs]
    jobs = [(0, stored["rmat22_eps0.01"]), (1, stored["pgrid1024"]), (0, stored["rmat22_eps0.05"]),
            (2, stored["rmat18"])]
    for j, k in enumerate(picks):
        jobs.append((3 + j, stored["batch64"][k]))
    print("case serve workload graphs: serving", len(jobs), "queries", flush=True)
    with Server(handles) as srv:
        tickets = [srv.submit(gi, ref["eps"], ref["delta"], ref["seed"], ref["check_interval"])
                   for gi, ref in jobs]
        for t, (gi, ref) in zip(tickets, jobs):
            assert srv.wait(t, timeout=120.0)
            got, _ = srv.result(t, gi, scores=False)
            assert graphs[gi].sha256() == ref["graph_sha256"]
            assert got.tau == ref["tau"], gi
            assert hashlib.sha256(got.counts.astype("<i4").tobytes()).hexdigest() == ref["counts_sha256"], gi
            assert got.counts[ref["sample_idx"]].tolist() == ref["sample_counts"]
            for k in WORK_KEYS:
                assert got.stats[k] == ref["stats"][k], (gi, k)
            srv.release(t)
            print("  served graph", gi, "tau", got.tau, "equals the oracle", flush=True)
    for h in handles:
        h.close()
