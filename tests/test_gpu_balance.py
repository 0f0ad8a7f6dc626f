"""GPU parity of balanced delta_L(v), delta_U(v): the first phase, the plan
and the adaptive loop with per-vertex constants, through the C ABI, against
the CPU oracle.

Bar: bit-exact tau, decisions, every counter, the first-phase counters c1,
t* and every work counter, and bit-exact per-vertex constants
log(1/delta_L(v)), log(1/delta_U(v)): the library plans them on the host from
the first-phase count histogram, summed in the order the definition fixes
(nonzero rows in ascending count), with the same C library's exp and log as
the oracle.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1903_09422_amd import Batch, Graph, KadabraError, Server, _lib
from paper_1903_09422_amd import graphs as G

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
WORK_KEYS = ("v_exp", "e_scan", "e_bt", "path_interior", "disconnected")
FIRST_KEYS = ("v_exp", "e_scan", "e_bt", "path_interior", "disconnected")


def assert_bits(got, want):
    got = np.ascontiguousarray(got, dtype=np.float64)
    want = np.ascontiguousarray(want, dtype=np.float64)
    if not np.array_equal(got.view(np.uint64), want.view(np.uint64)):
        k = int(np.flatnonzero(got.view(np.uint64) != want.view(np.uint64))[0])
        raise AssertionError(f"constant {k} differs: {got[k]!r} vs {want[k]!r}")


def balanced_run(g, eps, delta, seed, n_check, first=0, **params):
    with Graph.from_csr(g) as dev:
        dev.set_param("check_interval", n_check)
        dev.set_param("balance", 1)
        dev.set_param("balance_samples", first)
        for k, v in params.items():
            dev.set_param(k, v)
        dev.run(eps, delta, seed)
        return dev.result(), dev.balance()


def assert_same_balanced(got, consts, want):
    LL, LU, c1 = consts
    assert np.array_equal(c1, want.c1)
    assert got.stats["first_samples"] == want.stats["first_samples"]
    assert got.stats["plan_tau"] == want.stats["plan_tau"]
    for k in FIRST_KEYS:
        assert got.stats["first_" + k] == want.stats["first_" + k], k
    assert_bits(LL, want.LL)
    assert_bits(LU, want.LU)
    assert got.tau == want.tau
    assert np.array_equal(got.decisions, want.decisions)
    if not np.array_equal(got.counts, want.counts):
        bad = np.flatnonzero(got.counts != want.counts)
        raise AssertionError(f"{bad.size} counters differ, first {bad[:5]}")
    for k in WORK_KEYS:
        assert got.stats[k] == want.stats[k], k


MIX = [
    (G.erdos_renyi(600, 6.0, seed=11), 0.05, 128),
    (G.rmat(10, 16, seed=5), 0.04, 256),
    (G.rhg(1 << 11, 10.0, 2.8, seed=7), 0.05, 200),
    (G.grid_graph(20, 20), 0.05, 64),
    (G.star_graph(30), 0.1, 33),  # no plan: uniform constants
    (G.disjoint_union(G.grid_graph(6, 6), G.cycle_graph(9)), 0.05, 77),
    (G.path_graph(50), 0.1, 100),
]


@pytest.mark.parametrize("team", [64, 256])
@pytest.mark.parametrize("k", range(len(MIX)))
def test_balanced_small_graphs(k, team):
    g, eps, n_check = MIX[k]
    for seed, first in ((1, 0), (4, 37)):
        print(f"case balanced {g.name} team={team} seed={seed} balance_samples={first}", flush=True)
        want = oracle.run(g, eps, 0.1, seed, n_check, first_samples=first if first else -1)
        got, consts = balanced_run(g, eps, 0.1, seed, n_check, first, team=team)
        assert_same_balanced(got, consts, want)


def test_balanced_mappings_and_epochs():
    """The first phase rides in the first sampling launch with any number of
    epochs per launch, overlap, frames and team."""
    g, eps, n_check = G.rmat(11, 16, seed=6), 0.03, 300
    want = oracle.run(g, eps, 0.1, 9, n_check, first_samples=-1)
    for params in ({"epochs_per_launch": 1}, {"epochs_per_launch": 3, "overlap": 0},
                   {"epochs_per_launch": 4}, {"frames": 3}, {"team": 128, "slots": 50},
                   {"team": 512}, {"probe_min": 0}):
        print("case balanced rmat11 mapping", params, flush=True)
        got, consts = balanced_run(g, eps, 0.1, 9, n_check, **params)
        assert_same_balanced(got, consts, want)


@pytest.mark.parametrize("name", ["rmat18", "pgrid1024", "er4096"])
def test_balanced_workload_against_stored_oracle(name):
    ref = json.load(open(os.path.join(GOLDEN, "oracle_runs.json")))[name + "_balanced"]
    g, eps, delta, n_check = G.workload(name)
    assert g.sha256() == ref["graph_sha256"]
    print(f"case {name} balanced, stored oracle result", flush=True)
    got, (LL, LU, c1) = balanced_run(g, eps, delta, ref["seed"], n_check)
    assert got.stats["plan_tau"] == ref["stats"]["plan_tau"]
    assert got.stats["first_samples"] == ref["stats"]["first_samples"]
    assert hashlib.sha256(c1.astype("<i4").tobytes()).hexdigest() == ref["c1_sha256"]
    idx = np.asarray(ref["sample_idx"])
    assert_bits(LL[idx], ref["sample_LL"])
    assert_bits(LU[idx], ref["sample_LU"])
    assert got.tau == ref["tau"]
    assert got.decisions.tolist() == ref["decisions"]
    assert got.counts[idx].tolist() == ref["sample_counts"]
    assert hashlib.sha256(got.counts.astype("<i4").tobytes()).hexdigest() == ref["counts_sha256"]
    for k in WORK_KEYS:
        assert got.stats[k] == ref["stats"][k], k
    for k in FIRST_KEYS:
        assert got.stats["first_" + k] == ref["stats"]["first_" + k], k


def test_balanced_then_uniform_on_one_handle():
    """Switching balance off again gives the uniform run (stored oracle
    result), and the constants read back as L."""
    ref = json.load(open(os.path.join(GOLDEN, "oracle_runs.json")))["er4096"]
    g, eps, delta, n_check = G.workload("er4096")
    print("case er4096 balanced then uniform", flush=True)
    with Graph.from_csr(g) as dev:
        dev.set_param("check_interval", n_check)
        dev.set_param("balance", 1)
        dev.run(eps, delta, 1)
        assert dev.result().stats["first_samples"] > 0
        dev.set_param("balance", 0)
        dev.run(eps, delta, 1)
        got = dev.result()
        assert got.tau == ref["tau"] and got.stats["first_samples"] == 0 and got.stats["plan_tau"] == 0
        assert hashlib.sha256(got.counts.astype("<i4").tobytes()).hexdigest() == ref["counts_sha256"]
        LL, LU, c1 = dev.balance()
        assert np.all(LL == ref["stats"]["L"]) and np.all(LU == LL) and not c1.any()
        for bad in (("balance", 2), ("balance_samples", -1)):
            with pytest.raises(KadabraError) as e:
                dev.set_param(*bad)
            assert e.value.status == _lib.EINVAL


def test_balanced_batch_and_server():
    """Balanced queries in a shared launch (batch) and under continuous
    batching (server) equal the oracle's balanced runs."""
    items = [(MIX[0], 3), (MIX[1], 4), (MIX[2], 5), (MIX[4], 6)]
    handles = [Graph.from_csr(g) for (g, _, _), _ in items]
    want = [oracle.run(g, eps, 0.1, seed, n_check, first_samples=-1) for (g, eps, n_check), seed in items]
    print("case balanced batch", flush=True)
    with Batch() as b:
        b.set_param("balance", 1)
        for h, ((g, eps, n_check), seed) in zip(handles, items):
            b.add(h, eps, 0.1, seed, n_check)
        b.run()
        for k, w in enumerate(want):
            got = b.result(k)
            assert got.tau == w.tau and np.array_equal(got.counts, w.counts)
            assert got.stats["plan_tau"] == w.stats["plan_tau"]
            assert got.stats["first_e_scan"] == w.stats["first_e_scan"]
        # the parameter applies to the queries already added, at the next run
        b.set_param("balance", 0)
        b.run()
        for k, ((g, eps, n_check), seed) in enumerate(items):
            got = b.result(k)
            u = oracle.run(g, eps, 0.1, seed, n_check)
            assert got.tau == u.tau and np.array_equal(got.counts, u.counts)
            assert got.stats["first_samples"] == 0
        b.set_param("balance", 1)
        b.run()
        for k, w in enumerate(want):
            got = b.result(k)
            assert got.tau == w.tau and np.array_equal(got.counts, w.counts)
    print("case balanced server", flush=True)
    with Server(handles) as srv:
        srv.set_param("balance", 1)
        tickets = [srv.submit(k, eps, 0.1, seed, n_check) for k, ((g, eps, n_check), seed) in enumerate(items)]
        for k, t in enumerate(tickets):
            assert srv.wait(t, timeout=60.0)
            got, _ = srv.result(t, k)
            assert got.tau == want[k].tau and np.array_equal(got.counts, want[k].counts)
            assert got.stats["plan_tau"] == want[k].stats["plan_tau"]
            srv.release(t)
        assert srv.info()["bytes_in_use"] == 0
    for h in handles:
        h.close()
