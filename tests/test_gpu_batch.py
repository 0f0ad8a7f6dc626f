"""Batched runs (many queries on many graphs in shared launches) and the
autotuner: every query's result equals the oracle's and its own single run,
bit for bit, whatever the mix and the mapping."""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle
from paper_1903_09422_amd import Batch, Graph, KadabraError, _lib
from paper_1903_09422_amd import graphs as G

pytestmark = pytest.mark.gpu

WORK_KEYS = ("v_exp", "e_scan", "e_bt", "path_interior", "disconnected")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")

MIX = [
    (G.erdos_renyi(600, 6.0, seed=11), 0.05, 7, 128),
    (G.rmat(10, 16, seed=5), 0.04, 8, 256),
    (G.rmat(11, 16, seed=6), 0.05, 9, 1024),
    (G.rhg(1 << 11, 10.0, 2.8, seed=7), 0.05, 10, 200),
    (G.grid_graph(20, 20), 0.05, 11, 64),
    (G.star_graph(30), 0.1, 12, 33),
    (G.path_graph(50), 0.1, 13, 100),
    (G.disjoint_union(G.grid_graph(6, 6), G.cycle_graph(9)), 0.05, 14, 77),
]


def _same(got, want):
    assert got.tau == want.tau
    assert np.array_equal(got.counts, want.counts)
    for k in WORK_KEYS:
        assert got.stats[k] == want.stats[k], k


@pytest.mark.parametrize("team,overlap,epl", [(256, 1, 2), (128, 1, 2), (64, 1, 1), (256, 0, 3), (256, 1, 4)])
def test_batch_mix_equals_oracle(team, overlap, epl):
    print(f"case batch mix team={team} overlap={overlap} epochs_per_launch={epl}", flush=True)
    handles = [Graph.from_csr(g) for g, *_ in MIX]
    with Batch() as b:
        b.set_param("team", team)
        b.set_param("overlap", overlap)
        b.set_param("epochs_per_launch", epl)
        for h, (g, eps, seed, n_check) in zip(handles, MIX):
            b.add(h, eps, 0.1, seed, n_check)
        b.run()
        for k, (g, eps, seed, n_check) in enumerate(MIX):
            _same(b.result(k), oracle.run(g, eps, 0.1, seed, n_check))
    for h in handles:
        h.close()


def test_batch_rerun_and_clear():
    g, eps, seed, n_check = MIX[0]
    h = Graph.from_csr(g)
    want = oracle.run(g, eps, 0.1, seed, n_check)
    with Batch() as b:
        with pytest.raises(KadabraError) as e:
            b.run()
        assert e.value.status == _lib.ESTATE
        i = b.add(h, eps, 0.1, seed, n_check)
        j = b.add(h, eps, 0.1, seed + 1, n_check)  # two queries on one graph
        b.run()
        _same(b.result(i), want)
        _same(b.result(j), oracle.run(g, eps, 0.1, seed + 1, n_check))
        b.run()  # again: same results
        _same(b.result(i), want)
        with pytest.raises(KadabraError):
            b.result(5)
        b.clear()
        with pytest.raises(KadabraError):
            b.run()
    h.close()


def same_as_stored(got, ref):
    """A result against a stored oracle result (tests/golden/oracle_runs.json,
    written by make_oracle_golden.py from the oracle alone): tau, every counter
    (sha256 and sampled values) and every work counter."""
    assert got.tau == ref["tau"]
    assert hashlib.sha256(got.counts.astype("<i4").tobytes()).hexdigest() == ref["counts_sha256"]
    assert got.counts[ref["sample_idx"]].tolist() == ref["sample_counts"]
    for k in WORK_KEYS:
        assert got.stats[k] == ref["stats"][k], k
    assert got.stats["omega"] == ref["stats"]["omega"]


def test_batch_pool_equals_oracle_and_single_runs():
    """The 64-graph batched workload: every query in the mix equals the
    oracle's stored result and the same query run alone."""
    pool = G.batch_pool()
    with open(os.path.join(GOLDEN, "oracle_runs.json")) as f:
        stored = json.load(f)["batch64"]
    assert len(stored) == len(pool) == 64
    print("case batch pool (64 graphs)", flush=True)
    handles = [Graph.from_csr(g) for g, *_ in pool]
    with Batch() as b:
        for h, (g, eps, delta, n_check, seed) in zip(handles, pool):
            b.add(h, eps, delta, seed, n_check)
        b.run()
        for k, (h, (g, eps, delta, n_check, seed)) in enumerate(zip(handles, pool)):
            ref = stored[k]
            assert (ref["graph_sha256"], ref["eps"], ref["seed"], ref["check_interval"]) == \
                (g.sha256(), eps, seed, n_check)
            mixed = b.result(k)
            same_as_stored(mixed, ref)
            h.set_param("check_interval", n_check)
            h.run(eps, delta, seed)
            _same(h.result(), mixed)
    for h in handles:
        h.close()


def test_autotune_is_result_neutral():
    g, eps, delta, n_check = G.workload("rmat18")
    with open(os.path.join(GOLDEN, "oracle_runs.json")) as f:
        ref = json.load(f)["rmat18"]
    print("case autotune rmat18", flush=True)
    with Graph.from_csr(g) as dev:
        dev.set_param("check_interval", n_check)
        chosen = dev.autotune(eps, delta, trial_samples=4096)
        assert chosen["team"] in (64, 128, 256) and chosen["slots"] > 0
        dev.run(eps, delta, ref["seed"])
        got = dev.result()
    assert got.tau == ref["tau"]
    assert hashlib.sha256(got.counts.astype("<i4").tobytes()).hexdigest() == ref["counts_sha256"]


def test_stopped_runs_in_speculative_launches():
    """The launch queued after a boundary is gated on that boundary's check.
    When every run of it has stopped, its workgroups leave at once; beside a
    run that goes on, a stopped run's claims are skipped.  Either way the claim
    counter ends where the next launch expects it, so repeated runs on the same
    handle or batch still equal the oracle."""
    a = (G.erdos_renyi(600, 6.0, seed=11), 0.05, 128)  # stops by the rule at 1024 of omega = 1400
    b = (G.grid_graph(20, 20), 0.05, 64)                # stops by the rule at 1536 of omega = 2000
    want_a = {s: oracle.run(a[0], a[1], 0.1, s, a[2]) for s in (1, 2)}
    want_b = oracle.run(b[0], b[1], 0.1, 1, b[2])
    assert want_a[1].tau < want_a[1].stats["omega"] and want_b.tau < want_b.stats["omega"]
    assert want_a[1].tau < want_b.tau  # a stops while b goes on
    ha, hb = Graph.from_csr(a[0]), Graph.from_csr(b[0])
    for epl in (1, 2):
        print(f"case stopped runs, epochs_per_launch={epl}", flush=True)
        ha.set_param("check_interval", a[2])
        ha.set_param("epochs_per_launch", epl)
        for s in (1, 2, 1):
            ha.run(a[1], 0.1, s)
            _same(ha.result(), want_a[s])
        with Batch() as bt:
            bt.set_param("epochs_per_launch", epl)
            bt.add(ha, a[1], 0.1, 1, a[2])
            bt.add(hb, b[1], 0.1, 1, b[2])
            for _ in range(2):
                bt.run()
                _same(bt.result(0), want_a[1])
                _same(bt.result(1), want_b)
    ha.close()
    hb.close()
