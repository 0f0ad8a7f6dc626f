"""Checkpoint and resume at a check boundary (Algorithm 1 checks only
consistent states; sample i depends on i alone, Appendix D): a run stopped at
a boundary and continued from its checkpoint, on another handle, gives
exactly the uninterrupted run -- tau, every decision, every counter, every
work counter -- and equals the oracle."""
import hashlib
import json
import os
import threading

import numpy as np
import pytest

import oracle
from paper_1903_09422_amd import Checkpoint, Graph, KadabraError, _lib
from paper_1903_09422_amd import graphs as G

pytestmark = pytest.mark.gpu

WORK_KEYS = ("v_exp", "e_scan", "e_bt", "path_interior", "disconnected")
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _same(got, want):
    assert got.tau == want.tau
    assert np.array_equal(got.decisions, want.decisions)
    assert np.array_equal(got.counts, want.counts)
    for k in WORK_KEYS:
        assert got.stats[k] == want.stats[k], k


@pytest.mark.parametrize("epl,overlap", [(1, 1), (2, 1), (3, 0)])
def test_stop_and_resume_chain(epl, overlap):
    """Stopped every two boundaries and resumed each time on a fresh handle
    until the run ends: the same result as the oracle's uninterrupted run."""
    g, eps, n_check, seed = G.grid_graph(20, 20), 0.05, 64, 1
    want = oracle.run(g, eps, 0.1, seed, n_check)
    assert len(want.decisions) > 6  # many boundaries
    print(f"case checkpoint chain epochs_per_launch={epl} overlap={overlap}", flush=True)
    with Graph.from_csr(g) as dev:
        for k, v in (("check_interval", n_check), ("stop_after_epochs", 2), ("epochs_per_launch", epl),
                     ("overlap", overlap)):
            dev.set_param(k, v)
        with pytest.raises(KadabraError) as e:
            dev.run(eps, 0.1, seed)
        assert e.value.status == _lib.ECANCELED
        ck, counts = dev.checkpoint()
    stops = 1
    while True:
        assert ck.tau == min(ck.epochs * n_check, ck.omega) and ck.tau < want.tau
        assert counts.sum() == ck.work[3]
        with Graph.from_csr(g) as dev:
            dev.set_param("stop_after_epochs", 2)
            dev.set_param("epochs_per_launch", epl)
            try:
                dev.resume(ck, counts)
            except KadabraError as err:
                assert err.status == _lib.ECANCELED
                ck, counts = dev.checkpoint()
                stops += 1
                continue
            got = dev.result()
            break
    assert stops >= 2
    _same(got, want)


def test_resume_rmat18_equals_stored_oracle():
    """R-MAT-18 stopped after its first boundary (16,384 samples) and resumed
    on another handle: the oracle's stored result."""
    g, eps, delta, n_check = G.workload("rmat18")
    with open(os.path.join(GOLDEN, "oracle_runs.json")) as f:
        ref = json.load(f)["rmat18"]
    print("case checkpoint rmat18", flush=True)
    with Graph.from_csr(g) as dev:
        dev.set_param("check_interval", n_check)
        dev.set_param("epochs_per_launch", 1)
        dev.set_param("stop_after_epochs", 1)
        with pytest.raises(KadabraError):
            dev.run(eps, delta, ref["seed"])
        ck, counts = dev.checkpoint()
        with pytest.raises(KadabraError) as e:
            dev.result()  # a stopped run has no result
        assert e.value.status == _lib.ESTATE
    assert ck.tau == 16384 and ck.epochs == 1
    # a checkpoint is plain data: it survives a copy
    ck2 = Checkpoint.from_buffer_copy(bytes(ck))
    with Graph.from_csr(g) as dev:
        dev.resume(ck2, counts.copy())
        got = dev.result()
    assert got.tau == ref["tau"] and got.decisions.tolist() == ref["decisions"]
    assert hashlib.sha256(got.counts.astype("<i4").tobytes()).hexdigest() == ref["counts_sha256"]
    for k in WORK_KEYS:
        assert got.stats[k] == ref["stats"][k], k


def test_cancel_leaves_a_checkpoint():
    """A run canceled from another thread stops at a boundary; resuming it
    gives the uninterrupted result."""
    g, eps, n_check, seed = G.erdos_renyi(3000, 6.0, seed=4), 0.02, 16, 2
    want = oracle.run(g, eps, 0.1, seed, n_check)
    print("case checkpoint after cancel", flush=True)
    with Graph.from_csr(g) as dev:
        dev.set_param("check_interval", n_check)
        dev.set_param("epochs_per_launch", 1)
        t = threading.Timer(0.002, dev.cancel)
        t.start()
        try:
            dev.run(eps, 0.1, seed)
            canceled = False
        except KadabraError as e:
            assert e.status == _lib.ECANCELED
            canceled = True
        t.join()
        if not canceled:
            pytest.skip("the run finished before the cancel arrived")
        ck, counts = dev.checkpoint()
    with Graph.from_csr(g) as dev:
        dev.resume(ck, counts)
        _same(dev.result(), want)


def test_resume_rejects_bad_checkpoints():
    g = G.grid_graph(12, 12)
    with Graph.from_csr(g) as dev:
        dev.set_param("check_interval", 32)
        dev.set_param("stop_after_epochs", 1)
        dev.set_param("epochs_per_launch", 1)
        with pytest.raises(KadabraError):
            dev.run(0.05, 0.1, 1)
        ck, counts = dev.checkpoint()
        dev.set_param("stop_after_epochs", 0)
        for field, value in (("n", ck.n + 1), ("tau", ck.tau + 1), ("omega", ck.omega + 1), ("epochs", 0)):
            bad = Checkpoint.from_buffer_copy(bytes(ck))
            setattr(bad, field, value)
            with pytest.raises(KadabraError) as e:
                dev.resume(bad, counts)
            assert e.value.status == _lib.EINVAL, field
        wrong = counts.copy()
        wrong[0] += 1  # no longer sums to the increments
        with pytest.raises(KadabraError) as e:
            dev.resume(ck, wrong)
        assert e.value.status == _lib.EINVAL
        dev.set_param("balance", 1)
        with pytest.raises(KadabraError) as e:
            dev.resume(ck, counts)
        assert e.value.status == _lib.EINVAL
        dev.set_param("balance", 0)
        dev.resume(ck, counts)  # the good one still works
        _same(dev.result(), oracle.run(g, 0.05, 0.1, 1, 32))
    with Graph.from_csr(g) as dev:
        with pytest.raises(KadabraError) as e:
            dev.checkpoint()  # no stopped run
        assert e.value.status == _lib.ESTATE
