"""kadabra_run_static (the run whose device state lives in the library's
static array, for callers that cannot allocate) against kadabra_run.

Bar: bit-exact tau, decision, every counter and every work counter, on two
calls in a row, the second on a smaller graph (so the array holds the first
call's larger state when the second starts), and once more on the first graph
afterwards.  The size limit is rejected with ERANGE before any device work.
"""
import numpy as np
import pytest

import oracle
from paper_1903_09422_amd import Graph, KadabraError, _lib
from paper_1903_09422_amd import graphs as G

pytestmark = pytest.mark.gpu

WORK_KEYS = ("v_exp", "e_scan", "e_bt", "path_interior", "disconnected")


def _static_equals_run(dev, g, eps, delta, seed, n_check):
    import torch

    dev.set_param("check_interval", n_check)
    dev.run(eps, delta, seed)
    want = dev.result()
    counts = torch.full((g.n,), -7, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()  # the fill is on torch's stream, the run on the handle's
    stats = dev.run_static(eps, delta, seed, counts)
    got = counts.cpu().numpy()
    assert stats["tau"] == want.tau
    assert stats["decision"] == want.stats["decision"]
    assert stats["epochs"] == len(want.decisions)
    assert stats["omega"] == want.stats["omega"]
    for k in WORK_KEYS:
        assert stats[k] == want.stats[k], k
    if not np.array_equal(got, want.counts):
        bad = np.flatnonzero(got != want.counts)
        raise AssertionError(f"{bad.size} counters differ, first {bad[:5]}: static {got[bad[:5]]} "
                             f"run {want.counts[bad[:5]]}")
    # the handle's own last result is left as kadabra_run wrote it
    assert np.array_equal(dev.result().counts, want.counts)
    return stats, want


def test_static_run_equals_run_twice_then_smaller():
    big = G.erdos_renyi(4096, 8.0, seed=1)  # 4,092 vertices
    small = G.grid_graph(30, 30)             # 900 vertices, relabelled (bound >= 64)
    print("case static er4096 then grid30", flush=True)
    with Graph.from_csr(big) as dbig, Graph.from_csr(small) as dsmall:
        assert dsmall.get_param("relabeled") == 1
        s1, w1 = _static_equals_run(dbig, big, 0.05, 0.1, 1, 1024)
        s2, w2 = _static_equals_run(dsmall, small, 0.1, 0.1, 3, 256)
        # and the oracle agrees with both
        o1 = oracle.run(big, 0.05, 0.1, 1, 1024)
        o2 = oracle.run(small, 0.1, 0.1, 3, 256)
        assert (s1["tau"], s2["tau"]) == (o1.tau, o2.tau)
        assert np.array_equal(w1.counts, o1.counts) and np.array_equal(w2.counts, o2.counts)
        # the larger graph again, with a few slots and a 64-lane team
        dbig.set_param("slots", 37)
        dbig.set_param("team", 64)
        _static_equals_run(dbig, big, 0.05, 0.1, 1, 1024)


def test_static_run_rejects_what_does_not_fit():
    import torch

    # one sample in flight of a 4.6M-vertex star needs more than the 256 MiB array
    g = G.star_graph(4_600_000)
    print("case static star 4.6M (ERANGE)", flush=True)
    with Graph.from_csr(g) as dev:
        counts = torch.zeros(g.n, dtype=torch.int32, device="cuda")
        torch.cuda.synchronize()
        with pytest.raises(KadabraError) as ei:
            dev.run_static(0.1, 0.1, 1, counts)
        assert ei.value.status == _lib.ERANGE
        assert "static array" in str(ei.value)
        dev.set_param("balance", 1)
        with pytest.raises(KadabraError) as ei:
            dev.run_static(0.1, 0.1, 1, counts)
        assert ei.value.status == _lib.EINVAL
