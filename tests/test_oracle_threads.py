"""The threaded run of the oracle (the CPU baseline on all host cores): each
epoch's samples are split by index over per-thread counter frames, added into
the counters at the boundary before the check (the local frames of Section 3
with the indexed-frame assignment of Appendix D.2).  Sample i depends on i
alone and every sum is an integer sum, so tau, the decisions, every counter
and every work counter equal the single-threaded run for any thread count."""
import numpy as np
import pytest

from paper_1903_09422_amd import graphs as G

CASES = [
    (G.erdos_renyi(4096, 8.0, seed=1), 0.05, 1024),    # stops by the rule at the first boundary
    (G.grid_graph(20, 20), 0.05, 64),                  # stops by the rule after several boundaries
    (G.star_graph(40), 0.1, 7),                        # runs to omega (a ragged last epoch)
    (G.disjoint_union(G.grid_graph(5, 5), G.path_graph(9)), 0.1, 100),  # disconnected pairs
    (G.rmat(11, 16, seed=6), 0.05, 333),
]


@pytest.mark.parametrize("threads", [1, 2, 3, 8])
@pytest.mark.parametrize("case", range(len(CASES)))
def test_threads_equal_single_thread(oracle_mod, case, threads):
    g, eps, n_check = CASES[case]
    want = oracle_mod.run(g, eps, 0.1, 3, n_check)
    got = oracle_mod.run_threads(g, eps, 0.1, 3, n_check, threads)
    assert got.tau == want.tau
    assert np.array_equal(got.decisions, want.decisions)
    assert np.array_equal(got.counts, want.counts)
    for k in ("omega", "vd", "epochs", "v_exp", "e_scan", "v_new", "e_pred", "e_bt", "path_interior",
              "disconnected", "rescaled_levels"):
        assert got.stats[k] == want.stats[k], k


def test_threads_more_than_samples(oracle_mod):
    # more threads than samples in an epoch: some threads draw nothing
    g = G.cycle_graph(12)
    want = oracle_mod.run(g, 0.2, 0.1, 5, 3)
    got = oracle_mod.run_threads(g, 0.2, 0.1, 5, 3, 16)
    assert got.tau == want.tau and np.array_equal(got.counts, want.counts)


def test_threads_bad_arguments(oracle_mod):
    g = G.path_graph(10)
    for threads in (0, -1, 2000):
        with pytest.raises(ValueError):
            oracle_mod.run_threads(g, 0.1, 0.1, 1, 10, threads)
