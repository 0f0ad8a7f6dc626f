"""Input generators: canonical CSR invariants and pinned workload hashes."""
import json
import os

import numpy as np
import pytest
from scipy.sparse.csgraph import connected_components

from paper_1903_09422_amd import graphs as G

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def check_canonical(g, connected=True):
    rp, col = g.row_ptr, g.col
    assert rp.dtype == np.int32 and col.dtype == np.int32
    assert rp[0] == 0 and np.all(np.diff(rp) >= 0) and rp[-1] == col.size
    src = np.repeat(np.arange(g.n), np.diff(rp))
    assert np.all(src != col)                      # no self-loops
    for v in range(0, g.n, max(1, g.n // 2000)):   # rows strictly ascending
        row = col[rp[v]:rp[v + 1]]
        assert np.all(np.diff(row) > 0)
    a = g.to_scipy()
    assert (a != a.T).nnz == 0                     # symmetric
    if connected:
        assert connected_components(a, directed=False)[0] == 1


@pytest.mark.parametrize("name", sorted(G.WORKLOADS))
def test_workloads_match_manifest(name):
    with open(os.path.join(GOLDEN, "graphs_manifest.json")) as f:
        want = json.load(f)[name]
    g, eps, delta, n_check = G.workload(name)
    check_canonical(g)
    assert (g.n, g.num_arcs, int(g.degrees().max())) == (want["n"], want["arcs"], want["max_degree"])
    assert g.sha256() == want["sha256"]
    assert (eps, delta, n_check) == (want["eps"], want["delta"], want["check_interval"])


def test_small_generators_canonical():
    for g in (G.path_graph(5), G.cycle_graph(7), G.star_graph(4), G.complete_graph(5),
              G.complete_bipartite(2, 3), G.grid_graph(3, 4), G.hypercube(3), G.barbell(4, 2),
              G.random_connected(30, 20, seed=1)):
        check_canonical(g)
    check_canonical(G.disjoint_union(G.path_graph(3), G.star_graph(3)), connected=False)


def test_from_edges_canonicalises():
    g = G.from_edges(6, [0, 1, 1, 2, 3, 5, 5], [1, 0, 1, 3, 2, 4, 4], lcc=False)
    assert g.num_edges == 3
    check_canonical(g, connected=False)
    h = G.from_edges(6, [0, 1, 1, 2, 3, 5, 5], [1, 0, 1, 3, 2, 4, 4], lcc=True)
    assert h.n == 2 and h.num_edges == 1  # first largest component: {0, 1}


def test_generator_sizes():
    g = G.perturbed_grid(32, seed=3, lcc=False)
    e = 2 * 32 * 31
    assert g.num_edges == e - round(0.05 * e) + round(0.001 * e)
    r = G.rmat(10, 8, seed=2, lcc=False)
    assert r.n == 1024 and r.num_edges <= 8 * 1024


def test_rhg_matches_brute_force():
    """The banded candidate search finds exactly the pairs at hyperbolic
    distance <= R (all-pairs check on a small disk)."""
    rng = np.random.default_rng(4)
    n, alpha, R = 1500, 0.9, 11.0
    theta = rng.random(n) * 2 * np.pi
    r = np.arccosh(1.0 + (np.cosh(alpha * R) - 1.0) * rng.random(n)) / alpha
    eu, ev = G._rhg_edges(r, theta, R)
    got = set(zip(np.minimum(eu, ev).tolist(), np.maximum(eu, ev).tolist()))
    i, j = np.triu_indices(n, 1)
    cosd = np.cosh(r[i]) * np.cosh(r[j]) - np.sinh(r[i]) * np.sinh(r[j]) * np.cos(theta[i] - theta[j])
    want = set(zip(i[cosd <= np.cosh(R)].tolist(), j[cosd <= np.cosh(R)].tolist()))
    assert len(want) > 1000
    assert got == want


def test_rhg_mean_degree_and_shape():
    g = G.rhg(1 << 14, 10.0, 2.8, seed=3, lcc=False)
    check_canonical(g, connected=False)
    assert abs(g.num_arcs / g.n - 10.0) <= 0.5
    deg = g.degrees()
    assert deg.max() > 20 * deg.mean()  # heavy-tailed


def test_serve_trace_deterministic_and_shaped():
    q1, g1 = G.serve_trace(66, 256, seed=8)
    q2, g2 = G.serve_trace(66, 256, seed=8)
    assert q1 == q2 and np.array_equal(g1, g2)
    assert len(q1) == 256 and g1[0] == 0.0 and np.all(g1[1:] > 0)
    gi = np.array([q[0] for q in q1])
    assert gi.min() >= 0 and gi.max() < 66 and len(set(gi.tolist())) > 40
    assert {q[1] for q in q1} == {0.05, 0.01}
    assert all(q[2] == 0.1 and q[3] == 16384 for q in q1)
    assert len({q[4] for q in q1}) == 256  # distinct sampling seeds
    # unit-rate exponential gaps: mean near 1
    assert 0.8 < float(np.mean(g1[1:])) < 1.2
    q3, _ = G.serve_trace(66, 256, seed=9)
    assert q3 != q1
