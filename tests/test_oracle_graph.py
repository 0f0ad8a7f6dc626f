"""Pins for the oracle's graph routines: components, the diameter bound,
omega, distances and shortest-path counts (sigma).

Checkers: scipy csgraph, networkx brute-force path enumeration, and closed
forms (grid binomials, complete bipartite graphs, cycles, hypercubes).
"""
import math

import networkx as nx
import numpy as np
import pytest
from scipy.sparse.csgraph import connected_components, shortest_path

from paper_1903_09422_amd import graphs as G


def _nx(g):
    h = nx.Graph()
    h.add_nodes_from(range(g.n))
    h.add_edges_from(g.edge_list().tolist())
    return h


SMALL = [
    G.path_graph(7), G.cycle_graph(8), G.cycle_graph(9), G.star_graph(6), G.complete_graph(6),
    G.complete_bipartite(3, 4), G.grid_graph(4, 5), G.hypercube(4), G.barbell(5, 3),
    G.random_connected(40, 30, seed=2), G.random_connected(60, 10, seed=3),
    G.disjoint_union(G.path_graph(4), G.cycle_graph(5), G.star_graph(3)),
]


@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_components_match_scipy(oracle_mod, g):
    k, comp = oracle_mod.components(g)
    k2, lab = connected_components(g.to_scipy(), directed=False)
    assert k == k2
    # same partition; oracle numbers components by their lowest vertex
    for c in range(k):
        members = np.flatnonzero(comp == c)
        assert members.size and np.all(lab[members] == lab[members[0]])
        assert comp[: members[0]].max(initial=-1) < c


@pytest.mark.parametrize("n", [2, 3, 5, 10, 50])
def test_vd_path_closed_form(oracle_mod, n):
    # path 0-1-...-(n-1): the lowest-id maximum-degree vertex is 1 (0 if n == 2),
    # eccentricity n-2 (1 if n == 2), VD = 2 ecc + 1
    g = G.path_graph(n)
    info = oracle_mod.setup(g, 0.1, 0.1)
    ecc = 1 if n == 2 else n - 2
    assert info["vd"] == 2 * ecc + 1


def test_vd_other_closed_forms(oracle_mod):
    assert oracle_mod.setup(G.star_graph(9), 0.1, 0.1)["vd"] == 3
    assert oracle_mod.setup(G.cycle_graph(10), 0.1, 0.1)["vd"] == 11
    assert oracle_mod.setup(G.complete_graph(5), 0.1, 0.1)["vd"] == 3
    # components: the largest bound wins (path of 6: root 1, ecc 4 -> 9)
    u = G.disjoint_union(G.star_graph(4), G.path_graph(6))
    assert oracle_mod.setup(u, 0.1, 0.1)["vd"] == 9
    # no edges: every component is one vertex, ecc 0
    assert oracle_mod.setup(G.empty_graph(4), 0.1, 0.1)["vd"] == 1


@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_vd_is_a_valid_bound(oracle_mod, g):
    info = oracle_mod.setup(g, 0.1, 0.1)
    h = _nx(g)
    diam = max(nx.diameter(h.subgraph(c)) for c in nx.connected_components(h))
    assert info["vd"] >= diam + 1


@pytest.mark.parametrize("vd,k", [(1, 0), (2, 0), (3, 0), (4, 1), (5, 1), (6, 2), (9, 2),
                                  (10, 3), (11, 3), (18, 4), (213, 7)])
def test_omega_hand_values(oracle_mod, vd, k):
    # omega = ceil((0.5/eps^2) (floor(log2(max(VD-2,1))) + 1 + ln(2/delta)))
    for eps, delta in ((0.05, 0.1), (0.01, 0.1), (0.02, 0.05)):
        want = math.ceil(0.5 / (eps * eps) * (k + 1 + math.log(2 / delta)))
        assert oracle_mod.omega(vd, eps, delta) == want


def test_omega_paper_workloads(oracle_mod):
    # G(4096, 8) LCC: VD = 11 -> ceil(200 * (4 + ln 20)) = ceil(1399.15) = 1400
    assert oracle_mod.omega(11, 0.05, 0.1) == 1400
    assert oracle_mod.omega(11, 0.01, 0.1) == 34979


def test_log_inv_delta(oracle_mod):
    # uniform delta_L = delta / (4n): log(1/delta_L) = log(4n/delta)
    for n, d in ((2, 0.1), (4092, 0.1), (10**6, 0.01)):
        assert oracle_mod.log_inv_delta(n, d) == pytest.approx(math.log(4 * n / d), rel=1e-15)


@pytest.mark.parametrize("g", SMALL + [G.erdos_renyi(300, 4.0, seed=5)], ids=lambda g: g.name)
def test_bfs_distances_match_scipy(oracle_mod, g):
    ref = shortest_path(g.to_scipy(), method="D", unweighted=True, directed=False)
    for s in range(0, g.n, max(1, g.n // 12)):
        dist, _ = oracle_mod.bfs_sigma(g, s)
        want = np.where(np.isinf(ref[s]), -1, ref[s]).astype(np.int64)
        assert np.array_equal(dist.astype(np.int64), want)


@pytest.mark.parametrize("g", SMALL[:10], ids=lambda g: g.name)
def test_sigma_brute_force(oracle_mod, g):
    h = _nx(g)
    for s in range(g.n):
        dist, sig = oracle_mod.bfs_sigma(g, s)
        for t in range(g.n):
            if t == s or dist[t] < 0:
                continue
            assert sig[t] == len(list(nx.all_shortest_paths(h, s, t)))


def test_sigma_closed_forms(oracle_mod):
    g = G.grid_graph(9, 11)
    _, sig = oracle_mod.bfs_sigma(g, 0)
    for r in range(9):
        for c in range(11):
            assert sig[r * 11 + c] == math.comb(r + c, r)
    g = G.complete_bipartite(4, 7)
    _, sig = oracle_mod.bfs_sigma(g, 0)
    assert np.all(sig[1:4] == 7) and np.all(sig[4:] == 1)
    for n in (6, 10, 20):
        _, sig = oracle_mod.bfs_sigma(G.cycle_graph(n), 0)
        assert sig[n // 2] == 2
    for k in (3, 4, 6):
        _, sig = oracle_mod.bfs_sigma(G.hypercube(k), 0)
        assert sig[(1 << k) - 1] == math.factorial(k)
