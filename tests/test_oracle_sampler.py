"""Pins for the oracle's KADABRA sample (Section 2.3) and exact betweenness.

* the bidirectional search finds d(s, t) (scipy) and sigma_st (networkx brute
  force / unidirectional BFS), and every sampled path is a shortest path;
* the path law is uniform over the shortest s-t paths (chi-square over
  enumerated paths);
* exact Brandes betweenness matches networkx and closed forms;
* the estimator is unbiased: the counters of many samples converge to the
  normalised betweenness (per-vertex z test);
* sigma is exact below 2^104 and, beyond, stays within the rounding bound of
  its level rescaling against Python's exact integers.
"""
import math
from collections import Counter, defaultdict

import networkx as nx
import numpy as np
import pytest
from scipy import stats
from scipy.sparse.csgraph import shortest_path

from paper_1903_09422_amd import graphs as G


def _nx(g):
    h = nx.Graph()
    h.add_nodes_from(range(g.n))
    h.add_edges_from(g.edge_list().tolist())
    return h


GRAPHS = [
    G.grid_graph(4, 4), G.hypercube(4), G.cycle_graph(10), G.complete_bipartite(3, 5),
    G.barbell(4, 2), G.random_connected(50, 60, seed=7), G.erdos_renyi(120, 5.0, seed=3),
    G.disjoint_union(G.grid_graph(3, 3), G.cycle_graph(6)),
]


@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: g.name)
def test_sample_is_a_shortest_path(oracle_mod, g):
    _, comp = oracle_mod.components(g)
    dist = shortest_path(g.to_scipy(), method="D", unweighted=True, directed=False)
    adj = g.to_scipy().tolil().rows
    for i in range(400):
        interior, info = oracle_mod.sample(g, comp, 17, i)
        s, t = info.s, info.t
        if np.isinf(dist[s, t]):
            assert interior is None and info.d == -1
            continue
        d = int(dist[s, t])
        assert info.d == d
        assert len(interior) == d - 1
        assert len(set(interior.tolist())) == d - 1
        # order the interior by distance from s and check it is an s-t walk of length d
        verts = sorted(interior.tolist(), key=lambda v: dist[s, v])
        walk = [s] + verts + [t]
        assert [int(dist[s, v]) for v in walk] == list(range(d + 1))
        for a, b in zip(walk[:-1], walk[1:]):
            assert b in adj[a]


@pytest.mark.parametrize("g", GRAPHS, ids=lambda g: g.name)
def test_bidirectional_sigma_equals_exact(oracle_mod, g):
    """sigma_st from the meeting set (sum of sigma_s sigma_t) equals the
    unidirectional count; all these graphs stay below 2^40, so it is exact."""
    _, comp = oracle_mod.components(g)
    for i in range(300):
        _, info = oracle_mod.sample(g, comp, 23, i)
        if info.d < 0:
            continue
        _, sig = oracle_mod.bfs_sigma(g, info.s)
        assert info.sigma_scale == 0
        assert info.sigma == int(sig[info.t])
        assert 1 <= info.meet_size


def test_sigma_against_networkx_enumeration(oracle_mod):
    g = G.random_connected(30, 45, seed=11)
    h = _nx(g)
    _, comp = oracle_mod.components(g)
    for i in range(200):
        _, info = oracle_mod.sample(g, comp, 5, i)
        assert info.sigma == len(list(nx.all_shortest_paths(h, info.s, info.t)))


def _path_law_chi2(oracle_mod, g, samples, seed):
    h = _nx(g)
    _, comp = oracle_mod.components(g)
    seen = defaultdict(Counter)
    for i in range(samples):
        interior, info = oracle_mod.sample(g, comp, seed, i)
        seen[(info.s, info.t)][frozenset(interior.tolist())] += 1
    chi2, dof = 0.0, 0
    for (s, t), cnt in seen.items():
        paths = {frozenset(p[1:-1]) for p in nx.all_shortest_paths(h, s, t)}
        assert set(cnt) <= paths  # only shortest paths are ever drawn
        if len(paths) == 1:
            continue
        tot = sum(cnt.values())
        exp = tot / len(paths)
        chi2 += sum((cnt.get(p, 0) - exp) ** 2 / exp for p in paths)
        dof += len(paths) - 1
    return chi2, dof


@pytest.mark.parametrize("g,samples", [(G.hypercube(4), 240_000), (G.grid_graph(4, 4), 160_000)],
                         ids=["Q4", "grid4x4"])
def test_path_law_uniform(oracle_mod, g, samples):
    chi2, dof = _path_law_chi2(oracle_mod, g, samples, seed=3)
    p = stats.chi2.sf(chi2, dof)
    assert p > 1e-4, (chi2, dof, p)


# -------------------------------------------------------------------------
# exact betweenness
# -------------------------------------------------------------------------

@pytest.mark.parametrize("g", GRAPHS + [G.star_graph(7), G.path_graph(9)], ids=lambda g: g.name)
def test_brandes_matches_networkx(oracle_mod, g):
    bc = oracle_mod.brandes(g)
    ref = nx.betweenness_centrality(_nx(g), normalized=False)
    # networkx sums over unordered pairs; the normalised quantity here sums over
    # ordered pairs and divides by n(n-1)
    want = np.array([2.0 * ref[v] / (g.n * (g.n - 1)) for v in range(g.n)])
    np.testing.assert_allclose(bc, want, rtol=1e-12, atol=1e-15)


def test_brandes_closed_forms(oracle_mod):
    for k in (2, 5, 30):
        bc = oracle_mod.brandes(G.star_graph(k))
        assert bc[0] == pytest.approx((k - 1) / (k + 1), rel=1e-14)
        assert np.all(bc[1:] == 0)
    bc = oracle_mod.brandes(G.path_graph(3))
    assert bc[1] == pytest.approx(1 / 3, rel=1e-14)
    assert oracle_mod.brandes(G.complete_graph(6)).max() == 0


# -------------------------------------------------------------------------
# unbiasedness of the estimator (Section 2.3): E[x_i(v)] = b(v)
# -------------------------------------------------------------------------

@pytest.mark.parametrize("g,m", [(G.erdos_renyi(150, 4.0, seed=9), 300_000),
                                 (G.grid_graph(8, 8), 200_000),
                                 (G.disjoint_union(G.star_graph(8), G.grid_graph(4, 4)), 200_000)],
                         ids=["er150", "grid8", "union"])
def test_estimator_unbiased(oracle_mod, g, m):
    _, comp = oracle_mod.components(g)
    _, acc = oracle_mod.accumulate(g, comp, 99, 0, m)
    b = oracle_mod.brandes(g)
    # x_i(v) is Bernoulli(b(v)): the count is Binomial(m, b(v))
    var = m * b * (1 - b)
    z = np.where(var > 0, (acc - m * b) / np.sqrt(np.maximum(var, 1e-300)), acc - m * b)
    assert np.all(acc[b == 0] == 0)
    assert np.abs(z).max() < 5.0, np.abs(z).max()


# -------------------------------------------------------------------------
# sigma beyond 2^104: the level rescaling
# -------------------------------------------------------------------------

def layered_graph(layers: int, width: int) -> "G.CSR":
    """``layers`` groups of ``width`` vertices, consecutive groups joined
    completely: a vertex in group a and one in group b != a are at distance
    |a - b| with exactly width^(|a - b| - 1) shortest paths."""
    u, v = [], []
    for a in range(layers - 1):
        for i in range(width):
            for j in range(width):
                u.append(a * width + i)
                v.append((a + 1) * width + j)
    return G.from_edges(layers * width, u, v, lcc=False, name=f"layers{layers}x{width}")


def test_sigma_exact_below_2_104(oracle_mod):
    # 64 x 64 grid: sigma up to C(63, 31) ~ 2^60 per side, exact
    g = G.grid_graph(64, 64)
    _, comp = oracle_mod.components(g)
    for i in range(60):
        _, info = oracle_mod.sample(g, comp, 1, i)
        _, sig = oracle_mod.bfs_sigma(g, info.s)
        assert info.sigma_scale == 0
        if sig[info.t] < 2**53:
            assert info.sigma == int(sig[info.t])


def test_sigma_rescaled_levels_bound(oracle_mod):
    width, layers = 17, 80
    g = layered_graph(layers, width)
    _, comp = oracle_mod.components(g)
    rescaled = 0
    for i in range(400):
        _, info = oracle_mod.sample(g, comp, 4, i)
        a, b = info.s // width, info.t // width
        if a == b:
            # two vertices of one group: one path through each neighbouring group's vertex
            assert info.d == 2 and info.sigma == width * ((a > 0) + (a < layers - 1))
            continue
        exact = width ** (abs(a - b) - 1)
        assert info.d == abs(a - b)
        est = info.sigma << info.sigma_scale
        if info.sigma_scale == 0:
            assert est == exact
        else:
            rescaled += 1
            # every level is rounded up once by less than one unit of a >= 2^103
            # mantissa, and all vertices of a level carry the same count here
            assert exact <= est
            assert (est - exact) / exact < info.d * 2.0**-102
    assert rescaled >= 10  # the test reaches the rescaled regime
