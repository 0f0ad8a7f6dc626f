"""Graph preprocessing on the device: component count and the vertex-diameter
bound VD equal the oracle's (its host BFS from each component's maximum-degree
vertex, lowest id on ties), on graphs that stress each kernel: long paths
(one-workgroup levels), many components, isolated vertices, hub-heavy graphs
(load-balanced arcs), and a large frontier (multi-workgroup levels)."""
import numpy as np
import pytest

import oracle
from paper_1903_09422_amd import Graph
from paper_1903_09422_amd import graphs as G

pytestmark = pytest.mark.gpu


def _cases():
    many = G.disjoint_union(*[G.path_graph(3 + (k % 7)) for k in range(300)])
    return [
        G.path_graph(2),
        G.path_graph(20000),                 # deepest BFS: 19,998 levels from vertex 1
        G.cycle_graph(5001),
        G.empty_graph(50),                   # 50 components, VD 1
        many,                                # 300 components of varied diameter
        G.disjoint_union(G.star_graph(2000), G.path_graph(40), G.complete_graph(30)),
        G.grid_graph(300, 200),              # frontiers of a few hundred vertices
        G.rmat(16, 16, seed=3),              # hubs; frontier > one workgroup's small limit
        G.random_connected(5000, 400, seed=9),
    ]


@pytest.mark.parametrize("g", _cases(), ids=lambda g: g.name)
def test_components_and_vd(g):
    print(f"case prep {g.name} n={g.n}", flush=True)
    k, _ = oracle.components(g)
    want_vd = oracle.setup(g, 0.1, 0.1)["vd"]
    with Graph.from_csr(g) as dev:
        assert dev.get_param("components") == k
        assert dev.get_param("vd_bound") == want_vd


def test_component_labels_separate_pairs():
    """Pairs in different components are counted without a search: a run on a
    union of components equals the oracle's, work counters included."""
    g = G.disjoint_union(G.grid_graph(15, 15), G.star_graph(40), G.cycle_graph(33), G.empty_graph(5))
    print("case prep labels", flush=True)
    want = oracle.run(g, 0.05, 0.1, 3, 128)
    with Graph.from_csr(g) as dev:
        dev.set_param("check_interval", 128)
        dev.run(0.05, 0.1, 3)
        got = dev.result()
    assert got.tau == want.tau and np.array_equal(got.counts, want.counts)
    assert got.stats["disconnected"] == want.stats["disconnected"] > 0
