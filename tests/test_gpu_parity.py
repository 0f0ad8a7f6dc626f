"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: bit-exact tau, per-boundary decisions, every counter and every
algorithm-defined work counter (integer work), for every graph, seed, check
interval and mapping (team, slots, frames, overlap).
"""
import hashlib
import json
import os
import threading
import time

import numpy as np
import pytest

import oracle
from paper_1903_09422_amd import Graph, KadabraError, _lib, eval_stop_fg
from paper_1903_09422_amd import graphs as G

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
WORK_KEYS = ("v_exp", "e_scan", "e_bt", "path_interior", "disconnected")


def gpu_run(g, eps, delta, seed, n_check, **params):
    with Graph.from_csr(g) as dev:
        dev.set_param("check_interval", n_check)
        for k, v in params.items():
            dev.set_param(k, v)
        dev.run(eps, delta, seed)
        return dev.result()


def assert_same(got, want):
    assert got.tau == want.tau
    assert np.array_equal(got.decisions, want.decisions)
    if not np.array_equal(got.counts, want.counts):
        bad = np.flatnonzero(got.counts != want.counts)
        raise AssertionError(f"{bad.size} counters differ, first {bad[:5]}: "
                             f"gpu {got.counts[bad[:5]]} oracle {want.counts[bad[:5]]}")
    for k in WORK_KEYS:
        assert got.stats[k] == want.stats[k], k
    assert got.stats["omega"] == want.stats["omega"]
    assert got.stats["vd_bound"] == want.stats["vd"]
    np.testing.assert_array_equal(got.scores, want.counts / float(want.tau))


SMALL = [
    G.path_graph(2), G.path_graph(40), G.star_graph(25), G.complete_graph(9), G.cycle_graph(31),
    G.grid_graph(12, 9), G.hypercube(6), G.barbell(7, 6), G.complete_bipartite(5, 8),
    G.empty_graph(6), G.disjoint_union(G.grid_graph(5, 5), G.star_graph(12), G.path_graph(3)),
    G.erdos_renyi(700, 7.0, seed=2), G.random_connected(300, 50, seed=4),
]


@pytest.mark.parametrize("team,probe", [(64, -1), (128, -1), (256, -1), (512, -1), (64, 0), (128, 0), (256, 0)])
@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_small_graphs(g, team, probe):
    print(f"case {g.name} team={team} probe_min={probe}", flush=True)
    for seed, n_check in ((1, 64), (9, 333)):
        want = oracle.run(g, 0.05, 0.1, seed, n_check)
        got = gpu_run(g, 0.05, 0.1, seed, n_check, team=team, probe_min=probe)
        assert_same(got, want)


@pytest.mark.parametrize("probe", [-1, 0])
@pytest.mark.parametrize("g", SMALL, ids=lambda g: g.name)
def test_small_graphs_pull_probe(g, probe):
    """The pull form of the meeting probe gives the oracle's result."""
    print(f"case {g.name} pull probe, probe_min={probe}", flush=True)
    for seed, n_check in ((1, 64), (9, 333)):
        want = oracle.run(g, 0.05, 0.1, seed, n_check)
        got = gpu_run(g, 0.05, 0.1, seed, n_check, team=256, probe_min=probe, probe_pull=1)
        assert_same(got, want)


@pytest.mark.parametrize("n_check", [1, 7, 1000, 10**6])
def test_check_intervals_and_ragged_last_epoch(n_check):
    """Every check interval, with one to four epochs per sampling launch (a run
    may stop at any boundary inside a launch, and at omega mid-launch)."""
    g = G.erdos_renyi(400, 5.0, seed=8)
    print(f"case er400 n_check={n_check}", flush=True)
    want = oracle.run(g, 0.04, 0.1, 3, n_check)
    for epl, overlap in ((2, 1), (1, 1), (3, 1), (4, 0), (4, 1)):
        got = gpu_run(g, 0.04, 0.1, 3, n_check, epochs_per_launch=epl, overlap=overlap)
        assert_same(got, want)


def _double_star(a, b):
    """Centers 0 and 1 adjacent; a leaves on 0, b leaves on 1."""
    u = [0] + [0] * a + [1] * b
    v = [1] + list(range(2, 2 + a)) + list(range(2 + a, 2 + a + b))
    return G.from_edges(2 + a + b, np.array(u), np.array(v), name=f"dstar{a}_{b}")


def _layered(a, b):
    """Vertex 0 joined to a layer of a vertices, each joined to all of a layer
    of b vertices: every vertex of the last layer has a predecessors."""
    u = [0] * a
    v = list(range(1, 1 + a))
    for i in range(1, 1 + a):
        u += [i] * b
        v += list(range(1 + a, 1 + a + b))
    return G.from_edges(1 + a + b, np.array(u), np.array(v), name=f"layered{a}_{b}")


@pytest.mark.parametrize("team", [64, 256])
@pytest.mark.parametrize("probe", [-1, 1 << 40])
def test_level_sigma_paths(team, probe):
    """A full level sums sigma in LDS for its first STAGE/2 new vertices and in
    global memory past them: levels of up to 1500 leaves with one predecessor
    each (a center's expansion with the probe off), levels whose vertices have
    many predecessors over many rounds of arcs and over several frontier chunks
    (layered graphs, a complete bipartite graph), and multi-chunk levels (a
    grid's wide rings), with the meeting probe on (auto) and off."""
    # double stars: with the probe off, the smaller center is expanded in
    # full: 1000 or 600 new vertices (past STAGE/2 for any team) or 300
    cases = [(_double_star(1500, 1000), 0.1, 100), (_double_star(700, 600), 0.1, 100),
             (_double_star(400, 300), 0.1, 64), (G.grid_graph(40, 40), 0.05, 200),
             (G.complete_bipartite(3, 700), 0.1, 50), (_layered(150, 400), 0.1, 100),
             (_layered(60, 1200), 0.1, 100)]
    for g, eps, n_check in cases:
        print(f"case {g.name} team={team} probe_min={probe}", flush=True)
        for seed in (2, 3):
            want = oracle.run(g, eps, 0.1, seed, n_check)
            assert_same(gpu_run(g, eps, 0.1, seed, n_check, team=team, probe_min=probe), want)


def _broom(handle, leaves):
    """A path of `handle` vertices whose last vertex is the center of a star."""
    u = list(range(handle - 1)) + [handle - 1] * leaves
    v = list(range(1, handle)) + list(range(handle, handle + leaves))
    return G.from_edges(handle + leaves, np.array(u), np.array(v), name=f"broom{handle}_{leaves}")


@pytest.mark.parametrize("team", [64, 256])
def test_relabelled_graphs(team):
    """High-diameter graphs run in an internal vertex order (BFS-grown
    clusters seeded in reverse Cuthill-McKee order) with every tie still
    broken by original id: the results
    equal the oracle's.  Meeting sets larger than a 64-lane team (grid), and
    backtracking through a hub by the level-list search (broom)."""
    cases = [(G.cycle_graph(300), 0.05, 128), (G.path_graph(200), 0.05, 100),
             (G.grid_graph(100, 100), 0.05, 256), (_broom(100, 500), 0.05, 128),
             (G.disjoint_union(G.path_graph(150), G.grid_graph(9, 9)), 0.05, 64)]
    for g, eps, n_check in cases:
        print(f"case relabelled {g.name} team={team}", flush=True)
        with Graph.from_csr(g) as dev:
            assert dev.get_param("relabeled") == 1
        for seed in (1, 6):
            assert_same(gpu_run(g, eps, 0.1, seed, n_check, team=team), oracle.run(g, eps, 0.1, seed, n_check))
    with Graph.from_csr(G.erdos_renyi(500, 6.0, seed=3)) as dev:
        assert dev.get_param("relabeled") == 0  # low diameter: original order


def test_layered_graph_with_huge_sigma():
    # 17^(d-1) shortest paths: sigma beyond 2^104 forces level rescaling
    width, layers = 17, 80
    u, v = [], []
    for a in range(layers - 1):
        for i in range(width):
            for j in range(width):
                u.append(a * width + i)
                v.append((a + 1) * width + j)
    g = G.from_edges(layers * width, u, v, lcc=False)
    print("case layered 80x17", flush=True)
    want = oracle.run(g, 0.05, 0.1, 2, 512)
    for team, probe, pull in ((64, -1, 0), (256, -1, 0), (256, 0, 0), (256, 0, 1)):
        got = gpu_run(g, 0.05, 0.1, 2, 512, team=team, probe_min=probe, probe_pull=pull)
        assert_same(got, want)


def test_er4096_workload():
    g, eps, delta, n_check = G.workload("er4096")
    print("case er4096 full", flush=True)
    want = oracle.run(g, eps, delta, 1, n_check)
    for team in (64, 128, 256, 512):
        assert_same(gpu_run(g, eps, delta, 1, n_check, team=team), want)


def test_rmat18_workload_full():
    g, eps, delta, n_check = G.workload("rmat18")
    print("case rmat18 full (oracle ~5 s)", flush=True)
    want = oracle.run(g, eps, delta, 1, n_check)
    got = gpu_run(g, eps, delta, 1, n_check)
    assert_same(got, want)


def _golden(name):
    with open(os.path.join(GOLDEN, "oracle_runs.json")) as f:
        return json.load(f)[name]


@pytest.mark.parametrize("name", ["rmat18", "pgrid1024"])
def test_workload_against_stored_oracle(name):
    """Full-size runs against the oracle's stored result (written by
    tests/golden/make_oracle_golden.py, which calls only oracle/)."""
    ref = _golden(name)
    g, eps, delta, n_check = G.workload(name)
    assert g.sha256() == ref["graph_sha256"]
    print(f"case {name} stored oracle result", flush=True)
    got = gpu_run(g, eps, delta, ref["seed"], n_check)
    assert got.tau == ref["tau"]
    assert got.decisions.tolist() == ref["decisions"]
    idx = np.asarray(ref["sample_idx"])
    assert got.counts[idx].tolist() == ref["sample_counts"]
    assert int(got.counts.sum()) == ref["counts_sum"]
    assert hashlib.sha256(got.counts.astype("<i4").tobytes()).hexdigest() == ref["counts_sha256"]
    for k in WORK_KEYS:
        assert got.stats[k] == ref["stats"][k], k


def test_mapping_does_not_change_results():
    """Every mapping knob on R-MAT-18 gives the oracle's stored result."""
    g, eps, delta, n_check = G.workload("rmat18")
    with open(os.path.join(GOLDEN, "oracle_runs.json")) as f:
        ref = json.load(f)["rmat18"]
    print("case rmat18 mappings", flush=True)
    base = gpu_run(g, eps, delta, ref["seed"], n_check, team=256)
    assert base.tau == ref["tau"]
    assert hashlib.sha256(base.counts.astype("<i4").tobytes()).hexdigest() == ref["counts_sha256"]
    for k in WORK_KEYS:
        assert base.stats[k] == ref["stats"][k], k
    for params in ({"team": 64}, {"team": 128}, {"team": 512}, {"team": 256, "slots": 37}, {"team": 64, "slots": 1000},
                   {"team": 128, "slots": 2048}, {"epochs_per_launch": 1}, {"epochs_per_launch": 3},
                   {"epochs_per_launch": 4, "overlap": 0},
                   {"frames": 8}, {"overlap": 0}, {"team": 64, "frames": 3, "overlap": 0},
                   {"probe_min": 0}, {"probe_min": 1 << 40}, {"team": 64, "probe_min": 0},
                   {"team": 256, "probe_pull": 1}, {"team": 256, "probe_pull": 1, "probe_min": 0}, {}):
        print("  mapping", params, flush=True)
        got = gpu_run(g, eps, delta, ref["seed"], n_check, **params)
        assert got.tau == base.tau and np.array_equal(got.counts, base.counts), params
        for k in WORK_KEYS:
            assert got.stats[k] == base.stats[k], (params, k)


def test_repeated_runs_on_one_handle():
    g = G.erdos_renyi(1500, 6.0, seed=5)
    print("case repeated runs", flush=True)
    with Graph.from_csr(g) as dev:
        dev.set_param("check_interval", 128)
        for seed in (1, 2, 1):
            dev.run(0.03, 0.1, seed)
            got = dev.result()
            assert_same(got, oracle.run(g, 0.03, 0.1, seed, 128))
        dev.set_param("team", 64)  # new buffers, same results
        dev.run(0.03, 0.1, 2)
        assert_same(dev.result(), oracle.run(g, 0.03, 0.1, 2, 128))


def test_stop_functions_bitwise():
    """The device f, g (IEEE double, no contraction) equal the oracle's bit for
    bit on 10^7 inputs: 40 draws of (omega, tau, L), omega log-uniform below
    2^31, tau = omega, tau = 1 or uniform, L = log(4n/delta) over n < 2^23,
    each with 250,000 counters (half uniform in [0, tau], half in the small
    range [0, min(tau, 64)] where most counters lie, and both ends)."""
    rng = np.random.default_rng(0)
    total = 0
    for call in range(40):
        omega = min(int(np.exp(rng.uniform(0.0, np.log(2.0**31 - 2)))) + 1, 2**31 - 1)
        tau = omega if call % 10 == 0 else (1 if call % 10 == 1 else int(rng.integers(1, omega + 1)))
        L = float(np.log(4 * int(rng.integers(2, 2**23)) / rng.uniform(0.001, 0.999)))
        m = 250_000
        counts = np.concatenate([rng.integers(0, tau + 1, size=m // 2),
                                 rng.integers(0, min(tau, 64) + 1, size=m - m // 2)]).astype(np.int32)
        counts[:2] = (0, tau)
        f, g = eval_stop_fg(counts, tau, omega, L)
        fo, go = oracle.fg_batch(counts, tau, omega, L)
        for got, want, name in ((f, fo, "f"), (g, go, "g")):
            if not np.array_equal(got.view(np.uint64), want.view(np.uint64)):
                k = int(np.flatnonzero(got.view(np.uint64) != want.view(np.uint64))[0])
                raise AssertionError(f"{name} differs at c={counts[k]} tau={tau} omega={omega} L={L!r}: "
                                     f"device {got[k]!r} oracle {want[k]!r}")
        total += m
    assert total == 10**7


def test_errors_and_state():
    g = G.grid_graph(6, 6)
    with Graph.from_csr(g) as dev:
        with pytest.raises(KadabraError) as e:
            dev.result()
        assert e.value.status == _lib.ESTATE
        for eps, delta in ((0.0, 0.1), (1.5, 0.1), (0.1, 0.0), (0.1, 1.0)):
            with pytest.raises(KadabraError) as e:
                dev.run(eps, delta, 1)
            assert e.value.status == _lib.EINVAL
        with pytest.raises(KadabraError) as e:
            dev.run(1e-6, 0.1, 1)  # omega beyond int32 counters
        assert e.value.status == _lib.ERANGE
        with pytest.raises(KadabraError) as e:
            dev.set_param("nonsense", 1)
        assert e.value.status == _lib.EINVAL
        with pytest.raises(KadabraError):
            dev.set_param("team", 96)
        # forced allocation failure: ENOMEM, no result, handle still usable
        dev.set_param("test_fail_alloc", 3)
        with pytest.raises(KadabraError) as e:
            dev.run(0.1, 0.1, 1)
        assert e.value.status == _lib.ENOMEM
        with pytest.raises(KadabraError) as e:
            dev.result()
        assert e.value.status == _lib.ESTATE
        dev.run(0.1, 0.1, 1)
        assert_same(dev.result(), oracle.run(g, 0.1, 0.1, 1, 1024))


def test_allocation_failure_at_every_point():
    """The k-th device allocation of a first run fails (k = 1, 2, ...: the
    sample pool, launch tables, control blocks, per-query buffers): the run
    returns ENOMEM and leaves no result, and the same handle's next run equals
    the oracle; past the last allocation the run simply succeeds."""
    g = G.erdos_renyi(300, 5.0, seed=8)
    want = oracle.run(g, 0.1, 0.1, 2, 256)
    print("case allocation failure sweep", flush=True)
    failures = 0
    for k in range(1, 60):
        with Graph.from_csr(g) as dev:
            dev.set_param("check_interval", 256)
            dev.set_param("test_fail_alloc", k)
            try:
                dev.run(0.1, 0.1, 2)
            except KadabraError as e:
                assert e.status == _lib.ENOMEM
                failures += 1
                with pytest.raises(KadabraError):
                    dev.result()
                dev.run(0.1, 0.1, 2)
            assert_same(dev.result(), want)
    assert 5 < failures < 59  # every allocation point was hit, then the runs succeed


def test_device_check_failure_reported_and_recoverable():
    """A device-side check that fails (forced from the host: room for only 3 BFS
    levels per side) ends the run with EDEVICE naming the check; the handle
    stays usable and its next run equals the oracle."""
    g = G.path_graph(40)
    print("case device check failure", flush=True)
    want = oracle.run(g, 0.1, 0.1, 3, 64)
    with Graph.from_csr(g) as dev:
        dev.set_param("check_interval", 64)
        dev.set_param("test_level_cap", 3)
        assert dev.get_param("test_level_cap") == 3
        with pytest.raises(KadabraError) as e:
            dev.run(0.1, 0.1, 3)
        assert e.value.status == _lib.EDEVICE
        assert "vertex-diameter bound" in str(e.value) and "seed 3" in str(e.value)
        with pytest.raises(KadabraError) as e:
            dev.result()
        assert e.value.status == _lib.ESTATE
        dev.set_param("test_level_cap", 0)
        dev.run(0.1, 0.1, 3)
        assert_same(dev.result(), want)
    with Graph.from_csr(g) as dev:
        for bad in (1, 2, -1):
            with pytest.raises(KadabraError):
                dev.set_param("test_level_cap", bad)


def test_cancel_from_another_thread():
    g, _, _, _ = G.workload("pgrid1024")
    print("case cancel", flush=True)
    with Graph.from_csr(g) as dev:
        dev.set_param("check_interval", 64)  # many boundaries
        th = threading.Timer(0.3, dev.cancel)
        th.start()
        t0 = time.time()
        with pytest.raises(KadabraError) as e:
            dev.run(0.002, 0.1, 1)  # omega ~ 1.4M samples: far longer than 0.3 s
        th.join()
        assert e.value.status == _lib.ECANCELED
        assert time.time() - t0 < 30
        with pytest.raises(KadabraError):
            dev.result()


def test_torch_stream_and_device_outputs():
    torch = pytest.importorskip("torch")
    g = G.erdos_renyi(900, 6.0, seed=6)
    want = oracle.run(g, 0.05, 0.1, 4, 256)
    stream = torch.cuda.Stream()
    with Graph.from_csr(g) as dev:
        dev.set_stream(stream)
        dev.set_param("check_interval", 256)
        dev.run(0.05, 0.1, 4)
        scores = torch.empty(g.n, dtype=torch.float64, device="cuda")
        counts = torch.empty(g.n, dtype=torch.int32, device="cuda")
        dev.result_device(scores=scores, counts=counts)
        stream.synchronize()
        assert np.array_equal(counts.cpu().numpy(), want.counts)
        assert np.array_equal(scores.cpu().numpy(), want.counts / float(want.tau))
