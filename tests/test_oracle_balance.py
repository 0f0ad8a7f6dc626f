"""Pins for the oracle's balancing of delta_L(v), delta_U(v) (the step before
the adaptive loop; Section 2.3 requires only that their sum stays within
delta).

The planning constants are pinned by what they are meant to be: L_f (L_g) is
the largest log(1/delta) for which f (g) of Appendix B stays <= eps at the
planned sample count; this is checked against a numerical inversion of f and
g, not against the closed form.  The budget is pinned by its sum, the floor
share by its cap, the first phase by the sample indices it draws (a stream the
adaptive loop never reaches), and the whole rule by the (eps, delta)
guarantee against exact betweenness.
"""
import json
import math
import os

import numpy as np
import pytest

from paper_1903_09422_amd import graphs as G

BETA = 0.1  # floor share of the budget
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _invert(fn, eps, hi=1e6):
    """Largest L in (0, hi] with fn(L) <= eps (fn increasing), by bisection in
    log space; hi if fn(hi) <= eps."""
    if fn(hi) <= eps:
        return hi
    lo_l, hi_l = math.log(1e-12), math.log(hi)
    for _ in range(200):
        mid = 0.5 * (lo_l + hi_l)
        if fn(math.exp(mid)) <= eps:
            lo_l = mid
        else:
            hi_l = mid
    return math.exp(lo_l)


def test_plan_lfg_is_the_inverse_of_f_and_g(oracle_mod):
    rng = np.random.default_rng(3)
    checked_inf = checked_fin = 0
    for _ in range(300):
        omega = int(rng.integers(50, 10**6))
        t = int(rng.integers(1, omega))
        c = int(rng.integers(0, t + 1)) if rng.random() < 0.5 else int(rng.integers(0, max(2, t // 50)))
        eps = float(rng.choice([0.05, 0.02, 0.01, 0.005]))
        b = c / t
        lf, lg = oracle_mod.plan_lfg(b, t, omega, eps)
        nf = _invert(lambda L: oracle_mod.fg(c, t, omega, L)[0], eps)
        ng = _invert(lambda L: oracle_mod.fg(c, t, omega, L)[1], eps)
        assert lg == pytest.approx(ng, rel=1e-9)
        assert oracle_mod.fg(c, t, omega, lg)[1] == pytest.approx(eps, rel=1e-9)
        if math.isinf(lf):
            assert nf == 1e6  # f stays below eps for every L
            checked_inf += 1
        else:
            assert lf == pytest.approx(nf, rel=1e-9)
            assert oracle_mod.fg(c, t, omega, lf)[0] == pytest.approx(eps, rel=1e-9)
            checked_fin += 1
    assert checked_inf > 20 and checked_fin > 20


def _first_phase(oracle_mod, g, seed, m1):
    st = oracle_mod.setup(g, 0.1, 0.1)
    base = oracle_mod.FIRST_PHASE_BASE
    _, acc = oracle_mod.accumulate(g, st["comp"], seed, base, base + m1)
    return acc.astype(np.int32)


@pytest.mark.parametrize("name,g,eps", [
    ("rmat12", G.rmat(12, 16, seed=2), 0.02),
    ("grid", G.grid_graph(24, 24), 0.02),
    ("rhg", G.rhg(1 << 11, 10.0, 2.8, seed=7), 0.05),
    ("er", G.erdos_renyi(800, 6.0, seed=4), 0.05),
])
def test_plan_budget_and_floor(oracle_mod, name, g, eps):
    delta = 0.1
    st = oracle_mod.setup(g, eps, delta)
    omega, L = st["omega"], st["L"]
    m1 = oracle_mod.first_phase_samples(omega)
    assert m1 == -(-omega // 20)
    c1 = _first_phase(oracle_mod, g, 5, m1)
    t, LL, LU = oracle_mod.plan(c1, m1, omega, eps, delta, L)
    assert 0 < t < omega, name
    total = float(np.exp(-LL).sum() + np.exp(-LU).sum())
    assert total <= delta / 2
    assert total >= BETA * delta / 2
    cap = math.log(4 * g.n / (BETA * delta))  # the floor share alone
    assert LL.max() <= cap * (1 + 1e-12) and LU.max() <= cap * (1 + 1e-12)
    # a larger first-phase count never gets a larger constant
    order = np.argsort(c1, kind="stable")
    assert np.all(np.diff(LU[order]) <= 1e-9)
    # t* is the first sample count the budget admits (S is monotone here)
    target = (1 - BETA) * delta / 2 * (1 - 1e-6)
    assert oracle_mod.plan_sum(c1, m1, t, omega, eps) <= target
    assert oracle_mod.plan_sum(c1, m1, t - 1, omega, eps) > target
    # the constants are the planning inverse at t*, mixed with the floor
    v = int(np.argmax(c1))
    lf, lg = oracle_mod.plan_lfg((c1[v] + 1) / m1, t, omega, eps)
    floor = BETA * delta / (4 * g.n)
    assert LU[v] == pytest.approx(-math.log((1 - BETA) * math.exp(-lg) + floor), rel=1e-14)
    assert LL[v] == pytest.approx(-math.log((1 - BETA) * math.exp(-lf) + floor), rel=1e-14)


def test_plan_falls_back_to_uniform(oracle_mod):
    # every vertex on every path with a coarse eps: the budget never fits
    n, m1, omega, eps, delta = 50, 40, 100, 0.3, 0.1
    L = oracle_mod.log_inv_delta(n, delta)
    t, LL, LU = oracle_mod.plan(np.full(n, m1, np.int32), m1, omega, eps, delta, L)
    assert t == 0
    assert np.all(LL == L) and np.all(LU == L)
    # a star's center lies on almost every path: g needs about 2 L / eps^2
    # samples, far beyond omega, so there is no plan and the run reaches omega
    # with either set of constants
    g, eps = G.star_graph(200), 0.05
    r = oracle_mod.run(g, eps, delta, 5, 64, first_samples=-1)
    assert r.stats["plan_tau"] == 0 and np.all(r.LL == r.stats["L"])
    u = oracle_mod.run(g, eps, delta, 5, 64)
    assert r.tau == u.tau == r.stats["omega"] and np.array_equal(r.counts, u.counts)


def test_first_phase_is_its_own_stream(oracle_mod):
    g, eps, delta, n_check = G.rmat(11, 16, seed=6), 0.03, 0.1, 512
    r = oracle_mod.run(g, eps, delta, 9, n_check, first_samples=300)
    assert r.stats["first_samples"] == 300
    # the first phase draws sample indices 2^63 .. 2^63 + 299
    assert np.array_equal(r.c1, _first_phase(oracle_mod, g, 9, 300))
    assert r.stats["first_path_interior"] == int(r.c1.sum())
    # the adaptive samples are those of the uniform run: indices 0 .. tau - 1
    st = oracle_mod.setup(g, eps, delta)
    _, acc = oracle_mod.accumulate(g, st["comp"], 9, 0, r.tau)
    assert np.array_equal(r.counts, acc.astype(np.int32))
    # and the check at each boundary used the per-vertex constants
    assert bool(r.decisions[-1] == 1) == oracle_mod.check_stop_v(r.counts, r.tau, r.stats["omega"],
                                                                 r.LL, r.LU, eps)
    t, LL, LU = oracle_mod.plan(r.c1, 300, r.stats["omega"], eps, delta, r.stats["L"])
    assert t == r.stats["plan_tau"] and np.array_equal(LL, r.LL) and np.array_equal(LU, r.LU)


def test_uniform_run_unchanged(oracle_mod):
    g, eps, delta, n_check = G.workload("er4096")
    with open(os.path.join(GOLDEN, "oracle_runs.json")) as f:
        ref = json.load(f)["er4096"]
    r = oracle_mod.run(g, eps, delta, 1, n_check, first_samples=0)
    assert r.tau == ref["tau"] and r.LL is None
    assert r.stats["first_samples"] == 0 and r.stats["plan_tau"] == 0


def test_balanced_stops_earlier_on_hub_graph(oracle_mod):
    """R-MAT scale 18: uniform constants stop at 32768 samples (stored run);
    the balanced constants stop at the first boundary."""
    g, eps, delta, n_check = G.workload("rmat18")
    with open(os.path.join(GOLDEN, "oracle_runs.json")) as f:
        golden = json.load(f)
    assert golden["rmat18"]["tau"] == 32768
    r = oracle_mod.run(g, eps, delta, 1, n_check, first_samples=-1)
    ref = golden["rmat18_balanced"]
    assert r.tau == ref["tau"] == 16384
    assert r.stats["plan_tau"] == ref["stats"]["plan_tau"]


EPS_GRAPHS = [G.star_graph(20), G.barbell(8, 4), G.grid_graph(8, 8), G.erdos_renyi(256, 6.0, seed=1)]


@pytest.mark.parametrize("g", EPS_GRAPHS, ids=lambda g: g.name)
def test_balanced_eps_guarantee_over_seeds(oracle_mod, g):
    eps, delta, seeds = 0.03, 0.1, 100
    b = oracle_mod.brandes(g)
    fails = 0
    worst = 0.0
    for seed in range(1, seeds + 1):
        r = oracle_mod.run(g, eps, delta, seed, 256, first_samples=-1)
        err = float(np.abs(r.scores - b).max())
        worst = max(worst, err)
        fails += err > eps
    # P(Binomial(100, 0.1) >= 21) < 0.2%; the bound is conservative, so ~0 expected
    assert fails < 21, (fails, worst)
