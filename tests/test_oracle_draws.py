"""Pins for the oracle's random draws of a sample (Section 2.3: a uniformly
random shortest s-t path), in the regimes where its integer arithmetic is
widest:

* the meeting-vertex draw when the products sigma_s(v) sigma_t(v) exceed 2^40,
  so that the weights are rounded up by a common shift;
* predecessor draws whose candidate sum exceeds 2^64 (the high half of the
  64 x 128-bit multiply), and levels whose counts exceed 2^104 (rescaled).

Every check recomputes from scratch with Python's exact integers: distances
and path counts by a BFS of its own, the meeting set by the expansion rule
(the side with the smaller frontier degree sum, s on ties), the weights, the
totals and each draw r = floor(U * total / 2^64) with U the pinned Philox
word.  The laws are then checked against the mathematics: the meeting vertex
must follow sigma_s(v) sigma_t(v) / sigma_st and each predecessor p of x must
follow sigma(p) / sigma(x), by chi-square over many draws at a fixed pair.
"""
from collections import Counter
from fractions import Fraction

import numpy as np
import pytest
from scipy import stats

from paper_1903_09422_amd import graphs as G

WEIGHT_BITS = 40
SIGMA_BITS = 104


def layered_graph(layers, width):
    """Consecutive groups of `width` vertices joined completely."""
    u, v = [], []
    for a in range(layers - 1):
        for i in range(width):
            for j in range(width):
                u.append(a * width + i)
                v.append((a + 1) * width + j)
    return G.from_edges(layers * width, u, v, lcc=False, name=f"layers{layers}x{width}")


def random_layered(layers, width, p, seed):
    """Groups of `width` vertices; each vertex of group a + 1 is joined to a
    random nonempty subset of group a (each member with probability p), and a
    few edges inside groups.  Path counts grow unevenly, about (p width)^k."""
    rng = np.random.default_rng(seed)
    u, v = [], []
    for a in range(layers - 1):
        for j in range(width):
            pick = np.flatnonzero(rng.random(width) < p)
            if pick.size == 0:
                pick = np.array([rng.integers(width)])
            for i in pick:
                u.append(a * width + int(i))
                v.append((a + 1) * width + j)
        if rng.random() < 0.3:
            i, j = rng.choice(width, 2, replace=False)
            u.append(a * width + int(i))
            v.append(a * width + int(j))
    return G.from_edges(layers * width, u, v, lcc=False, name=f"rlayers{layers}x{width}")


def rows_of(g):
    return [g.col[g.row_ptr[x]:g.row_ptr[x + 1]].tolist() for x in range(g.n)]


def bfs_exact(rows, src):
    """Distances and exact shortest-path counts (Python integers) from src."""
    n = len(rows)
    dist = [-1] * n
    sig = [0] * n
    dist[src], sig[src] = 0, 1
    order = [src]
    for u in order:
        for w in rows[u]:
            if dist[w] < 0:
                dist[w] = dist[u] + 1
                order.append(w)
            if dist[w] == dist[u] + 1:
                sig[w] += sig[u]
    return dist, sig


def replay_search(rows, s, t):
    """The bidirectional search of a sample at pair (s, t), recomputed from
    full BFS distances: returns dict with the expanded side X at the meeting
    level, the meeting set M (ascending), d, the levels each side built, and
    the stored counts m_s, m_t (exact counts, each built level divided by
    2^sh, rounding up, if its largest count reaches 2^104)."""
    ds, ss = bfs_exact(rows, s)
    dt, st = bfs_exact(rows, t)
    dist = (ds, dt)
    deg = [len(r) for r in rows]
    lvl = [0, 0]
    dsum = [deg[s], deg[t]]
    built = [0, 0]
    while True:
        X = 0 if dsum[0] <= dsum[1] else 1
        Y = 1 - X
        new = [w for w in range(len(rows)) if dist[X][w] == lvl[X] + 1]
        assert new, "the balls must grow inside one component"
        built[X] = lvl[X] + 1
        M = sorted(w for w in new if 0 <= dist[Y][w] <= lvl[Y])
        if M:
            assert all(dist[Y][w] == lvl[Y] for w in M)
            d = lvl[X] + 1 + lvl[Y]
            break
        lvl[X] += 1
        dsum[X] = sum(deg[w] for w in new)
    # stored counts, level by level, with the rescale of the reading
    m = []
    rescaled = 0
    for side, src in ((0, s), (1, t)):
        mm = {src: 1}
        for k in range(1, built[side] + 1):
            level = [w for w in range(len(rows)) if dist[side][w] == k]
            raw = {w: sum(mm[p] for p in rows[w] if dist[side][p] == k - 1) for w in level}
            sh = max(0, max(raw.values()).bit_length() - SIGMA_BITS)
            if sh:
                rescaled += 1
            for w in level:
                mm[w] = -((-raw[w]) >> sh)  # ceil(raw / 2^sh)
        m.append(mm)
    return {"X": X, "M": M, "d": d, "dist": dist, "sig": (ss, st), "m": m, "rescaled": rescaled}


def meeting_weights(R):
    P = [R["m"][0][v] * R["m"][1][v] for v in R["M"]]
    sh = max(0, max(P).bit_length() - WEIGHT_BITS)
    W = [-((-p) >> sh) for p in P]
    return P, sh, W


def draw(u64, total):
    return (u64 * total) >> 64


def replay_path(rows, R, uniform, v):
    """The interior path the reading draws from meeting vertex v: s-side
    predecessors from v down, then t-side ones (the oracle's order)."""
    out = [v] if R["dist"][0][v] > 0 and R["dist"][1][v] > 0 else []
    wide = 0
    for side in (0, 1):
        dist, m = R["dist"][side], R["m"][side]
        x = v
        while dist[x] > 1:
            cands = [p for p in rows[x] if dist[p] == dist[x] - 1]  # CSR (ascending) order
            tot = sum(m[p] for p in cands)
            wide += tot >= 1 << 64
            r = draw(uniform(2 * dist[x] + side), tot)
            acc = 0
            for p in cands:
                acc += m[p]
                if acc > r:
                    break
            x = p
            out.append(x)
    return out, wide


DRAW_GRAPHS = [
    (G.grid_graph(64, 64), 60),
    (layered_graph(80, 17), 80),
    (random_layered(120, 6, 0.5, seed=4), 80),
    (G.hypercube(7), 60),
    (G.erdos_renyi(300, 4.0, seed=5), 60),
]


@pytest.mark.parametrize("g,samples", DRAW_GRAPHS, ids=lambda x: getattr(x, "name", str(x)))
def test_sample_draws_replayed_with_exact_integers(oracle_mod, g, samples):
    """Every sample's meeting set, shift, weight total, sigma sum, meeting
    vertex and predecessor draws equal an exact-integer replay of the reading;
    the rounded meeting weights stay within |M| / T of the exact law."""
    rows = rows_of(g)
    _, comp = oracle_mod.components(g)
    seed = 11
    shifted = wide = rescaled = 0
    for i in range(samples):
        interior, info = oracle_mod.sample(g, comp, seed, i)
        if info.d < 0:
            continue
        R = replay_search(rows, info.s, info.t)
        assert info.d == R["d"] and info.side_x_last == R["X"]
        assert info.meet_size == len(R["M"])
        P, sh, W = meeting_weights(R)
        T = sum(W)
        assert info.meet_shift == sh, (i, info.meet_shift, sh)
        assert info.meet_total == T, (i, info.meet_total, T)
        assert T < 1 << 63 and min(W) >= 1
        assert info.sigma == sum(P)
        if R["rescaled"] == 0:
            assert info.sigma_scale == 0
            assert info.sigma == R["sig"][0][info.t]  # sigma_st, exact
            exact = sum(P)
            for p, w in zip(P, W):
                assert abs(Fraction(w, T) - Fraction(p, exact)) <= Fraction(len(P), T)
        else:
            assert info.sigma_scale > 0
        r = draw(oracle_mod.uniform64(seed, i, 1), T)
        acc = 0
        for v, w in zip(R["M"], W):
            acc += w
            if acc > r:
                break
        assert info.meet_vertex == v
        path, nwide = replay_path(rows, R, lambda j: oracle_mod.uniform64(seed, i, j), v)
        assert interior.tolist() == path
        shifted += sh > 0
        wide += nwide
        rescaled += R["rescaled"] > 0
    if g.name.startswith("grid64"):
        assert shifted >= samples // 4  # the rounded draw is exercised
    if g.name.startswith("layers"):
        assert wide >= 100 and rescaled >= 10
    if g.name.startswith("rlayers"):
        assert shifted >= samples // 2 and wide >= 100 and rescaled >= 5


def _chi2(observed, expected_p):
    n = sum(observed)
    exp = np.array(expected_p, dtype=float) * n
    obs = np.array(observed, dtype=float)
    keep = exp > 0
    return float(((obs[keep] - exp[keep]) ** 2 / exp[keep]).sum()), int(keep.sum()) - 1


def _fixed_pair_laws(oracle_mod, g, s, t, count, min_shift=1):
    """Draws `count` samples at (s, t).  Returns the chi-square statistic and
    degrees of freedom of (a) the meeting vertex against
    sigma_s(v) sigma_t(v) / sum, (b) every predecessor step against
    sigma(p) / sum over the candidates, with the step's candidate sum."""
    rows = rows_of(g)
    _, comp = oracle_mod.components(g)
    paths, meet, info = oracle_mod.sample_pair(g, comp, 29, s, t, 0, count)
    R = replay_search(rows, s, t)
    ss, st = R["sig"]
    assert info.meet_shift >= min_shift
    # (a) meeting vertex, exact law
    P = [ss[v] * st[v] for v in R["M"]]
    cnt = Counter(meet.tolist())
    assert set(cnt) <= set(R["M"])
    chi_m, dof_m = _chi2([cnt.get(v, 0) for v in R["M"]], [Fraction(p, sum(P)) for p in P])
    # (b) predecessor steps, grouped by (side, x); exact law sigma(p) / sigma(x)
    steps = {}
    d = R["d"]
    for row in paths.tolist():
        order = sorted(row, key=lambda x: R["dist"][0][x])  # s-side distance 1 .. d - 1
        full = [s] + order + [t]
        v_at = [x for x in full if x in set(R["M"])]
        assert len(v_at) == 1
        kv = R["dist"][0][v_at[0]]
        for k in range(kv, 1, -1):  # s side: x at distance k picks the vertex at k - 1
            steps.setdefault((0, full[k]), Counter())[full[k - 1]] += 1
        for k in range(kv, d - 1):  # t side: x at t-distance d - k picks full[k + 1]
            steps.setdefault((1, full[k]), Counter())[full[k + 1]] += 1
    chi_p, dof_p, widest = 0.0, 0, 0
    for (side, x), c in steps.items():
        dist, sig = R["dist"][side], R["sig"][side]
        cands = [p for p in rows[x] if dist[p] == dist[x] - 1]
        assert set(c) <= set(cands)
        tot = sum(sig[p] for p in cands)
        assert tot == sig[x]
        if len(cands) < 2 or sum(c.values()) < 20 * len(cands):
            continue
        a, b = _chi2([c.get(p, 0) for p in cands], [Fraction(sig[p], tot) for p in cands])
        chi_p += a
        dof_p += b
        widest = max(widest, tot.bit_length())
    return (chi_m, dof_m), (chi_p, dof_p), widest


@pytest.mark.parametrize("case", ["grid64", "rlayers", "layers"])
def test_path_law_at_wide_counts(oracle_mod, case):
    """At fixed far-apart pairs, the meeting vertex (with rounded weights) and
    every predecessor step (with candidate sums beyond 2^64 and levels beyond
    2^104) follow the exact law of a uniformly random shortest path."""
    if case == "grid64":
        g, s, t, count = G.grid_graph(64, 64), 0, 64 * 40 + 63, 30000
    elif case == "rlayers":
        g, t, count = random_layered(120, 6, 0.5, seed=4), 119 * 6 + 3, 20000
        _, comp = oracle_mod.components(g)
        s = next(v for v in range(6) if comp[v] == comp[t])
    else:
        g, s, t, count = layered_graph(80, 17), 5, 79 * 17 + 11, 6000
    (chi_m, dof_m), (chi_p, dof_p), widest = _fixed_pair_laws(oracle_mod, g, s, t, count)
    if dof_m > 0:
        assert stats.chi2.sf(chi_m, dof_m) > 1e-4, (chi_m, dof_m)
    assert dof_p > 0 and stats.chi2.sf(chi_p, dof_p) > 1e-4, (chi_p, dof_p)
    if case != "grid64":
        assert widest > 64  # candidate sums beyond 2^64 are among the checked steps
