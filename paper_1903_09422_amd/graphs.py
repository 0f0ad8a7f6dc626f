"""Seeded synthetic graph generators and the canonical CSR form.

This module is the only code shared by the CPU oracle's tests and the HIP
path's tests and benchmarks.  It produces inputs and nothing else: it holds
none of the sampling method's arithmetic.

The paper evaluates on undirected real-world networks of two shapes
(Section 4 and the instance table of Appendix F): social / hyperlink graphs
with small diameter and heavy-tailed degrees, and road networks with large
diameter and degrees of about 2-4.  Those datasets are not available here, so
the generators below stand in for them:

* ``erdos_renyi``      -- small plain workload, G(n, p);
* ``rmat``             -- heavy-tailed, low-diameter (social-network shape);
* ``perturbed_grid``   -- high-diameter, low-degree (road-network shape);
* small named graphs   -- closed-form and brute-force test cases.

Canonical form (every generator returns it): undirected simple graph as a
symmetric int32 CSR, no self-loops, no duplicate arcs, each row sorted
ascending; when ``lcc=True`` only the largest connected component is kept and
its vertices are relabelled 0..n-1 in increasing original ID.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components


@dataclass(frozen=True)
class CSR:
    """Undirected graph in symmetric CSR form (int32 arrays)."""

    n: int
    row_ptr: np.ndarray  # int32[n + 1]
    col: np.ndarray      # int32[row_ptr[n]]
    name: str = ""

    @property
    def num_arcs(self) -> int:
        return int(self.row_ptr[-1])

    @property
    def num_edges(self) -> int:
        return self.num_arcs // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr).astype(np.int64)

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.row_ptr, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.col, dtype=np.int32).tobytes())
        return h.hexdigest()

    def to_scipy(self) -> sp.csr_matrix:
        data = np.ones(self.num_arcs, dtype=np.int8)
        return sp.csr_matrix((data, self.col, self.row_ptr), shape=(self.n, self.n))

    def edge_list(self) -> np.ndarray:
        """Undirected edges (u < v) as an int64 array of shape (m, 2)."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        dst = self.col.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)


def from_edges(n: int, u, v, *, lcc: bool = True, name: str = "") -> CSR:
    """Canonicalise an undirected edge list on vertices 0..n-1.

    Symmetrises, removes self-loops and duplicates, optionally keeps the
    largest connected component (ties: the component holding the lowest
    vertex ID) relabelled in increasing original ID, and sorts every row.
    """
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    if u.shape != v.shape:
        raise ValueError("u and v differ in length")
    if u.size and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("vertex id out of range")
    keep = u != v
    u, v = u[keep], v[keep]
    src = np.concatenate([u, v])
    dst = np.concatenate([v, u])
    key = np.unique(src * np.int64(n) + dst)  # sorted by (src, dst): dedup + row order
    src = key // n
    dst = key % n
    if lcc:
        a = sp.csr_matrix((np.ones(src.size, dtype=np.int8), (src, dst)), shape=(n, n))
        ncomp, label = connected_components(a, directed=False)
        if ncomp > 1:
            sizes = np.bincount(label, minlength=ncomp)
            best = int(np.flatnonzero(sizes == sizes.max())[0])
            # label ids are assigned in order of first vertex, so the first
            # maximal label holds the lowest vertex id among the tied ones
            keep_v = label == best
            new_id = np.full(n, -1, dtype=np.int64)
            new_id[keep_v] = np.arange(int(keep_v.sum()), dtype=np.int64)
            m = keep_v[src]
            src = new_id[src[m]]
            dst = new_id[dst[m]]
            n = int(keep_v.sum())
            # relabelling is monotone, so (src, dst) order is preserved
    counts = np.bincount(src, minlength=n).astype(np.int64)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("too many arcs for int32 CSR")
    return CSR(n=n, row_ptr=row_ptr.astype(np.int32), col=dst.astype(np.int32), name=name)


# --------------------------------------------------------------------------
# Workload generators (the paper's two graph shapes, synthetic stand-ins)
# --------------------------------------------------------------------------

def erdos_renyi(n: int = 4096, mean_degree: float = 8.0, seed: int = 1, *, lcc: bool = True) -> CSR:
    """G(n, p) with p = mean_degree / (n - 1): each unordered pair is an edge
    independently with probability p."""
    rng = np.random.default_rng(seed)
    p = mean_degree / (n - 1)
    iu, ju = np.triu_indices(n, 1)
    take = rng.random(iu.size) < p
    return from_edges(n, iu[take], ju[take], lcc=lcc, name=f"er_n{n}_d{mean_degree:g}_s{seed}")


def rmat(scale: int = 18, edge_factor: int = 16, abcd=(0.57, 0.19, 0.19, 0.05), seed: int = 1,
         *, lcc: bool = True) -> CSR:
    """R-MAT generator: edge_factor * 2**scale directed draws, each choosing one
    of four quadrants (a: 00, b: 01, c: 10, d: 11) per bit of (src, dst), then
    symmetrised and canonicalised.  No vertex permutation is applied."""
    a, b, c, d = abcd
    if abs(a + b + c + d - 1.0) > 1e-9:
        raise ValueError("R-MAT probabilities must sum to 1")
    rng = np.random.default_rng(seed)
    n = 1 << scale
    m = edge_factor * n
    src = np.zeros(m, dtype=np.int64)
    dst = np.zeros(m, dtype=np.int64)
    for bit in range(scale):
        r = rng.random(m)
        s_bit = r >= a + b
        d_bit = ((r >= a) & (r < a + b)) | (r >= a + b + c)
        src |= s_bit.astype(np.int64) << bit
        dst |= d_bit.astype(np.int64) << bit
    return from_edges(n, src, dst, lcc=lcc, name=f"rmat_s{scale}_ef{edge_factor}_s{seed}")


def perturbed_grid(side: int = 1024, delete_frac: float = 0.05, shortcut_frac: float = 0.001,
                   seed: int = 1, *, lcc: bool = True) -> CSR:
    """side x side 4-neighbour grid (vertex id = row * side + col) with
    round(delete_frac * E) edges deleted uniformly at random and
    round(shortcut_frac * E) uniformly random non-duplicate long-range edges
    added, E being the grid's edge count."""
    rng = np.random.default_rng(seed)
    n = side * side
    ids = np.arange(n, dtype=np.int64).reshape(side, side)
    hu, hv = ids[:, :-1].ravel(), ids[:, 1:].ravel()
    vu, vv = ids[:-1, :].ravel(), ids[1:, :].ravel()
    eu = np.concatenate([hu, vu])
    ev = np.concatenate([hv, vv])
    n_edges = eu.size
    n_del = int(round(delete_frac * n_edges))
    perm = rng.permutation(n_edges)
    keep = np.sort(perm[n_del:])
    eu, ev = eu[keep], ev[keep]
    n_add = int(round(shortcut_frac * n_edges))
    existing = set((np.minimum(eu, ev) * n + np.maximum(eu, ev)).tolist())
    add_u, add_v = [], []
    while len(add_u) < n_add:
        x = int(rng.integers(n))
        y = int(rng.integers(n))
        if x == y:
            continue
        k = min(x, y) * n + max(x, y)
        if k in existing:
            continue
        existing.add(k)
        add_u.append(x)
        add_v.append(y)
    eu = np.concatenate([eu, np.asarray(add_u, dtype=np.int64)])
    ev = np.concatenate([ev, np.asarray(add_v, dtype=np.int64)])
    return from_edges(n, eu, ev, lcc=lcc, name=f"pgrid_{side}_s{seed}")


def _rhg_edges(r: np.ndarray, theta: np.ndarray, R: float, bands: int = 16):
    """Pairs (i, j), i < j, of points at hyperbolic distance <= R, where
    cosh d = cosh r_i cosh r_j - sinh r_i sinh r_j cos(theta_i - theta_j).
    Candidates come from angular windows per radial band: for r_j >= b, the
    largest angle that still connects shrinks as b grows, so the window at the
    band's lower bound b holds every partner in that band."""
    n = r.size
    order = np.argsort(theta, kind="stable")
    r, theta = r[order], theta[order]
    ch, sh = np.cosh(r), np.sinh(r)
    coshR = np.cosh(R)
    edges_u, edges_v = [], []
    bounds = np.linspace(0.0, R, bands + 1)
    band_of = np.minimum(np.searchsorted(bounds, r, side="right") - 1, bands - 1)
    two_pi = 2.0 * np.pi
    for c in range(bands):
        members = np.flatnonzero(band_of == c)  # sorted by angle already
        if members.size == 0:
            continue
        ang_c = theta[members]
        b = bounds[c]
        chb, shb = np.cosh(b), np.sinh(b)
        for i0 in range(0, n, 65536):
            ii = np.arange(i0, min(n, i0 + 65536))
            with np.errstate(divide="ignore", invalid="ignore"):
                arg = (ch[ii] * chb - coshR) / (sh[ii] * shb)
            dmax = np.where(np.isfinite(arg), np.arccos(np.clip(arg, -1.0, 1.0)), np.pi)
            dmax = np.where(arg <= -1.0, np.pi, dmax)
            lo_a, hi_a = theta[ii] - dmax, theta[ii] + dmax
            # the window, split where it wraps around 2 pi
            parts = [(np.maximum(lo_a, 0.0), np.minimum(hi_a, two_pi)),
                     (np.where(lo_a < 0.0, lo_a + two_pi, two_pi), np.full(ii.size, two_pi)),
                     (np.zeros(ii.size), np.where(hi_a > two_pi, hi_a - two_pi, 0.0))]
            for a, z in parts:
                s0 = np.searchsorted(ang_c, a, side="left")
                s1 = np.searchsorted(ang_c, z, side="right")
                cnt = np.maximum(s1 - s0, 0)
                tot = int(cnt.sum())
                if tot == 0:
                    continue
                src = np.repeat(ii, cnt)
                start = np.repeat(s0 - np.cumsum(cnt) + cnt, cnt)
                dst = members[np.arange(tot) + start]
                keep = src < dst
                src, dst = src[keep], dst[keep]
                cosd = ch[src] * ch[dst] - sh[src] * sh[dst] * np.cos(theta[src] - theta[dst])
                ok = cosd <= coshR
                edges_u.append(order[src[ok]])
                edges_v.append(order[dst[ok]])
    if not edges_u:
        return np.zeros(0, np.int64), np.zeros(0, np.int64)
    return np.concatenate(edges_u), np.concatenate(edges_v)


def rhg(n: int, mean_degree: float = 10.0, gamma: float = 2.8, seed: int = 1, *,
        lcc: bool = True) -> CSR:
    """Threshold random hyperbolic graph: n points on a hyperbolic disk of
    radius R, angle uniform, radius density alpha sinh(alpha r) / (cosh(alpha R)
    - 1) with alpha = (gamma - 1) / 2; vertices adjacent iff their hyperbolic
    distance is at most R.  R is bisected until the mean degree is within 0.5
    of mean_degree (the same points are reused for every R)."""
    rng = np.random.default_rng(seed)
    alpha = (gamma - 1.0) / 2.0
    theta = rng.random(n) * 2.0 * np.pi
    u = rng.random(n)

    def build(R):
        r = np.arccosh(1.0 + (np.cosh(alpha * R) - 1.0) * u) / alpha
        return _rhg_edges(r, theta, R)

    xi = alpha / (alpha - 0.5)
    R = 2.0 * np.log(2.0 * xi * xi * n / (np.pi * mean_degree))  # asymptotic estimate
    lo, hi = R - 4.0, R + 4.0
    for _ in range(40):
        eu, ev = build(R)
        deg = 2.0 * eu.size / n
        if abs(deg - mean_degree) <= 0.5:
            break
        if deg > mean_degree:
            lo = R
        else:
            hi = R
        R = 0.5 * (lo + hi)
    return from_edges(n, eu, ev, lcc=lcc, name=f"rhg_n{n}_d{mean_degree:g}_s{seed}")


def batch_pool(seed: int = 1):
    """The batched workload: 64 graphs, 32 R-MAT of scale 12 + (k mod 5)
    (edge factor 16) and 32 threshold random hyperbolic graphs of
    n = 2^(14 + k mod 4), mean degree 10, power-law exponent 2.8; each query's
    eps drawn from {0.05, 0.02, 0.01}; delta = 0.1, checks every 1024 samples.
    Returns a list of (graph, eps, delta, check_interval, query_seed)."""
    rng = np.random.default_rng(seed)
    eps_choices = np.array([0.05, 0.02, 0.01])
    out = []
    for k in range(32):
        g = rmat(12 + (k % 5), 16, seed=1000 + k)
        out.append((g, float(eps_choices[rng.integers(3)]), 0.1, 1024, 1 + k))
    for k in range(32):
        g = rhg(1 << (14 + (k % 4)), 10.0, 2.8, seed=2000 + k)
        out.append((g, float(eps_choices[rng.integers(3)]), 0.1, 1024, 33 + k))
    return out


def serve_pool(seed: int = 1, with_rmat22: bool = True):
    """Graphs of the served workload: the 64 graphs of batch_pool, the
    perturbed 1024 x 1024 grid and (optionally) R-MAT scale 22, edge factor 16."""
    pool = [g for g, *_ in batch_pool(seed)]
    pool.append(perturbed_grid(1024, seed=1))
    if with_rmat22:
        pool.append(rmat(22, 16, seed=1))
    return pool


def serve_trace(num_graphs: int, num_queries: int = 256, seed: int = 7):
    """A seeded query stream for serving: each query picks a graph uniformly,
    eps from {0.05, 0.01}, delta 0.1, checks every 16384 samples, and its own
    sampling seed; unit-rate exponential gaps (scaled to a rate by the caller)
    give Poisson arrivals.  Returns (queries, gaps): queries as
    (graph_index, eps, delta, check_interval, query_seed)."""
    rng = np.random.default_rng(seed)
    gi = rng.integers(0, num_graphs, num_queries)
    eps = np.array([0.05, 0.01])[rng.integers(0, 2, num_queries)]
    queries = [(int(gi[i]), float(eps[i]), 0.1, 16384, 5000 + i) for i in range(num_queries)]
    gaps = rng.exponential(1.0, num_queries)
    gaps[0] = 0.0
    return queries, gaps


# --------------------------------------------------------------------------
# Small named graphs (closed forms and brute force)
# --------------------------------------------------------------------------

def path_graph(n: int) -> CSR:
    i = np.arange(n - 1)
    return from_edges(n, i, i + 1, lcc=False, name=f"path{n}")


def cycle_graph(n: int) -> CSR:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, lcc=False, name=f"cycle{n}")


def star_graph(leaves: int) -> CSR:
    i = np.arange(1, leaves + 1)
    return from_edges(leaves + 1, np.zeros_like(i), i, lcc=False, name=f"star{leaves}")


def complete_graph(n: int) -> CSR:
    iu, ju = np.triu_indices(n, 1)
    return from_edges(n, iu, ju, lcc=False, name=f"K{n}")


def complete_bipartite(a: int, b: int) -> CSR:
    u = np.repeat(np.arange(a), b)
    v = a + np.tile(np.arange(b), a)
    return from_edges(a + b, u, v, lcc=False, name=f"K{a}_{b}")


def grid_graph(rows: int, cols: int) -> CSR:
    ids = np.arange(rows * cols, dtype=np.int64).reshape(rows, cols)
    u = np.concatenate([ids[:, :-1].ravel(), ids[:-1, :].ravel()])
    v = np.concatenate([ids[:, 1:].ravel(), ids[1:, :].ravel()])
    return from_edges(rows * cols, u, v, lcc=False, name=f"grid{rows}x{cols}")


def hypercube(k: int) -> CSR:
    n = 1 << k
    u, v = [], []
    for x in range(n):
        for b in range(k):
            y = x ^ (1 << b)
            if x < y:
                u.append(x)
                v.append(y)
    return from_edges(n, u, v, lcc=False, name=f"Q{k}")


def barbell(clique: int, bridge: int) -> CSR:
    """Two cliques of ``clique`` vertices joined by a path of ``bridge`` extra vertices."""
    u, v = [], []
    for off in (0, clique + bridge):
        for i in range(clique):
            for j in range(i + 1, clique):
                u.append(off + i)
                v.append(off + j)
    chain = [clique - 1] + [clique + k for k in range(bridge)] + [clique + bridge]
    for x, y in zip(chain[:-1], chain[1:]):
        u.append(x)
        v.append(y)
    n = 2 * clique + bridge
    return from_edges(n, u, v, lcc=False, name=f"barbell{clique}_{bridge}")


def disjoint_union(*graphs: CSR) -> CSR:
    """Vertex-disjoint union (several connected components)."""
    us, vs, off = [], [], 0
    for g in graphs:
        e = g.edge_list()
        us.append(e[:, 0] + off)
        vs.append(e[:, 1] + off)
        off += g.n
    return from_edges(off, np.concatenate(us), np.concatenate(vs), lcc=False, name="union")


def empty_graph(n: int) -> CSR:
    return CSR(n=n, row_ptr=np.zeros(n + 1, dtype=np.int32), col=np.zeros(0, dtype=np.int32),
               name=f"empty{n}")


def random_connected(n: int, extra_edges: int, seed: int) -> CSR:
    """A random spanning tree plus ``extra_edges`` random edges (connected)."""
    rng = np.random.default_rng(seed)
    parent = np.array([int(rng.integers(i)) for i in range(1, n)], dtype=np.int64)
    u = np.concatenate([np.arange(1, n), rng.integers(0, n, extra_edges)])
    v = np.concatenate([parent, rng.integers(0, n, extra_edges)])
    return from_edges(n, u, v, lcc=False, name=f"rc{n}_{extra_edges}_s{seed}")


# --------------------------------------------------------------------------
# Named workloads: the plain-method configurations
# --------------------------------------------------------------------------

WORKLOADS = {
    # name: (builder, eps, delta, check_interval)
    "er4096": (lambda: erdos_renyi(4096, 8.0, seed=1), 0.05, 0.1, 1024),
    "rmat18": (lambda: rmat(18, 16, seed=1), 0.01, 0.1, 16384),
    "pgrid1024": (lambda: perturbed_grid(1024, seed=1), 0.01, 0.1, 16384),
}

_cache: dict = {}


def workload(name: str):
    """Return (graph, eps, delta, check_interval) for a named workload (cached)."""
    if name not in _cache:
        build, eps, delta, n_check = WORKLOADS[name]
        _cache[name] = (build(), eps, delta, n_check)
    return _cache[name]
