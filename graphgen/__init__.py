"""Seeded synthetic inputs: undirected graphs in CSR form and personalization vectors.

This module is shared by the FP64 oracle, the tests and the benchmark. It holds
only input construction (random graph models, CSR assembly, source sampling) and
none of the PageRank / Chebyshev arithmetic, so neither side of a parity test
can borrow the other's computation through it.

All randomness comes from numpy's Philox-4x32-10 counter-based generator
(Salmon et al., SC'11), keyed by an explicit integer seed, so every workload is
reproducible bit for bit on any host.

The paper (Table 1, Sec. 5.1) measures on six undirected meshes / k-mer graphs
that are not available here; the generators below are the synthetic stand-ins:
Erdos-Renyi, Chung-Lu power-law, a perturbed road-like lattice, an uneven batch
of small Chung-Lu graphs, plus tiny structured graphs (cycle, complete, star,
path) whose PageRank has a closed form.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "CSR", "philox", "csr_from_edges", "drop_isolated", "erdos_renyi", "chung_lu",
    "perturbed_grid", "uneven_batch", "cycle", "complete", "star", "path",
    "random_connected", "random_sources", "uniform_personalization",
    "source_personalization", "degrees", "batch_sources", "subgraph", "mpnn_init",
]


def philox(seed) -> np.random.Generator:
    """Philox-4x32-10 generator keyed by ``seed`` (an int or a pair of ints)."""
    return np.random.Generator(np.random.Philox(key=seed))


@dataclass
class CSR:
    """Symmetric 0/1 adjacency pattern of an undirected graph.

    ``row_ptr`` (int32, n+1) and ``col_idx`` (int32, nnz) hold each undirected
    edge twice (u->v and v->u); columns are sorted within a row, there are no
    self-loops and no duplicate entries.  ``graph_ptr`` is set for a
    block-diagonal batch of independent graphs: graph g owns vertices
    [graph_ptr[g], graph_ptr[g+1]).
    """

    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    graph_ptr: np.ndarray | None = None
    meta: dict = field(default_factory=dict)

    @property
    def nnz(self) -> int:
        return int(self.col_idx.shape[0])

    @property
    def num_graphs(self) -> int:
        return 1 if self.graph_ptr is None else int(self.graph_ptr.shape[0] - 1)


def degrees(g: CSR) -> np.ndarray:
    """Vertex degrees (int64) read off the row pointer."""
    return np.diff(g.row_ptr.astype(np.int64))


def csr_from_edges(n: int, u: np.ndarray, v: np.ndarray) -> CSR:
    """Build the symmetric CSR pattern from an undirected edge list.

    Self-loops are dropped and parallel edges merged.
    """
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * n + hi)
    lo = key // n
    hi = key - lo * n
    del key
    rows = np.concatenate([lo, hi])
    cols = np.concatenate([hi, lo])
    del lo, hi
    key = rows * n + cols
    del rows, cols
    key.sort()
    rows = key // n
    cols = (key - rows * n).astype(np.int32)
    del key
    counts = np.bincount(rows, minlength=n)
    del rows
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**31:
        raise ValueError("graph too large for int32 CSR")
    return CSR(n=n, row_ptr=row_ptr.astype(np.int32), col_idx=cols)


def drop_isolated(g: CSR) -> tuple[CSR, np.ndarray]:
    """Remove degree-0 vertices and relabel the rest in their original order.

    Returns the new graph and the kept original vertex ids.
    """
    deg = degrees(g)
    keep = np.nonzero(deg > 0)[0]
    if keep.shape[0] == g.n:
        return g, keep
    remap = np.full(g.n, -1, dtype=np.int64)
    remap[keep] = np.arange(keep.shape[0])
    row_ptr = np.zeros(keep.shape[0] + 1, dtype=np.int64)
    np.cumsum(deg[keep], out=row_ptr[1:])
    col = remap[g.col_idx].astype(np.int32)  # rows of dropped vertices are empty
    out = CSR(n=int(keep.shape[0]), row_ptr=row_ptr.astype(np.int32), col_idx=col,
              meta=dict(g.meta))
    out.meta["dropped_isolated"] = int(g.n - keep.shape[0])
    return out, keep


# ----------------------------------------------------------------------------
# Random graph models
# ----------------------------------------------------------------------------

def erdos_renyi(n: int, avg_deg: float, seed) -> CSR:
    """G(n, p) with p = avg_deg/(n-1); isolated vertices are dropped."""
    rng = philox(seed)
    pairs_total = n * (n - 1) // 2
    p = avg_deg / (n - 1)
    m = int(rng.binomial(pairs_total, p))
    keys = np.empty(0, dtype=np.int64)
    while keys.shape[0] < m:
        need = m - keys.shape[0]
        a = rng.integers(0, n, size=int(need * 1.2) + 16)
        b = rng.integers(0, n, size=a.shape[0])
        ok = a != b
        a, b = a[ok], b[ok]
        k = np.minimum(a, b) * n + np.maximum(a, b)
        keys = np.unique(np.concatenate([keys, k]))
    keys = rng.permutation(keys)[:m]
    lo = keys // n
    hi = keys - lo * n
    g = csr_from_edges(n, lo, hi)
    g, _ = drop_isolated(g)
    g.meta.update(model="erdos_renyi", n_target=n, avg_deg_target=avg_deg)
    return g


def _chung_lu_weights(n: int, avg_deg: float, gamma: float, dmin: float, dmax: float):
    """Expected degrees w_i ~ i^(-1/(gamma-1)), clipped to [dmin, dmax], mean avg_deg."""
    i = np.arange(1, n + 1, dtype=np.float64)
    w = i ** (-1.0 / (gamma - 1.0))
    for _ in range(100):
        w = np.clip(w * (avg_deg / w.mean()), dmin, dmax)
        if abs(w.mean() - avg_deg) < 1e-9 * avg_deg:
            break
    return w


def chung_lu(n: int, avg_deg: float, gamma: float, seed, dmin: float = 1.0,
             dmax: float | None = None, connect_isolated: bool = True,
             topup_rounds: int = 4) -> CSR:
    """Chung-Lu power-law graph with degree exponent ``gamma``.

    Edge endpoints are drawn independently with probability proportional to
    the expected degrees w (so vertex i expects w_i endpoints); self-loops are
    dropped and multi-edges merged.  Because merging removes edges between
    heavy vertices, up to ``topup_rounds`` extra rounds draw the missing edge
    count again.  With ``connect_isolated`` every vertex left without an edge is
    joined to one partner drawn by weight, so the minimum degree is 1 and no
    vertex has to be dropped.  Vertex 0 has the largest expected degree.
    """
    if dmax is None:
        dmax = float(n - 1)
    dmax = min(float(dmax), float(n - 1))
    rng = philox(seed)
    w = _chung_lu_weights(n, avg_deg, gamma, dmin, dmax)
    cdf = np.cumsum(w)
    cdf /= cdf[-1]
    m_target = int(round(n * avg_deg / 2.0))

    def draw(count):
        a = np.searchsorted(cdf, rng.random(count), side="right")
        b = np.searchsorted(cdf, rng.random(count), side="right")
        np.minimum(a, n - 1, out=a)
        np.minimum(b, n - 1, out=b)
        ok = a != b
        a, b = a[ok], b[ok]
        return np.minimum(a, b) * n + np.maximum(a, b)

    keys = np.unique(draw(m_target))
    for _ in range(topup_rounds):
        deficit = m_target - keys.shape[0]
        if deficit <= max(1, int(0.002 * m_target)):
            break
        keys = np.unique(np.concatenate([keys, draw(int(deficit * 1.15) + 8)]))
    if keys.shape[0] > m_target:
        keys = np.sort(rng.choice(keys, size=m_target, replace=False))
    lo = keys // n
    hi = keys - lo * n
    del keys
    if connect_isolated:
        deg = np.bincount(lo, minlength=n) + np.bincount(hi, minlength=n)
        iso = np.nonzero(deg == 0)[0]
        if iso.shape[0]:
            partner = np.searchsorted(cdf, rng.random(iso.shape[0]), side="right")
            np.minimum(partner, n - 1, out=partner)
            clash = partner == iso
            partner[clash] = (iso[clash] + 1) % n
            lo = np.concatenate([lo, iso])
            hi = np.concatenate([hi, partner])
    g = csr_from_edges(n, lo, hi)
    g, _ = drop_isolated(g)
    g.meta.update(model="chung_lu", n_target=n, avg_deg_target=avg_deg, gamma=gamma,
                  dmin=dmin, dmax=dmax)
    return g


def perturbed_grid(side: int, delete_frac: float, shortcut_frac: float, seed,
                   max_deg: int = 5) -> CSR:
    """Road-like lattice: side x side grid, i.i.d. edge deletions, random shortcuts.

    Each lattice edge is deleted with probability ``delete_frac``; then
    ``shortcut_frac`` x (number of lattice edges) random long-range edges are
    added, rejecting self-loops, duplicates and any endpoint already at
    ``max_deg``.  Isolated vertices are dropped.  Vertex r*side+c is cell (r, c).
    """
    rng = philox(seed)
    n = side * side
    r, c = np.meshgrid(np.arange(side), np.arange(side), indexing="ij")
    vid = (r * side + c).astype(np.int64)
    hu, hv = vid[:, :-1].ravel(), vid[:, 1:].ravel()
    vu, vv = vid[:-1, :].ravel(), vid[1:, :].ravel()
    u = np.concatenate([hu, vu])
    v = np.concatenate([hv, vv])
    lattice_edges = u.shape[0]
    keep = rng.random(lattice_edges) >= delete_frac
    u, v = u[keep], v[keep]
    deg = np.bincount(u, minlength=n) + np.bincount(v, minlength=n)
    existing = set((np.minimum(u, v) * n + np.maximum(u, v)).tolist())
    want = int(round(shortcut_frac * lattice_edges))
    su, sv = [], []
    while len(su) < want:
        a = rng.integers(0, n, size=2 * (want - len(su)) + 64)
        b = rng.integers(0, n, size=a.shape[0])
        for x, y in zip(a.tolist(), b.tolist()):
            if len(su) >= want:
                break
            if x == y or deg[x] >= max_deg or deg[y] >= max_deg:
                continue
            k = min(x, y) * n + max(x, y)
            if k in existing:
                continue
            existing.add(k)
            deg[x] += 1
            deg[y] += 1
            su.append(x)
            sv.append(y)
    u = np.concatenate([u, np.asarray(su, dtype=np.int64)])
    v = np.concatenate([v, np.asarray(sv, dtype=np.int64)])
    g = csr_from_edges(n, u, v)
    g, _ = drop_isolated(g)
    g.meta.update(model="perturbed_grid", side=side, delete_frac=delete_frac,
                  shortcut_frac=shortcut_frac, max_deg=max_deg, shortcuts=len(su))
    return g


def delaunay(n: int, seed) -> CSR:
    """Delaunay triangulation of n uniform random points in the unit square
    (the construction of the delaunay_n* graphs: average degree just under 6,
    a planar mesh).  Vertices in the order the points were drawn."""
    from scipy.spatial import Delaunay
    rng = philox(seed)
    pts = rng.random((n, 2))
    tri = Delaunay(pts).simplices.astype(np.int64)
    del pts
    u = np.concatenate([tri[:, 0], tri[:, 1], tri[:, 2]])
    v = np.concatenate([tri[:, 1], tri[:, 2], tri[:, 0]])
    del tri
    g = csr_from_edges(n, u, v)
    g, _ = drop_isolated(g)
    g.meta.update(model="delaunay")
    return g


def directed_random(n: int, avg_deg: float, dangling_frac: float, seed) -> CSR:
    """Random directed graph: each vertex, except a random dangling_frac of them,
    sends edges to ~avg_deg/(1 - dangling_frac) random other vertices (the
    out-degree of a non-dangling vertex is at least 1).  Returned by targets:
    row u lists the sources v of the edges v -> u, sorted; no self loops, no
    duplicates.  Rows may be empty (vertices without in-edges)."""
    rng = philox(seed)
    dangling = rng.random(n) < dangling_frac
    src_ids = np.nonzero(~dangling)[0]
    k = 1 + rng.poisson(max(avg_deg / max(1.0 - dangling_frac, 1e-9) - 1.0, 0.0), src_ids.size)
    v = np.repeat(src_ids, k).astype(np.int64)
    u = rng.integers(0, n, v.size)
    keep = u != v
    u, v = u[keep], v[keep]
    key = np.unique(u * n + v)
    u, v = key // n, key - (key // n) * n
    counts = np.bincount(u, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    g = CSR(n=n, row_ptr=row_ptr.astype(np.int32), col_idx=v.astype(np.int32))
    g.meta.update(model="directed_random", directed=True, dangling=int(dangling.sum()))
    return g


def uneven_batch(num_graphs: int, seed, n_lo: int = 100, n_hi: int = 5000,
                 deg_lo: float = 4.0, deg_hi: float = 32.0, gamma_lo: float = 2.1,
                 gamma_hi: float = 3.0) -> CSR:
    """Block-diagonal batch of independent Chung-Lu graphs of uneven size.

    Graph g has n_g log-uniform in [n_lo, n_hi], average degree uniform in
    [deg_lo, deg_hi] (capped at n_g - 1) and exponent uniform in
    [gamma_lo, gamma_hi]; its own generator is keyed by (seed, g).
    """
    rng = philox(seed)
    ns = np.exp(rng.uniform(np.log(n_lo), np.log(n_hi), size=num_graphs))
    ns = np.rint(ns).astype(np.int64)
    degs = rng.uniform(deg_lo, deg_hi, size=num_graphs)
    gammas = rng.uniform(gamma_lo, gamma_hi, size=num_graphs)
    row_ptrs, cols, graph_ptr = [], [], [0]
    off_v = 0
    off_e = 0
    for gi in range(num_graphs):
        ng = int(ns[gi])
        dg = float(min(degs[gi], 0.5 * (ng - 1)))
        sub = chung_lu(ng, dg, float(gammas[gi]), seed=[int(seed), gi + 1], dmin=1.0,
                       dmax=float(ng - 1))
        row_ptrs.append(sub.row_ptr[:-1].astype(np.int64) + off_e)
        cols.append(sub.col_idx.astype(np.int64) + off_v)
        off_v += sub.n
        off_e += sub.nnz
        graph_ptr.append(off_v)
    row_ptr = np.concatenate(row_ptrs + [np.array([off_e], dtype=np.int64)])
    if off_e >= 2**31:
        raise ValueError("batch too large for int32 CSR")
    out = CSR(n=off_v, row_ptr=row_ptr.astype(np.int32),
              col_idx=np.concatenate(cols).astype(np.int32),
              graph_ptr=np.asarray(graph_ptr, dtype=np.int32))
    out.meta.update(model="uneven_chung_lu_batch", num_graphs=num_graphs)
    return out


# ----------------------------------------------------------------------------
# Tiny structured graphs (closed-form PageRank) and small random graphs
# ----------------------------------------------------------------------------

def cycle(n: int) -> CSR:
    """Cycle C_n (n >= 3): vertex i adjacent to i-1 and i+1 (mod n)."""
    i = np.arange(n)
    return csr_from_edges(n, i, (i + 1) % n)


def complete(n: int) -> CSR:
    """Complete graph K_n."""
    a, b = np.triu_indices(n, 1)
    return csr_from_edges(n, a, b)


def star(n: int) -> CSR:
    """Star: vertex 0 joined to vertices 1..n-1."""
    return csr_from_edges(n, np.zeros(n - 1, dtype=np.int64), np.arange(1, n))


def path(n: int) -> CSR:
    """Path 0-1-...-(n-1)."""
    i = np.arange(n - 1)
    return csr_from_edges(n, i, i + 1)


def random_connected(n: int, avg_deg: float, seed) -> CSR:
    """Small random graph: a random spanning tree plus G(n, p) extra edges.

    Connected, no isolated vertices; handy for dense-matrix checks.
    """
    rng = philox(seed)
    perm = rng.permutation(n)
    parents = np.array([perm[rng.integers(0, i)] for i in range(1, n)], dtype=np.int64)
    u = [perm[1:], ]
    v = [parents, ]
    extra = max(0.0, avg_deg - 2.0 * (n - 1) / n)
    p = min(1.0, extra / max(1, n - 1))
    a, b = np.triu_indices(n, 1)
    pick = rng.random(a.shape[0]) < p
    u.append(a[pick])
    v.append(b[pick])
    return csr_from_edges(n, np.concatenate(u), np.concatenate(v))


# ----------------------------------------------------------------------------
# Personalization vectors
# ----------------------------------------------------------------------------

def random_sources(n: int, count: int, seed, replace: bool = False) -> np.ndarray:
    """``count`` source vertices drawn uniformly at random (int64)."""
    rng = philox(seed)
    if replace or count > n:
        return rng.integers(0, n, size=count)
    return rng.choice(n, size=count, replace=False)


def uniform_personalization(n: int) -> np.ndarray:
    """p = e/n (global PageRank)."""
    return np.full(n, 1.0 / n)


def batch_sources(g: CSR, seed) -> tuple[np.ndarray, np.ndarray]:
    """One uniformly random source per graph of a block-diagonal batch.

    Returns (sources as global vertex ids, concatenated personalization vector
    whose block for graph k is the indicator of its source)."""
    rng = philox(seed)
    gp = g.graph_ptr.astype(np.int64)
    sizes = np.diff(gp)
    src = gp[:-1] + np.floor(rng.random(sizes.shape[0]) * sizes).astype(np.int64)
    p = np.zeros(g.n)
    p[src] = 1.0
    return src, p


def subgraph(g: CSR, k: int) -> CSR:
    """Graph k of a block-diagonal batch, relabelled from 0."""
    v0, v1 = int(g.graph_ptr[k]), int(g.graph_ptr[k + 1])
    e0, e1 = int(g.row_ptr[v0]), int(g.row_ptr[v1])
    return CSR(n=v1 - v0, row_ptr=(g.row_ptr[v0:v1 + 1] - e0).astype(np.int32),
               col_idx=(g.col_idx[e0:e1] - v0).astype(np.int32))


def mpnn_init(seed, layers: int = 3, hidden: int = 64, in_features: int = 2) -> dict:
    """Initial parameters of the warm-start network (Glorot-uniform weights,
    zero biases), FP32.  Keys: w_self{l}, w_nbr{l} (fan_in x hidden), b{l},
    w_out (hidden), b_out (1)."""
    rng = philox(seed)
    params = {}
    fan_in = in_features
    for l in range(layers):
        lim = np.sqrt(6.0 / (fan_in + hidden))
        params[f"w_self{l}"] = rng.uniform(-lim, lim, (fan_in, hidden)).astype(np.float32)
        params[f"w_nbr{l}"] = rng.uniform(-lim, lim, (fan_in, hidden)).astype(np.float32)
        params[f"b{l}"] = np.zeros(hidden, dtype=np.float32)
        fan_in = hidden
    lim = np.sqrt(6.0 / (hidden + 1))
    params["w_out"] = rng.uniform(-lim, lim, hidden).astype(np.float32)
    params["b_out"] = np.zeros(1, dtype=np.float32)
    return params


def source_personalization(n: int, sources) -> np.ndarray:
    """Dense (len(sources), n) FP64 array whose row j is the indicator of sources[j]."""
    sources = np.asarray(sources, dtype=np.int64)
    out = np.zeros((sources.shape[0], n))
    out[np.arange(sources.shape[0]), sources] = 1.0
    return out
