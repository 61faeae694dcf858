"""Seeded graph and starting-point generators.

Every graph is returned as an undirected edge list with canonical orientation
``i < j``, no self loops and no duplicate pairs, plus one weight per edge.
"""

from dataclasses import dataclass

import numpy as np


@dataclass
class Graph:
    """Undirected weighted graph: edges (ei[k], ej[k]) with ei[k] < ej[k]."""

    n: int
    ei: np.ndarray  # int64, length M
    ej: np.ndarray  # int64, length M
    w: np.ndarray   # float64, length M

    @property
    def m_edges(self) -> int:
        return int(self.ei.shape[0])


def draw_weights(rng, m, kind):
    """Edge weights: 'unit' (all 1), 'pm1' (uniform in {+1,-1}), 'gauss' (N(0,1))."""
    if kind == "unit":
        return np.ones(m, dtype=np.float64)
    if kind == "pm1":
        return rng.choice(np.array([-1.0, 1.0]), size=m)
    if kind == "gauss":
        return rng.standard_normal(m)
    raise ValueError(f"unknown weight kind {kind!r}")


def _canonical_sorted(n, i, j):
    lo = np.minimum(i, j).astype(np.int64)
    hi = np.maximum(i, j).astype(np.int64)
    key = lo * np.int64(n) + hi
    order = np.argsort(key, kind="stable")
    return lo[order], hi[order]


def er_graph(n, m_edges, seed, weights="unit"):
    """Erdos-Renyi G(n, M): a uniformly random set of M distinct pairs i != j.

    Pairs are drawn uniformly in batches (self pairs dropped) until at least M
    distinct pairs are held; a uniformly random M-subset of them is kept, which
    is again a uniform M-subset of all pairs.  Edges are sorted by (i, j) and
    weights are drawn in that order.
    """
    n = int(n)
    m_edges = int(m_edges)
    if m_edges > n * (n - 1) // 2:
        raise ValueError("more edges than pairs")
    rng = np.random.default_rng(seed)
    keys = np.empty(0, dtype=np.int64)
    while keys.shape[0] < m_edges:
        need = m_edges - keys.shape[0]
        k = int(need * 1.02) + 64
        a = rng.integers(0, n, size=k, dtype=np.int64)
        b = rng.integers(0, n, size=k, dtype=np.int64)
        keep = a != b
        a, b = a[keep], b[keep]
        new = np.minimum(a, b) * np.int64(n) + np.maximum(a, b)
        keys = np.unique(np.concatenate([keys, new]))
    if keys.shape[0] > m_edges:
        pick = rng.choice(keys.shape[0], size=m_edges, replace=False)
        keys = np.sort(keys[pick])
    ei = keys // n
    ej = keys % n
    w = draw_weights(rng, m_edges, weights)
    return Graph(n, ei, ej, w)


def torus_graph(rows, cols, seed, weights="pm1"):
    """2-D toroidal grid: vertex v = a*cols + b joined to (a+1 mod rows, b) and
    (a, b+1 mod cols).  Every vertex has degree exactly 4 when rows, cols >= 3."""
    rng = np.random.default_rng(seed)
    a, b = np.meshgrid(np.arange(rows, dtype=np.int64), np.arange(cols, dtype=np.int64),
                       indexing="ij")
    v = (a * cols + b).ravel()
    down = (((a + 1) % rows) * cols + b).ravel()
    right = (a * cols + (b + 1) % cols).ravel()
    i = np.concatenate([v, v])
    j = np.concatenate([down, right])
    ei, ej = _canonical_sorted(rows * cols, i, j)
    w = draw_weights(rng, ei.shape[0], weights)
    return Graph(rows * cols, ei, ej, w)


def cycle_graph(n, weights=None):
    i = np.arange(n, dtype=np.int64)
    ei, ej = _canonical_sorted(n, i, (i + 1) % n)
    w = np.ones(ei.shape[0]) if weights is None else np.asarray(weights, dtype=np.float64)
    return Graph(n, ei, ej, w)


def complete_graph(n):
    ei, ej = np.triu_indices(n, 1)
    return Graph(n, ei.astype(np.int64), ej.astype(np.int64), np.ones(ei.shape[0]))


def complete_bipartite_graph(p, q):
    a = np.repeat(np.arange(p, dtype=np.int64), q)
    b = np.tile(np.arange(p, p + q, dtype=np.int64), p)
    ei, ej = _canonical_sorted(p + q, a, b)
    return Graph(p + q, ei, ej, np.ones(ei.shape[0]))


def edgeless_graph(n):
    z = np.zeros(0, dtype=np.int64)
    return Graph(n, z, z.copy(), np.zeros(0))


def rmat_graph(scale, edge_factor, seed, weights="unit", abcd=(0.57, 0.19, 0.19, 0.05)):
    """R-MAT (Kronecker) graph with 2**scale vertices and about edge_factor*2**scale
    distinct edges (self loops and duplicates dropped, not resampled)."""
    rng = np.random.default_rng(seed)
    n = 1 << scale
    m = edge_factor * n
    a, b, c, _ = abcd
    i = np.zeros(m, dtype=np.int64)
    j = np.zeros(m, dtype=np.int64)
    for bit in range(scale):
        u = rng.random(m)
        ib = (u >= a + b).astype(np.int64)
        jb = (((u >= a) & (u < a + b)) | (u >= a + b + c)).astype(np.int64)
        i |= ib << bit
        j |= jb << bit
    keep = i != j
    lo = np.minimum(i[keep], j[keep])
    hi = np.maximum(i[keep], j[keep])
    keys = np.unique(lo * n + hi)
    ei, ej = keys // n, keys % n
    return Graph(n, ei, ej, draw_weights(rng, ei.shape[0], weights))


def batch_instances(count, seed, n_lo=1e3, n_hi=2e5, deg_lo=4.0, deg_hi=32.0,
                    ranks=(8, 16), weights="pm1"):
    """Uneven batch of MaxCut graphs: n_i log-uniform in [n_lo, n_hi], average
    degree uniform in [deg_lo, deg_hi], M_i = round(n_i * d_i / 2), rank drawn
    uniformly from ``ranks``.  Instance i uses seed ``seed*1000 + i``."""
    out = []
    for k in range(count):
        s = seed * 1000 + k
        rng = np.random.default_rng(s)
        n = int(round(float(np.exp(rng.uniform(np.log(n_lo), np.log(n_hi))))))
        d = float(rng.uniform(deg_lo, deg_hi))
        m = int(round(n * d / 2))
        m = min(m, n * (n - 1) // 2)
        r = int(rng.choice(np.asarray(ranks)))
        g = er_graph(n, m, s, weights)
        out.append((g, r))
    return out


def init_factor(n, r, seed):
    """Starting factor: i.i.d. N(0,1) entries, each row scaled to unit length."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((int(n), int(r)))
    nrm = np.sqrt(np.sum(x * x, axis=1))
    nrm[nrm == 0.0] = 1.0
    return x / nrm[:, None]
