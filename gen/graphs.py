"""Seeded graph generators producing simple undirected graphs as CSR.

Every generator returns a :class:`Graph` whose adjacency lists are sorted
ascending, symmetric, free of self-loops and duplicates, with every vertex
kept (degree-0 vertices included).  Vertex ids are the generator's own; no
degree ordering is applied here (that is part of graph ingest on the device
side and is deliberately not shared with the oracle).

Recipes (the data-graph model is the paper's simple graph of the
Preliminaries; the paper's datasets are not available, these stand in):

* ``erdos_renyi(n, p, seed)``: every unordered pair independently with
  probability p.
* ``rmat(scale, edge_factor, a, b, c, d, seed)``: ``edge_factor * 2**scale``
  directed draws, each choosing one quadrant per bit level with
  probabilities (a, b, c, d); self-loops dropped, pairs symmetrised and
  deduplicated; then a seeded random relabelling of the vertices.
* ``chung_lu(n, beta, mean_degree, seed)``: weights ``(i+1)^(-1/(beta-1))``
  scaled to the mean degree and capped at ``sqrt(sum w)``; ``mean_degree*n/2``
  edges drawn with both endpoints proportional to weight; self-loops and
  duplicates dropped.
* ``zipf_labels(n, num_labels, s, seed)``: i.i.d. labels with
  ``P(l) proportional to (l+1)^(-s)``.
"""
from __future__ import annotations

import hashlib
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Graph:
    n: int
    row_ptr: np.ndarray  # uint32[n+1]
    col: np.ndarray  # uint32[2m], each row sorted ascending
    labels: np.ndarray | None = None  # uint8[n] or None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return int(self.row_ptr[-1]) // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr.astype(np.int64))

    def neighbors(self, v: int) -> np.ndarray:
        return self.col[self.row_ptr[v]:self.row_ptr[v + 1]]

    def with_labels(self, labels: np.ndarray | None) -> "Graph":
        return Graph(self.n, self.row_ptr, self.col,
                     None if labels is None else np.ascontiguousarray(labels, dtype=np.uint8),
                     self.name, dict(self.meta))

    def edges(self) -> np.ndarray:
        """Undirected edges (u < v) as an int64[m, 2] array."""
        deg = self.degrees()
        src = np.repeat(np.arange(self.n, dtype=np.int64), deg)
        dst = self.col.astype(np.int64)
        keep = src < dst
        return np.stack([src[keep], dst[keep]], axis=1)


def sha256_of(g: Graph) -> str:
    h = hashlib.sha256()
    h.update(np.uint64(g.n).tobytes())
    h.update(np.ascontiguousarray(g.row_ptr, dtype=np.uint32).tobytes())
    h.update(np.ascontiguousarray(g.col, dtype=np.uint32).tobytes())
    if g.labels is not None:
        h.update(np.ascontiguousarray(g.labels, dtype=np.uint8).tobytes())
    return h.hexdigest()


def from_edges(n: int, u: np.ndarray, v: np.ndarray, name: str = "") -> Graph:
    """Build a simple undirected CSR from endpoint arrays (any direction,
    duplicates and self-loops allowed: they are removed)."""
    u = np.asarray(u, dtype=np.int64).ravel()
    v = np.asarray(v, dtype=np.int64).ravel()
    keep = u != v
    u, v = u[keep], v[keep]
    lo = np.minimum(u, v)
    hi = np.maximum(u, v)
    key = np.unique(lo * np.int64(n) + hi)
    lo = key // n
    hi = key % n
    src = np.concatenate([lo, hi])
    dst = np.concatenate([hi, lo])
    order = np.lexsort((dst, src))
    src = src[order]
    dst = dst[order]
    counts = np.bincount(src, minlength=n)
    row_ptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=row_ptr[1:])
    if row_ptr[-1] >= 2**32:
        raise ValueError("graph too large for uint32 CSR")
    return Graph(n, row_ptr.astype(np.uint32), dst.astype(np.uint32), None, name)


def erdos_renyi(n: int, p: float, seed: int) -> Graph:
    rng = np.random.Generator(np.random.PCG64(seed))
    iu, ju = np.triu_indices(n, k=1)
    keep = rng.random(iu.shape[0]) < p
    g = from_edges(n, iu[keep], ju[keep], name=f"er_n{n}_p{p}_s{seed}")
    g.meta.update(kind="erdos_renyi", n=n, p=p, seed=seed)
    return g


def rmat(scale: int, edge_factor: int, a: float = 0.57, b: float = 0.19,
         c: float = 0.19, d: float = 0.05, seed: int = 0,
         chunk: int = 1 << 22) -> Graph:
    n = 1 << scale
    draws = edge_factor * n
    rng = np.random.Generator(np.random.PCG64(seed))
    us = []
    vs = []
    ab = a + b
    abc = a + b + c
    done = 0
    while done < draws:
        cnt = min(chunk, draws - done)
        u = np.zeros(cnt, dtype=np.int64)
        v = np.zeros(cnt, dtype=np.int64)
        for bit in range(scale):
            r = rng.random(cnt)
            ubit = (r >= ab).astype(np.int64)           # quadrants c, d
            vbit = (((r >= a) & (r < ab)) | (r >= abc)).astype(np.int64)  # b, d
            u |= ubit << bit
            v |= vbit << bit
        us.append(u)
        vs.append(v)
        done += cnt
    u = np.concatenate(us)
    v = np.concatenate(vs)
    perm = rng.permutation(n).astype(np.int64)
    g = from_edges(n, perm[u], perm[v],
                   name=f"rmat_s{scale}_ef{edge_factor}_s{seed}")
    g.meta.update(kind="rmat", scale=scale, edge_factor=edge_factor,
                  abcd=(a, b, c, d), seed=seed)
    return g


def chung_lu(n: int, beta: float = 2.1, mean_degree: float = 20.0,
             seed: int = 0) -> Graph:
    rng = np.random.Generator(np.random.PCG64(seed))
    w = (np.arange(n, dtype=np.float64) + 1.0) ** (-1.0 / (beta - 1.0))
    w *= mean_degree / w.mean()
    cap = np.sqrt(w.sum())
    w = np.minimum(w, cap)
    prob = w / w.sum()
    cdf = np.cumsum(prob)
    cdf[-1] = 1.0
    m_draw = int(round(mean_degree * n / 2))
    u = np.searchsorted(cdf, rng.random(m_draw), side="right")
    v = np.searchsorted(cdf, rng.random(m_draw), side="right")
    perm = rng.permutation(n).astype(np.int64)
    g = from_edges(n, perm[u], perm[v], name=f"chunglu_n{n}_b{beta}_s{seed}")
    g.meta.update(kind="chung_lu", n=n, beta=beta, mean_degree=mean_degree,
                  seed=seed, weight_cap=float(cap))
    return g


def zipf_labels(n: int, num_labels: int = 16, s: float = 1.2,
                seed: int = 0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    p = (np.arange(num_labels, dtype=np.float64) + 1.0) ** (-s)
    p /= p.sum()
    return rng.choice(num_labels, size=n, p=p).astype(np.uint8)


# ---- small structured graphs used as special cases -------------------------

def complete_graph(n: int) -> Graph:
    iu, ju = np.triu_indices(n, k=1)
    return from_edges(n, iu, ju, name=f"K{n}")


def complete_bipartite(a: int, b: int) -> Graph:
    u, v = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_edges(a + b, u.ravel(), v.ravel(), name=f"K{a},{b}")


def star_graph(leaves: int) -> Graph:
    return from_edges(leaves + 1, np.zeros(leaves, dtype=np.int64),
                      np.arange(1, leaves + 1), name=f"star{leaves}")


def cycle_graph(n: int) -> Graph:
    u = np.arange(n)
    return from_edges(n, u, (u + 1) % n, name=f"C{n}")


def graph_from_mask(n: int, mask: int) -> Graph:
    """Graph on n vertices whose edge (i<j) is present when bit
    ``j*(j-1)/2 + i`` of ``mask`` is set."""
    us, vs = [], []
    for j in range(n):
        for i in range(j):
            if (mask >> (j * (j - 1) // 2 + i)) & 1:
                us.append(i)
                vs.append(j)
    return from_edges(n, np.array(us, dtype=np.int64), np.array(vs, dtype=np.int64),
                      name=f"mask{n}_{mask}")
