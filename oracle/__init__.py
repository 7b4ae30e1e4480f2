"""Oracle for pattern-morphing counts -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s
``cpu_baseline`` leg may import, call or run anything in this package.  It
shares no code, header, table or helper with the HIP path; the only inputs
they share come from the ``gen`` package of seeded generators.

Contents:
  * ``pattern``: pattern algebra (canonical form, automorphisms, phi(p,q),
    morph coefficients, Theorem 3.1 / Corollary 3.1 in counting form).
  * ``match.c`` (loaded through ctypes): tier A injective-map counting,
    tier A' induced-subgraph census, tier C closed forms, MNI domains.

Every floating-point-free count here is exact (128-bit accumulation in C,
Python integers above it).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from math import comb, factorial

import numpy as np

from . import pattern as P

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile match.c with the host C compiler (plain gcc + OpenMP)."""
    src = os.path.join(_HERE, "match.c")
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(src):
        tmp = _SO + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-Wall",
                               "-o", tmp, src])
        os.replace(tmp, _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        u32p = ctypes.POINTER(ctypes.c_uint32)
        u8p = ctypes.POINTER(ctypes.c_uint8)
        u64p = ctypes.POINTER(ctypes.c_uint64)
        ip = ctypes.POINTER(ctypes.c_int)
        L.or_count_maps.argtypes = [ctypes.c_uint32, u32p, u32p, u8p, ctypes.c_int, ip,
                                    ctypes.c_uint32, ctypes.c_uint32, ip, ctypes.c_uint32,
                                    ctypes.c_uint32, u64p, u64p]
        L.or_mni_maps.argtypes = [ctypes.c_uint32, u32p, u32p, u8p, ctypes.c_int, ip,
                                  ctypes.c_uint32, ctypes.c_uint32, ip, u8p, u64p, u64p]
        L.or_census.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_int, u64p]
        L.or_tier_c4.argtypes = [ctypes.c_uint32, u32p, u32p, u64p]
        L.or_tier_c4_sample.argtypes = [ctypes.c_uint32, u32p, u32p, ctypes.c_uint32, ctypes.c_uint32, u64p]
        L.or_mni_column.argtypes = [ctypes.c_uint32, u32p, u32p, u8p, ctypes.c_int, ip,
                                    ctypes.c_uint32, ctypes.c_uint32, ip, u64p]
        i32p = ctypes.POINTER(ctypes.c_int32)
        L.or_mni_labelings.argtypes = [ctypes.c_uint32, u32p, u32p, u8p, ctypes.c_int, ip,
                                       ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int, i32p,
                                       ctypes.c_int, u64p]
        L.or_list_maps.argtypes = [ctypes.c_uint32, u32p, u32p, u8p, ctypes.c_int, ip,
                                   ctypes.c_uint32, ctypes.c_uint32, ip, ctypes.c_uint64, u32p, u64p]
        L.or_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().or_num_threads())


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _graph_arrays(g):
    rp = np.ascontiguousarray(g.row_ptr, dtype=np.uint32)
    col = np.ascontiguousarray(g.col, dtype=np.uint32)
    if col.size == 0:
        col = np.zeros(1, dtype=np.uint32)
    return rp, col


def _pattern_args(k, mask, induced, plabels):
    order = np.array(P.connected_order(k, mask), dtype=np.int32)
    amask = (P.clique_mask(k) & ~mask) if induced else 0
    pl = np.full(8, -1, dtype=np.int32)
    if plabels is not None:
        pl[:k] = np.asarray(plabels, dtype=np.int32)
    return order, amask, pl


def count_maps(g, k: int, mask: int, induced: bool, plabels=None,
               roots: tuple[int, int] | None = None) -> int:
    """Number of matches (injective maps, Preliminaries) of the pattern,
    restricted to maps whose first-ordered vertex is a root in ``roots``."""
    rp, col = _graph_arrays(g)
    order, amask, pl = _pattern_args(k, mask, induced, plabels)
    lab = None
    if g.labels is not None:
        lab = np.ascontiguousarray(g.labels, dtype=np.uint8)
    lo = ctypes.c_uint64()
    hi = ctypes.c_uint64()
    r0, r1 = roots if roots is not None else (0, g.n)
    rc = lib().or_count_maps(g.n, _ptr(rp, ctypes.c_uint32), _ptr(col, ctypes.c_uint32),
                             None if lab is None else _ptr(lab, ctypes.c_uint8), k,
                             _ptr(order, ctypes.c_int), mask, amask,
                             _ptr(pl, ctypes.c_int), r0, r1, ctypes.byref(lo),
                             ctypes.byref(hi))
    if rc != 0:
        raise ValueError(f"or_count_maps failed: {rc}")
    return (hi.value << 64) | lo.value


def count(g, k: int, mask: int, induced: bool, plabels=None) -> int:
    """Distinct subgraphs = #matches / |Aut(p)| (label-preserving Aut)."""
    maps = count_maps(g, k, mask, induced, plabels)
    aut = P.num_automorphisms(k, mask, plabels)
    assert maps % aut == 0
    return maps // aut


def motif_counts(g, k: int, induced: bool) -> dict:
    """Tier A counts for every connected class on k vertices."""
    return {m: count(g, k, m, induced) for m in P.connected_classes(k)}


def census(g, k: int) -> dict:
    """Tier A': vertex-induced counts of every connected class, from the
    connected-induced-subgraph census."""
    rp, col = _graph_arrays(g)
    nh = 1 << P.num_pairs(k)
    hist = np.zeros(nh, dtype=np.uint64)
    rc = lib().or_census(g.n, _ptr(rp, ctypes.c_uint32), _ptr(col, ctypes.c_uint32), k,
                         _ptr(hist, ctypes.c_uint64))
    if rc != 0:
        raise ValueError(f"or_census failed: {rc}")
    cls = P.class_of_mask(k)
    out = {m: 0 for m in P.connected_classes(k)}
    for raw in np.nonzero(hist)[0]:
        out[cls[int(raw)]] += int(hist[raw])
    return out


def full_census_tiny(g, k: int) -> dict:
    """Every k-subset (connected or not) classified; tiny graphs only."""
    from itertools import combinations
    cls = P.class_of_mask(k)
    adj = set()
    for v in range(g.n):
        for w in g.neighbors(v):
            adj.add((v, int(w)))
    out = {m: 0 for m in P.all_classes(k)}
    for sub in combinations(range(g.n), k):
        mask = 0
        for j in range(k):
            for i in range(j):
                if (sub[i], sub[j]) in adj:
                    mask |= 1 << P.pair_bit(i, j)
        out[cls[mask]] += 1
    return out


TIER_C4_KEYS = ("edges", "wedges", "triangles", "star3", "path4", "tailed_triangle",
                "cycle4", "diamond", "clique4")


def tier_c4(g) -> dict:
    """Closed-form edge-induced counts for 3- and 4-vertex patterns."""
    rp, col = _graph_arrays(g)
    out = np.zeros(2 * len(TIER_C4_KEYS), dtype=np.uint64)
    rc = lib().or_tier_c4(g.n, _ptr(rp, ctypes.c_uint32), _ptr(col, ctypes.c_uint32),
                          _ptr(out, ctypes.c_uint64))
    if rc != 0:
        raise ValueError(f"or_tier_c4 failed: {rc}")
    return {key: (int(out[2 * i + 1]) << 64) | int(out[2 * i])
            for i, key in enumerate(TIER_C4_KEYS)}


def tier_c4_sample(g, stride: int, offset: int) -> dict:
    """The closed forms of tier_c4 credited to the roots u with
    u % stride == offset, as raw sums (triangles counted 3 times, the 3-path
    slot holding P4 + 3T, 4-cycles counted twice); over every offset they
    add up to tier_c4's raw sums."""
    rp, col = _graph_arrays(g)
    out = np.zeros(2 * len(TIER_C4_KEYS), dtype=np.uint64)
    rc = lib().or_tier_c4_sample(g.n, _ptr(rp, ctypes.c_uint32), _ptr(col, ctypes.c_uint32), stride, offset,
                                 _ptr(out, ctypes.c_uint64))
    if rc != 0:
        raise ValueError(f"or_tier_c4_sample failed: {rc}")
    return {key: (int(out[2 * i + 1]) << 64) | int(out[2 * i])
            for i, key in enumerate(TIER_C4_KEYS)}


def tier_c4_from_raw(raw: dict) -> dict:
    """tier_c4's values from summed raw sums (exact divisions)."""
    out = dict(raw)
    assert raw["triangles"] % 3 == 0 and raw["cycle4"] % 2 == 0
    out["triangles"] = raw["triangles"] // 3
    out["path4"] = raw["path4"] - raw["triangles"]
    out["cycle4"] = raw["cycle4"] // 2
    return out


# canonical masks of the named 4-vertex classes
def named_4():
    """Canonical masks of the six connected 4-vertex classes by name."""
    def canon(edges):
        m = 0
        for i, j in edges:
            m |= 1 << P.pair_bit(i, j)
        return P.canonical(4, m)[0]
    return {
        "star3": canon([(0, 1), (0, 2), (0, 3)]),
        "path4": canon([(0, 1), (1, 2), (2, 3)]),
        "tailed_triangle": canon([(0, 1), (1, 2), (0, 2), (0, 3)]),
        "cycle4": canon([(0, 1), (1, 2), (2, 3), (0, 3)]),
        "diamond": canon([(0, 1), (1, 2), (2, 3), (0, 3), (0, 2)]),
        "clique4": P.clique_mask(4),
    }


def edge_induced_4_from_tier_c(g) -> dict:
    """Tier C edge-induced counts keyed by canonical 4-vertex mask."""
    t = tier_c4(g)
    names = named_4()
    return {names[k]: t[k] for k in names}


def vertex_induced_4_from_tier_c(g) -> dict:
    """Vertex-induced 4-vertex counts derived by Corollary 3.1 from tier C."""
    return P.vertex_induced_from_edge_induced(4, edge_induced_4_from_tier_c(g))


def mni_domains(g, k: int, mask: int, induced: bool, plabels=None) -> np.ndarray:
    """bool[k, n]: domain of each pattern vertex over ALL matches."""
    rp, col = _graph_arrays(g)
    order, amask, pl = _pattern_args(k, mask, induced, plabels)
    lab = None
    if g.labels is not None:
        lab = np.ascontiguousarray(g.labels, dtype=np.uint8)
    dom = np.zeros((k, g.n), dtype=np.uint8)
    lo = ctypes.c_uint64()
    hi = ctypes.c_uint64()
    rc = lib().or_mni_maps(g.n, _ptr(rp, ctypes.c_uint32), _ptr(col, ctypes.c_uint32),
                           None if lab is None else _ptr(lab, ctypes.c_uint8), k,
                           _ptr(order, ctypes.c_int), mask, amask, _ptr(pl, ctypes.c_int),
                           _ptr(dom, ctypes.c_uint8), ctypes.byref(lo), ctypes.byref(hi))
    if rc != 0:
        raise ValueError(f"or_mni_maps failed: {rc}")
    return dom.astype(bool)


def mni_support(g, k: int, mask: int, induced: bool, plabels=None) -> int:
    """MNI support: the smallest pattern-vertex domain (Preliminaries, FSM)."""
    dom = mni_domains(g, k, mask, induced, plabels)
    return int(dom.sum(axis=1).min()) if k > 0 else 0


def _rooted_order(k, mask, v):
    order = [v]
    seen = {v}
    i = 0
    while i < len(order):
        x = order[i]
        i += 1
        for y in range(k):
            if y not in seen and P.has_edge(mask, x, y):
                seen.add(y)
                order.append(y)
    assert len(order) == k, "pattern is not connected"
    return order


def mni_column(g, k: int, mask: int, induced: bool, plabels, v: int) -> int:
    """|D(v)| by rooted existence search (large graphs)."""
    rp, col = _graph_arrays(g)
    order = np.array(_rooted_order(k, mask, v), dtype=np.int32)
    amask = (P.clique_mask(k) & ~mask) if induced else 0
    pl = np.full(8, -1, dtype=np.int32)
    if plabels is not None:
        pl[:k] = np.asarray(plabels, dtype=np.int32)
    lab = np.ascontiguousarray(g.labels, dtype=np.uint8)
    out = ctypes.c_uint64()
    rc = lib().or_mni_column(g.n, _ptr(rp, ctypes.c_uint32), _ptr(col, ctypes.c_uint32),
                             _ptr(lab, ctypes.c_uint8), k, _ptr(order, ctypes.c_int), mask, amask,
                             _ptr(pl, ctypes.c_int), ctypes.byref(out))
    if rc != 0:
        raise ValueError(f"or_mni_column failed: {rc}")
    return int(out.value)


def mni_support_rooted(g, k: int, mask: int, induced: bool, plabels) -> int:
    """MNI support as the smallest column, each column by rooted search."""
    return min(mni_column(g, k, mask, induced, plabels, v) for v in range(k))


def list_maps(g, k: int, mask: int, induced: bool, plabels=None) -> np.ndarray:
    """Every match (Preliminaries: injective map preserving edges, anti-edges
    when vertex-induced, and labels) as rows of k data vertices in
    pattern-vertex order; tiny graphs only."""
    rp, col = _graph_arrays(g)
    order, amask, pl = _pattern_args(k, mask, induced, plabels)
    lab = None
    if g.labels is not None:
        lab = np.ascontiguousarray(g.labels, dtype=np.uint8)
    cap = max(1, count_maps(g, k, mask, induced, plabels))
    out = np.zeros(cap * k, dtype=np.uint32)
    cnt = ctypes.c_uint64()
    rc = lib().or_list_maps(g.n, _ptr(rp, ctypes.c_uint32), _ptr(col, ctypes.c_uint32),
                            None if lab is None else _ptr(lab, ctypes.c_uint8), k,
                            _ptr(order, ctypes.c_int), mask, amask, _ptr(pl, ctypes.c_int), cap,
                            _ptr(out, ctypes.c_uint32), ctypes.byref(cnt))
    if rc != 0:
        raise ValueError(f"or_list_maps failed: {rc}")
    return out[: cnt.value * k].reshape(cnt.value, k)


def mni_labelings(g, k: int, mask: int, induced: bool, num_labels: int, labelings) -> list[int]:
    """MNI support of several labelings of one pattern shape at once.

    ``labelings`` is a list of label tuples (label of pattern vertex 0..k-1).
    Every match of the unlabeled shape is a match of exactly one labeled
    pattern: the one whose vertex v carries the label of its image
    (Preliminaries, "Graph Isomorphism" with labels).  All matches are
    enumerated once and each pattern vertex's image goes into the column of
    that labeling; the support is the smallest column (Preliminaries, FSM)."""
    rp, col = _graph_arrays(g)
    order = np.array(P.connected_order(k, mask), dtype=np.int32)
    amask = (P.clique_mask(k) & ~mask) if induced else 0
    lab = np.ascontiguousarray(g.labels, dtype=np.uint8)
    sel = np.full(num_labels ** k, -1, dtype=np.int32)
    keys = []
    for t in labelings:
        key = 0
        for v in reversed(range(k)):
            key = key * num_labels + int(t[v])
        keys.append(key)
    uniq = sorted(set(keys))
    for i, key in enumerate(uniq):
        sel[key] = i
    out = np.zeros(len(uniq) * k, dtype=np.uint64)
    rc = lib().or_mni_labelings(g.n, _ptr(rp, ctypes.c_uint32), _ptr(col, ctypes.c_uint32),
                                _ptr(lab, ctypes.c_uint8), k, _ptr(order, ctypes.c_int), mask,
                                amask, num_labels, _ptr(sel, ctypes.c_int32), len(uniq),
                                _ptr(out, ctypes.c_uint64))
    if rc != 0:
        raise ValueError(f"or_mni_labelings failed: {rc}")
    cols = out.reshape(len(uniq), k)
    return [int(cols[sel[key]].min()) for key in keys]


__all__ = ["P", "build", "lib", "count_maps", "count", "motif_counts", "census",
           "full_census_tiny", "tier_c4", "named_4", "edge_induced_4_from_tier_c",
           "vertex_induced_4_from_tier_c", "mni_domains", "mni_support", "num_threads",
           "mni_column", "mni_support_rooted", "mni_labelings", "list_maps", "tier_c4_sample", "tier_c4_from_raw",
           "comb", "factorial"]
