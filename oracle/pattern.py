"""Oracle pattern algebra -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path never calls it.

Plain, slow, obviously-correct definitions from the paper's Preliminaries
and Section 3.2 (Semantics of Pattern Morphing):

* A pattern is a simple connected graph on k vertices, optionally labeled.
  Its edges are stored as a bitmask: pair (i<j) is bit ``j*(j-1)/2 + i``.
  A vertex-induced pattern carries an anti-edge on every non-adjacent pair;
  an edge-induced pattern carries none (Preliminaries, "Pattern Semantics").
* A subgraph isomorphism between two patterns on the same k vertices is a
  permutation that maps edges to edges (and anti-edges to anti-edges); the
  set of them is phi(p, q) (Section 3.2.1, "Subgraph Isomorphisms").
* The morph coefficient c(p, q) = |phi(p^E, q^E)| / |Aut(p)| is the number of
  distinct copies of p inside one copy of q, so that for every data graph
  N_E(p) = sum_q c(p, q) N_V(q) over the same-size superpatterns q of p
  (counting form of Theorem 3.1 / Theorem 3.2 with lambda = size, + = sum),
  and vertex-induced counts follow by back-substitution (Corollary 3.1,
  recursion ending at the clique).
* Counts are reported as distinct subgraphs: #matches / |Aut(p)|, where a
  match is an injective map (Preliminaries, "match") and automorphisms are
  label-preserving when labels are present.
"""
from __future__ import annotations

from functools import lru_cache
from itertools import permutations
from math import comb


def pair_bit(i: int, j: int) -> int:
    if i > j:
        i, j = j, i
    return j * (j - 1) // 2 + i


def num_pairs(k: int) -> int:
    return k * (k - 1) // 2


def has_edge(mask: int, i: int, j: int) -> bool:
    return bool((mask >> pair_bit(i, j)) & 1)


def edges_of(k: int, mask: int) -> list[tuple[int, int]]:
    return [(i, j) for j in range(k) for i in range(j) if has_edge(mask, i, j)]


def edge_count(mask: int) -> int:
    return bin(mask).count("1")


def permute_mask(k: int, mask: int, perm) -> int:
    """Image of the edge set under vertex map i -> perm[i]."""
    out = 0
    for (i, j) in edges_of(k, mask):
        out |= 1 << pair_bit(perm[i], perm[j])
    return out


def is_connected(k: int, mask: int) -> bool:
    if k == 1:
        return True
    seen = {0}
    stack = [0]
    while stack:
        x = stack.pop()
        for y in range(k):
            if y != x and y not in seen and has_edge(mask, x, y):
                seen.add(y)
                stack.append(y)
    return len(seen) == k


def _labels_tuple(k: int, labels) -> tuple:
    if labels is None:
        return tuple([-1] * k)
    return tuple(int(x) for x in labels)


def canonical(k: int, mask: int, labels=None) -> tuple[int, tuple]:
    """Smallest (mask, labels) over all relabellings of the k vertices."""
    lab = _labels_tuple(k, labels)
    best = None
    for perm in permutations(range(k)):
        m2 = permute_mask(k, mask, perm)
        l2 = [0] * k
        for i in range(k):
            l2[perm[i]] = lab[i]
        key = (m2, tuple(l2))
        if best is None or key < best:
            best = key
    return best


def automorphisms(k: int, mask: int, labels=None) -> list[tuple[int, ...]]:
    lab = _labels_tuple(k, labels)
    out = []
    for perm in permutations(range(k)):
        if permute_mask(k, mask, perm) != mask:
            continue
        if any(lab[perm[i]] != lab[i] for i in range(k)):
            continue
        out.append(perm)
    return out


def num_automorphisms(k: int, mask: int, labels=None) -> int:
    return len(automorphisms(k, mask, labels))


@lru_cache(maxsize=None)
def connected_classes(k: int) -> tuple[int, ...]:
    """Canonical edge masks of all connected unlabeled graphs on k vertices,
    sorted by (edge count, mask)."""
    seen = set()
    for mask in range(1 << num_pairs(k)):
        if not is_connected(k, mask):
            continue
        seen.add(canonical(k, mask)[0])
    return tuple(sorted(seen, key=lambda m: (edge_count(m), m)))


@lru_cache(maxsize=None)
def all_classes(k: int) -> tuple[int, ...]:
    seen = set()
    for mask in range(1 << num_pairs(k)):
        seen.add(canonical(k, mask)[0])
    return tuple(sorted(seen, key=lambda m: (edge_count(m), m)))


@lru_cache(maxsize=None)
def class_of_mask(k: int) -> dict:
    """Raw mask -> canonical mask, for every mask on k vertices."""
    return {m: canonical(k, m)[0] for m in range(1 << num_pairs(k))}


def subgraph_isomorphisms(k: int, p_mask: int, q_mask: int, p_labels=None,
                          q_labels=None, induced: bool = False):
    """phi(p, q) for two patterns on the same k vertices: permutations f with
    f(E(p)) subset of E(q), labels preserved.  With ``induced`` both are read
    as vertex-induced, so anti-edges must map to anti-edges too (then f must
    be an isomorphism)."""
    pl = _labels_tuple(k, p_labels)
    ql = _labels_tuple(k, q_labels)
    out = []
    for f in permutations(range(k)):
        if any(pl[i] != ql[f[i]] for i in range(k)):
            continue
        img = permute_mask(k, p_mask, f)
        if img & ~q_mask:
            continue
        if induced and img != q_mask:
            continue
        out.append(f)
    return out


def coefficient(k: int, p_mask: int, q_mask: int, p_labels=None,
                q_labels=None) -> int:
    """c(p, q) = |phi(p^E, q^E)| / |Aut(p)| (exact: phi is a union of
    right cosets of Aut(p))."""
    phi = len(subgraph_isomorphisms(k, p_mask, q_mask, p_labels, q_labels))
    aut = num_automorphisms(k, p_mask, p_labels)
    assert phi % aut == 0, (p_mask, q_mask, phi, aut)
    return phi // aut


def morph_matrix(k: int, classes=None) -> tuple[tuple[int, ...], list[list[int]]]:
    """Forward morph matrix C with N_E = C @ N_V over the given unlabeled
    classes (default: all connected classes on k vertices)."""
    cls = tuple(classes) if classes is not None else connected_classes(k)
    mat = [[coefficient(k, p, q) for q in cls] for p in cls]
    return cls, mat


def vertex_induced_from_edge_induced(k: int, n_e: dict, classes=None) -> dict:
    """Corollary 3.1 back-substitution: starting at the clique (most edges),
    N_V(p) = N_E(p) - sum_{q superpattern, q != p} c(p, q) N_V(q)."""
    cls = tuple(classes) if classes is not None else connected_classes(k)
    order = sorted(cls, key=lambda m: (-edge_count(m), m))
    n_v = {}
    for p in order:
        acc = int(n_e[p])
        for q in order:
            if q == p or q not in n_v:
                continue
            c = coefficient(k, p, q)
            acc -= c * n_v[q]
        n_v[p] = acc
    return n_v


def edge_induced_from_vertex_induced(k: int, n_v: dict, classes=None) -> dict:
    """Theorem 3.1 (counting form): N_E(p) = sum_q c(p, q) N_V(q)."""
    cls = tuple(classes) if classes is not None else connected_classes(k)
    return {p: sum(coefficient(k, p, q) * int(n_v[q]) for q in cls) for p in cls}


def labeled_connected_count(k: int) -> int:
    """Number of labelled (vertex-numbered) connected graphs on k vertices
    obtained as sum over classes of k!/|Aut|."""
    from math import factorial
    return sum(factorial(k) // num_automorphisms(k, m) for m in connected_classes(k))


def clique_mask(k: int) -> int:
    return (1 << num_pairs(k)) - 1


def connected_order(k: int, mask: int) -> list[int]:
    """A vertex order in which every vertex after the first has an earlier
    neighbour (BFS from vertex 0)."""
    order = [0]
    seen = {0}
    i = 0
    while i < len(order):
        x = order[i]
        i += 1
        for y in range(k):
            if y not in seen and has_edge(mask, x, y):
                seen.add(y)
                order.append(y)
    assert len(order) == k, "pattern is not connected"
    return order


__all__ = [name for name in dir() if not name.startswith("_")] + ["comb"]
