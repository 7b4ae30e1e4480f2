"""Seeded query streams for the serving workload.

Per query: a resident graph chosen uniformly; a vertex count k uniform over
{3, 4, 5}; 1-4 patterns whose topology is uniform over the connected
k-vertex classes; vertex- or edge-induced with probability 1/2 each;
labeled with probability `p_labeled`, pattern labels drawn from the same
truncated Zipf as the vertex labels.  Arrivals form a Poisson process
(exponential inter-arrival times).  Pure input generation: the connected
classes are listed by brute force over edge masks, nothing else.
"""
from __future__ import annotations

from dataclasses import dataclass
from functools import lru_cache
from itertools import permutations

import numpy as np


def _bit(i: int, j: int) -> int:
    if i > j:
        i, j = j, i
    return j * (j - 1) // 2 + i


def _connected(k: int, mask: int) -> bool:
    seen = {0}
    stack = [0]
    while stack:
        x = stack.pop()
        for y in range(k):
            if y not in seen and (mask >> _bit(x, y)) & 1:
                seen.add(y)
                stack.append(y)
    return len(seen) == k


@lru_cache(maxsize=None)
def connected_masks(k: int) -> tuple[int, ...]:
    """One representative edge mask per connected k-vertex class."""
    reps = set()
    for mask in range(1 << (k * (k - 1) // 2)):
        if not _connected(k, mask):
            continue
        best = None
        for p in permutations(range(k)):
            m2 = 0
            for j in range(k):
                for i in range(j):
                    if (mask >> _bit(i, j)) & 1:
                        m2 |= 1 << _bit(p[i], p[j])
            best = m2 if best is None or m2 < best else best
        reps.add(best)
    return tuple(sorted(reps))


@dataclass
class Query:
    arrival_s: float
    graph: int                 # index into the list of resident graphs
    patterns: list             # [(k, edge_mask, induced, labels or None)]


def query_stream(n_queries: int, qps: float, n_graphs: int, num_labels: int = 16,
                 zipf_s: float = 1.2, p_labeled: float = 0.3, seed: int = 56,
                 k_choices=(3, 4, 5), max_patterns: int = 4) -> list[Query]:
    rng = np.random.Generator(np.random.PCG64(seed))
    lp = (np.arange(num_labels, dtype=np.float64) + 1.0) ** (-zipf_s)
    lp /= lp.sum()
    t = 0.0
    out = []
    for _ in range(n_queries):
        t += rng.exponential(1.0 / qps)
        g = int(rng.integers(0, n_graphs))
        k = int(rng.choice(k_choices))
        classes = connected_masks(k)
        npat = int(rng.integers(1, max_patterns + 1))
        pats = []
        for _ in range(npat):
            mask = int(classes[int(rng.integers(0, len(classes)))])
            induced = bool(rng.random() < 0.5)
            labels = None
            if rng.random() < p_labeled:
                labels = [int(x) for x in rng.choice(num_labels, size=k, p=lp)]
            pats.append((k, mask, induced, labels))
        out.append(Query(t, g, pats))
    return out
