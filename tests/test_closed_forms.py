"""The counting identities behind the engine's closed forms over triangle
counts, checked on the CPU against the oracle's census (no product code):
each edge-induced count below equals its closed form over per-edge triangle
counts t(e), per-vertex triangle counts T(v), degrees, 4-cycles and
4-cliques, written out here by brute force on small graphs.  The GPU tests
check the kernels that evaluate the same forms against the same census."""
from itertools import combinations

import numpy as np
import pytest

import gen
import oracle
from oracle import P


def _union(a, b):
    ea, eb = a.edges(), b.edges()
    u = np.concatenate([ea[:, 0], eb[:, 0] + a.n])
    v = np.concatenate([ea[:, 1], eb[:, 1] + a.n])
    return gen.from_edges(a.n + b.n, u, v)


GRAPHS = {
    "er": lambda: gen.erdos_renyi(70, 0.15, seed=71),
    "k9_rmat5": lambda: _union(gen.complete_graph(9), gen.rmat(5, 8, seed=72)),
    "rmat6": lambda: gen.rmat(6, 8, seed=73),
}


@pytest.fixture(scope="module", params=sorted(GRAPHS))
def case(request):
    g = GRAPHS[request.param]()
    ei5 = P.edge_induced_from_vertex_induced(5, oracle.census(g, 5))
    ei4 = P.edge_induced_from_vertex_induced(4, oracle.census(g, 4))
    adj = [set() for _ in range(g.n)]
    for a, b in g.edges():
        adj[a].add(b)
        adj[b].add(a)
    return g, adj, ei4, ei5


def _t(adj, a, b):
    return len(adj[a] & adj[b])


def _edges(adj):
    return [(a, b) for a in range(len(adj)) for b in adj[a] if a < b]


def test_triangle_and_tailed_triangle(case):
    g, adj, ei4, ei5 = case
    E = _edges(adj)
    tri = sum(_t(adj, a, b) for a, b in E)
    assert tri % 3 == 0
    assert tri // 3 == P.edge_induced_from_vertex_induced(3, oracle.census(g, 3))[0x7]
    d = [len(x) for x in adj]
    tailed = sum(_t(adj, a, b) * (d[a] + d[b] - 4) for a, b in E)
    assert tailed % 2 == 0 and tailed // 2 == ei4[0xF]


def test_bowtie_and_triangle_with_path(case):
    g, adj, ei4, ei5 = case
    E = _edges(adj)
    d = [len(x) for x in adj]
    T = [0] * len(adj)
    for a, b in E:
        t = _t(adj, a, b)
        T[a] += t
        T[b] += t
    T = [x // 2 for x in T]
    bowtie = sum(x * (x - 1) // 2 for x in T) - sum(_t(adj, a, b) * (_t(adj, a, b) - 1) for a, b in E)
    assert bowtie == ei5[0xEB]
    path = sum((T[a] - _t(adj, a, b)) * (d[b] - 1) + (T[b] - _t(adj, a, b)) * (d[a] - 1)
               - 2 * _t(adj, a, b) * (_t(adj, a, b) - 1) for a, b in E)
    assert path == ei5[0x75]


def test_house_from_four_cycle_support_sums(case):
    g, adj, ei4, ei5 = case
    E = _edges(adj)
    # every 4-cycle at its highest vertex x, through the pair (x, y), y opposite
    w4 = 0
    for x in range(len(adj)):
        below = {}
        for a in adj[x]:
            if a < x:
                for y in adj[a]:
                    if y < x:
                        below.setdefault(y, []).append(a)
        for y, bridges in below.items():
            c = len(bridges)
            w4 += (c - 1) * sum(_t(adj, x, a) + _t(adj, a, y) for a in bridges)
    house = w4 - 2 * sum(_t(adj, a, b) * (_t(adj, a, b) - 1) for a, b in E)
    assert house == ei5[0xED]


def test_per_triangle_forms(case):
    g, adj, ei4, ei5 = case
    d = [len(x) for x in adj]
    dtail = fan = 0
    for a in range(len(adj)):
        for b in adj[a]:
            if b <= a:
                continue
            for c in adj[a] & adj[b]:
                if c <= b:
                    continue
                tab, tac, tbc = _t(adj, a, b), _t(adj, a, c), _t(adj, b, c)
                dtail += (d[a] - 2) * (tbc - 1) + (d[b] - 2) * (tac - 1) + (d[c] - 2) * (tab - 1)
                fan += (tab - 1) * (tac - 1) + (tab - 1) * (tbc - 1) + (tac - 1) * (tbc - 1)
    assert dtail - 12 * ei4[0x3F] == ei5[0x77]
    assert fan - 12 * ei4[0x3F] == ei5[0xEF]


def test_four_clique_with_an_ear(case):
    g, adj, ei4, ei5 = case
    # per root r, the graph induced on its higher neighbours: each edge (i, j)
    # of it on lt triangles adds lt (2 (t(i, j) - 2) + (t(r, i) - 2) + (t(r, j) - 2))
    s = 0
    for r in range(len(adj)):
        up = {x for x in adj[r] if x > r}
        for i, j in combinations(sorted(up), 2):
            if j not in adj[i]:
                continue
            lt = len(adj[i] & adj[j] & up)
            s += lt * (2 * (_t(adj, i, j) - 2) + (_t(adj, r, i) - 2) + (_t(adj, r, j) - 2))
    assert s % 2 == 0 and s // 2 == ei5[0xFF]
    # and directly: the sum over 4-cliques of t(e) - 2 over their six edges
    direct = 0
    for q in combinations(range(len(adj)), 4):
        if all(b in adj[a] for a, b in combinations(q, 2)):
            direct += sum(_t(adj, a, b) - 2 for a, b in combinations(q, 2))
    assert direct == ei5[0xFF]
