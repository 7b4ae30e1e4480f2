"""Pins for the oracle: every check here compares the oracle against
something other than itself (paper values, closed forms, brute force on
tiny inputs, an independent enumeration route, invariants)."""
import os
from itertools import combinations, permutations
from math import comb, factorial

import numpy as np
import pytest

import gen
import oracle
from oracle import P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            rows.append(line.split())
    return rows


@pytest.fixture(scope="module", autouse=True)
def _built(oracle_lib):
    return oracle_lib


def test_pattern_universe_pins():
    names = oracle.named_4()
    for row in _read_golden("pattern_pins.txt"):
        if row[0] == "connected_classes":
            assert len(P.connected_classes(int(row[1]))) == int(row[2])
        elif row[0] == "connected_labelled":
            assert P.labeled_connected_count(int(row[1])) == int(row[2])
        elif row[0] == "aut":
            assert P.num_automorphisms(4, names[row[1]]) == int(row[2])


def test_paper_coefficients():
    names = oracle.named_4()
    for p, q, c in _read_golden("paper_coefficients.txt"):
        assert P.coefficient(4, names[p], names[q]) == int(c), (p, q)


def test_pr_e2_equation():
    # PR-E2 (Section 3.1): C4^E = C4^V + D^V + 3 K4 -- the forward morph row
    names = oracle.named_4()
    cls, mat = P.morph_matrix(4)
    row = dict(zip(cls, mat[cls.index(names["cycle4"])]))
    expect = {m: 0 for m in cls}
    expect[names["cycle4"]] = 1
    expect[names["diamond"]] = 1
    expect[names["clique4"]] = 3
    assert row == expect


def _copies_by_edge_subsets(k, p_mask, q_mask):
    """Distinct copies of p inside q, counted by enumerating edge subsets of
    q and testing isomorphism on the k fixed vertices -- a route that never
    forms phi or Aut."""
    q_edges = P.edges_of(k, q_mask)
    target = P.canonical(k, p_mask)[0]
    ne = P.edge_count(p_mask)
    cnt = 0
    for sub in combinations(q_edges, ne):
        m = 0
        for i, j in sub:
            m |= 1 << P.pair_bit(i, j)
        if P.canonical(k, m)[0] == target:
            cnt += 1
    return cnt


@pytest.mark.parametrize("k", [3, 4, 5])
def test_coefficients_independent_routes(k):
    cls = P.connected_classes(k)
    for p in cls:
        for q in cls:
            c = P.coefficient(k, p, q)
            assert c == _copies_by_edge_subsets(k, p, q)
        # clique superpattern: every permutation is an injection
        assert P.coefficient(k, p, P.clique_mask(k)) == factorial(k) // P.num_automorphisms(k, p)
        assert P.coefficient(k, p, p) == 1


@pytest.mark.parametrize("k", [4, 5])
def test_coefficients_are_edge_induced_counts_in_q(k):
    # c(p, q) equals the number of edge-induced p-subgraphs of the data graph q
    cls = P.connected_classes(k)
    for q in cls:
        g = gen.graph_from_mask(k, q)
        for p in cls:
            assert oracle.count(g, k, p, induced=False) == P.coefficient(k, p, q)


def test_triangles_and_stars_closed_forms():
    for seed in range(3):
        g = gen.erdos_renyi(30, 0.3, seed)
        A = np.zeros((g.n, g.n), dtype=np.int64)
        for u, v in g.edges():
            A[u, v] = A[v, u] = 1
        tri = int(np.trace(A @ A @ A)) // 6
        assert oracle.count(g, 3, P.clique_mask(3), induced=True) == tri
        d = g.degrees()
        star = [m for m in P.connected_classes(4) if P.num_automorphisms(4, m) == 6][0]
        assert oracle.count(g, 4, star, induced=False) == sum(comb(int(x), 3) for x in d)
        wedge = [m for m in P.connected_classes(3) if P.edge_count(m) == 2][0]
        assert oracle.count(g, 3, wedge, induced=False) == sum(comb(int(x), 2) for x in d)
        # tr(A^4) = 8 C4 + 2m + 4 sum C(d,2)
        c4 = oracle.named_4()["cycle4"]
        tr4 = int(np.trace(A @ A @ A @ A))
        m = g.m
        assert tr4 == 8 * oracle.count(g, 4, c4, False) + 2 * m + 4 * sum(comb(int(x), 2) for x in d)


@pytest.mark.parametrize("k", [3, 4, 5])
def test_complete_graph(k):
    N = 7
    g = gen.complete_graph(N)
    for p in P.connected_classes(k):
        assert oracle.count(g, k, p, False) == comb(N, k) * factorial(k) // P.num_automorphisms(k, p)
        expect_v = comb(N, k) if p == P.clique_mask(k) else 0
        assert oracle.count(g, k, p, True) == expect_v


def test_complete_bipartite_and_cycles():
    g = gen.complete_bipartite(4, 5)
    names = oracle.named_4()
    assert oracle.count(g, 3, P.clique_mask(3), True) == 0
    assert oracle.count(g, 4, names["cycle4"], True) == comb(4, 2) * comb(5, 2)
    c = gen.cycle_graph(9)
    assert oracle.count(c, 4, names["path4"], True) == 9
    assert oracle.count(c, 4, names["path4"], False) == 9
    assert oracle.count(c, 4, names["star3"], False) == 0
    s = gen.star_graph(6)
    assert oracle.count(s, 4, names["star3"], True) == comb(6, 3)


def test_exhaustive_five_vertex_graphs_census_and_morph():
    """Every graph on 5 vertices: tier A vertex-induced == census; all
    k-subsets sum to C(n, k); Theorem 3.1 forward holds; Corollary 3.1
    back-substitution recovers the vertex-induced counts."""
    for k in (3, 4):
        cls = P.connected_classes(k)
        for mask in range(1 << 10):
            g = gen.graph_from_mask(5, mask)
            vi = {p: oracle.count(g, k, p, True) for p in cls}
            ei = {p: oracle.count(g, k, p, False) for p in cls}
            assert vi == oracle.census(g, k)
            assert P.edge_induced_from_vertex_induced(k, vi) == ei
            assert P.vertex_induced_from_edge_induced(k, ei) == vi
            full = oracle.full_census_tiny(g, k)
            assert sum(full.values()) == comb(5, k)
            for p in cls:
                assert full[p] == vi[p]


def test_five_vertex_morph_on_graphs_with_six_vertices():
    rng = np.random.default_rng(5)
    cls = P.connected_classes(5)
    for _ in range(40):
        mask = int(rng.integers(0, 1 << 15))
        g = gen.graph_from_mask(6, mask)
        vi = {p: oracle.count(g, 5, p, True) for p in cls}
        ei = {p: oracle.count(g, 5, p, False) for p in cls}
        assert vi == oracle.census(g, 5)
        assert P.edge_induced_from_vertex_induced(5, vi) == ei
        assert P.vertex_induced_from_edge_induced(5, ei) == vi
        full = oracle.full_census_tiny(g, 5)
        assert sum(full.values()) == comb(6, 5)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_random_graphs_tiers_agree(seed):
    g = gen.erdos_renyi(60, 0.15, seed)
    for k in (4, 5):
        vi = oracle.motif_counts(g, k, True)
        assert vi == oracle.census(g, k)
        ei = oracle.motif_counts(g, k, False)
        assert P.edge_induced_from_vertex_induced(k, vi) == ei
    assert oracle.edge_induced_4_from_tier_c(g) == oracle.motif_counts(g, 4, False)


def test_tier_c_on_skewed_graph():
    g = gen.rmat(9, 8, seed=7)
    assert oracle.edge_induced_4_from_tier_c(g) == oracle.motif_counts(g, 4, False)


def test_relabel_invariance():
    g = gen.erdos_renyi(50, 0.2, 9)
    rng = np.random.default_rng(0)
    perm = rng.permutation(g.n)
    e = g.edges()
    h = gen.from_edges(g.n, perm[e[:, 0]], perm[e[:, 1]])
    assert oracle.motif_counts(g, 4, True) == oracle.motif_counts(h, 4, True)


def test_labeled_counts_sum_to_unlabeled():
    g = gen.erdos_renyi(40, 0.2, 3)
    L = 3
    g = g.with_labels(gen.zipf_labels(g.n, L, 1.2, 4))
    for k in (3, 4):
        for p in P.connected_classes(k):
            unl = oracle.count_maps(g, k, p, False)
            tot = 0
            for labs in np.ndindex(*([L] * k)):
                tot += oracle.count_maps(g, k, p, False, plabels=list(labs))
            assert tot == unl


def test_mni_pins():
    # one-edge pattern (a, b): support = min(#distinct a-endpoints,
    # #distinct b-endpoints) over edges whose endpoints carry (a, b)
    g = gen.erdos_renyi(40, 0.1, 2).with_labels(gen.zipf_labels(40, 3, 1.2, 5))
    lab = g.labels
    for a in range(3):
        for b in range(3):
            ends_a, ends_b = set(), set()
            for u, v in g.edges():
                for x, y in ((u, v), (v, u)):
                    if lab[x] == a and lab[y] == b:
                        ends_a.add(x)
                        ends_b.add(y)
            expect = min(len(ends_a), len(ends_b))
            assert oracle.mni_support(g, 2, 1, False, [a, b]) == expect
    # K_N with one label: every vertex is in every domain
    kn = gen.complete_graph(6).with_labels(np.zeros(6, dtype=np.uint8))
    for p in P.connected_classes(4):
        assert oracle.mni_support(kn, 4, p, False, [0] * 4) == 6
    # a star with N >= 3 leaves and the 3-star pattern: the centre column has 1
    s = gen.star_graph(5).with_labels(np.zeros(6, dtype=np.uint8))
    star = oracle.named_4()["star3"]
    assert oracle.mni_support(s, 4, star, False, [0] * 4) == 1


def test_mni_anti_monotone():
    g = gen.erdos_renyi(35, 0.15, 8).with_labels(np.zeros(35, dtype=np.uint8))
    names = oracle.named_4()
    # path4 is a subpattern of cycle4 and tailed_triangle (same vertex count)
    sp = oracle.mni_support(g, 4, names["path4"], False, [0] * 4)
    for sup in ("cycle4", "tailed_triangle", "diamond"):
        assert sp >= oracle.mni_support(g, 4, names[sup], False, [0] * 4)


def test_planted_mistake_is_caught():
    """A dropped term in the back-substitution must break the identity."""
    g = gen.erdos_renyi(30, 0.3, 11)
    ei = oracle.motif_counts(g, 4, False)
    vi = oracle.motif_counts(g, 4, True)
    names = oracle.named_4()
    good = P.vertex_induced_from_edge_induced(4, ei)
    assert good == vi
    bad = dict(good)
    bad[names["cycle4"]] = ei[names["cycle4"]] - good[names["diamond"]]  # drop 3*K4
    if vi[names["clique4"]]:
        assert bad != vi


def test_mni_rooted_search_equals_full_enumeration():
    """The rooted-existence column sizes equal the domains of the full
    match enumeration (two independent routes to the same definition)."""
    g = gen.erdos_renyi(30, 0.15, 12).with_labels(gen.zipf_labels(30, 3, 1.2, 13))
    rng = np.random.default_rng(2)
    for k in (3, 4):
        for m in P.connected_classes(k):
            labs = [int(x) for x in rng.integers(0, 3, size=k)]
            dom = oracle.mni_domains(g, k, m, False, labs)
            for v in range(k):
                assert oracle.mni_column(g, k, m, False, labs, v) == int(dom[v].sum())
            assert oracle.mni_support_rooted(g, k, m, False, labs) == oracle.mni_support(g, k, m, False, labs)


@pytest.mark.parametrize("k,L", [(3, 2), (3, 3), (4, 2), (4, 3), (5, 2)])
def test_labeled_automorphisms_orbit_count(k, L):
    """Label-preserving automorphisms, pinned by orbit counting.  The
    vertex-numbered connected graphs on k vertices with each vertex given
    one of L labels number L^k times the connected labelled-graph count
    (4, 38, 728; tests/golden/pattern_pins.txt).  Relabelling the vertices
    splits them into one orbit per labeled pattern, of size k!/|Aut_L(p)|,
    so the orbit sizes over the distinct canonical labeled patterns must sum
    to that number.  A label test missing from the automorphisms (or from
    the canonical form) breaks the sum."""
    from itertools import product
    labelled = {int(r[1]): int(r[2]) for r in _read_golden("pattern_pins.txt")
                if r[0] == "connected_labelled"}
    forms = set()
    for m in P.connected_classes(k):
        for labs in product(range(L), repeat=k):
            forms.add(P.canonical(k, m, labs))
    total = 0
    for m, labs in forms:
        aut = P.num_automorphisms(k, m, labs)
        assert factorial(k) % aut == 0
        total += factorial(k) // aut
    assert total == L ** k * labelled[k]
    # a planted mistake: automorphisms that ignore labels undercount
    wrong = sum(factorial(k) // P.num_automorphisms(k, m) for m, labs in forms)
    assert wrong != total


def test_mni_labelings_equals_per_pattern_support():
    """One enumeration of the unlabeled shape, filed by the labels of the
    images, against the per-pattern support (pinned above) for every
    labeling of every 3- and 4-vertex shape."""
    from itertools import product
    g = gen.erdos_renyi(28, 0.2, 21).with_labels(gen.zipf_labels(28, 3, 1.2, 22))
    for k in (3, 4):
        for m in P.connected_classes(k):
            labs = [list(t) for t in product(range(3), repeat=k)]
            got = oracle.mni_labelings(g, k, m, False, 3, labs)
            for t, sup in zip(labs, got):
                assert sup == oracle.mni_support(g, k, m, False, t), (k, m, t)


def test_tier_c_root_sample_adds_up():
    """The root-sampled closed forms (used to time the oracle on a bounded
    sample) add up over every residue class to the full closed forms."""
    g = gen.rmat(9, 16, seed=23)
    full = oracle.tier_c4(g)
    for stride in (1, 3, 7):
        raw = {k: 0 for k in oracle.TIER_C4_KEYS}
        for off in range(stride):
            part = oracle.tier_c4_sample(g, stride, off)
            for k in raw:
                raw[k] += part[k]
        assert oracle.tier_c4_from_raw(raw) == full, stride


def test_list_maps_pins():
    """Listing oracle: as many rows as matches counted, every row a match
    (brute-force check of edges, anti-edges and labels), and the rows
    collapse to count() distinct subgraphs; on K_6 the triangles are the
    C(6, 3) vertex triples."""
    g = gen.erdos_renyi(14, 0.35, 27).with_labels(gen.zipf_labels(14, 2, 1.0, 28))
    adj = {(u, int(v)) for u in range(g.n) for v in g.neighbors(u)}
    for k in (3, 4):
        for m in P.connected_classes(k):
            for induced in (False, True):
                for labs in (None, [0] + [1] * (k - 1)):
                    rows = oracle.list_maps(g, k, m, induced, labs)
                    assert len(rows) == oracle.count_maps(g, k, m, induced, labs)
                    keys = set()
                    for r in rows:
                        r = [int(x) for x in r]
                        assert len(set(r)) == k
                        for j in range(k):
                            for i in range(j):
                                e = (r[i], r[j]) in adj
                                assert e or not P.has_edge(m, i, j)
                                assert not (induced and e and not P.has_edge(m, i, j))
                        if labs is not None:
                            assert all(int(g.labels[r[v]]) == labs[v] for v in range(k))
                        keys.add((frozenset(r), frozenset(tuple(sorted((r[i], r[j]))) for i, j in P.edges_of(k, m))))
                    assert len(keys) == oracle.count(g, k, m, induced, labs)
    k6 = gen.complete_graph(6)
    rows = oracle.list_maps(k6, 3, 0b111, False)
    assert len({frozenset(int(x) for x in r) for r in rows}) == comb(6, 3)
