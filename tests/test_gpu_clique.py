"""GPU parity of the triangle-core, edge-support and 4-clique kernels: K3,
the tailed triangle, the 4-path (which needs K3), the diamond (from edge
supports), K4 and the 4-vertex sets that include them, against the
oracle's closed-form counts.  The R-MAT graphs
cut their hub roots into row slices and give the 4-clique kernel roots of
both its wavefront and workgroup sizes; the clique K_1040 gives roots with
more out-neighbours than either kernel takes, which run in the general
kernel.  Every count must also come out the same with the kernels switched
off."""
import numpy as np
import pytest

import gen
import oracle
from oracle import P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_04553_amd as pm
    e = pm.Engine(arena_bytes=8 << 30)
    yield e
    e.set_option("clique_kernel", 1)
    e.close()


def _union(a, b):
    ea, eb = a.edges(), b.edges()
    u = np.concatenate([ea[:, 0], eb[:, 0] + a.n])
    v = np.concatenate([ea[:, 1], eb[:, 1] + a.n])
    return gen.from_edges(a.n + b.n, u, v)


def _count(eng, gid, pats, morph, on):
    eng.set_option("clique_kernel", 1 if on else 0)
    return eng.count(gid, pats, morph=morph)


@pytest.mark.parametrize("scale,seed", [(12, 3), (16, 5)])
def test_clique_kernel_rmat(eng, scale, seed):
    import paper_2012_04553_amd as pm
    g = gen.rmat(scale, 16, seed=seed)
    print(f"R-MAT {scale} seed {seed}", flush=True)
    tc = oracle.tier_c4(g)
    classes = list(P.connected_classes(4))
    want_e = oracle.edge_induced_4_from_tier_c(g)
    want_v = P.vertex_induced_from_edge_induced(4, want_e)
    gid = eng.load(g)
    try:
        names = oracle.named_4()
        assert "triangle counts: tailed triangle" in eng.plan_describe(gid, (4, names["tailed_triangle"], False))
        assert "triangle counts: triangle" in eng.plan_describe(gid, (3, 0x7, False))
        assert "edge_support" in eng.plan_describe(gid, (4, names["diamond"], False))
        for on in (True, False):
            assert _count(eng, gid, [(3, 0x7, False)], pm.MORPH_NONE, on) == [tc["triangles"]]
            assert _count(eng, gid, [(4, m, False) for m in classes], pm.MORPH_NONE, on) == \
                [want_e[m] for m in classes]
            assert _count(eng, gid, [(4, m, True) for m in classes], pm.MORPH_NAIVE, on) == \
                [want_v[m] for m in classes]
        # without edge supports the triangle and the tailed triangle run as
        # triangle-core plans, the tail evaluated per triangle
        eng.set_option("edge_support", 0)
        try:
            assert "triangle_core" in eng.plan_describe(gid, (4, names["tailed_triangle"], False))
            assert "triangle_core" in eng.plan_describe(gid, (3, 0x7, False))
            assert _count(eng, gid, [(3, 0x7, False)], pm.MORPH_NONE, True) == [tc["triangles"]]
            assert _count(eng, gid, [(4, m, False) for m in classes], pm.MORPH_NONE, True) == \
                [want_e[m] for m in classes]
            assert _count(eng, gid, [(4, m, True) for m in classes], pm.MORPH_NAIVE, True) == \
                [want_v[m] for m in classes]
        finally:
            eng.set_option("edge_support", 1)
    finally:
        eng.graph_unload(gid)


def test_clique_kernel_dense_roots(eng):
    import paper_2012_04553_amd as pm
    g = _union(gen.complete_graph(1040), gen.rmat(10, 16, seed=6))
    tc = oracle.tier_c4(g)
    names = oracle.named_4()
    pats = [(3, 0x7, False), (4, names["tailed_triangle"], False), (4, names["path4"], False),
            (4, names["clique4"], False)]
    want = [tc["triangles"], tc["tailed_triangle"], tc["path4"], tc["clique4"]]
    # K_1040 alone holds C(1040, 3) triangles
    assert tc["triangles"] >= 1040 * 1039 * 1038 // 6
    gid = eng.load(g)
    try:
        assert eng.graph_stats(gid)["max_out_degree"] > 1024
        for on in (True, False):
            assert _count(eng, gid, pats, pm.MORPH_NONE, on) == want
    finally:
        eng.graph_unload(gid)


def test_clique_kernels_five_vertex(eng):
    """Five-vertex edge-induced patterns whose plans have triangle, 4-clique
    or edge-support cores, with tail monomials that do not hold the set-size
    term (an edge on no triangle still adds them)."""
    import paper_2012_04553_amd as pm
    g = gen.rmat(7, 8, seed=21)
    vi = oracle.census(g, 5)
    ei = P.edge_induced_from_vertex_induced(5, vi)
    classes = list(P.connected_classes(5))
    gid = eng.load(g)
    try:
        for on in (True, False):
            assert _count(eng, gid, [(5, m, False) for m in classes], pm.MORPH_NONE, on) == \
                [ei[m] for m in classes]
    finally:
        eng.graph_unload(gid)


def test_edge_supports_beyond_packed_ids(eng):
    """Above 2^22 - 2 vertices the support pass keeps its per-slot counters
    apart from the hash keys; an R-MAT graph padded with isolated vertices
    takes that path."""
    import paper_2012_04553_amd as pm
    h = gen.rmat(12, 16, seed=8)
    e = h.edges()
    n = (1 << 22) + 64
    g = gen.from_edges(n, e[:, 0] + 64, e[:, 1] + 64)
    tc = oracle.tier_c4(h)
    names = oracle.named_4()
    pats = [(4, names["diamond"], False), (4, names["tailed_triangle"], False), (3, 0x7, False)]
    want = [tc["diamond"], tc["tailed_triangle"], tc["triangles"]]
    gid = eng.load(g)
    try:
        assert "edge_support" in eng.plan_describe(gid, pats[0])
        for on in (True, False):
            assert _count(eng, gid, pats, pm.MORPH_NONE, on) == want
    finally:
        eng.graph_unload(gid)


_BOWTIE, _TRIPATH, _HOUSE, _DTAIL, _FAN, _K4EAR = 0x0EB, 0x075, 0x0ED, 0x077, 0x0EF, 0x0FF


@pytest.mark.parametrize("gname", ["rmat8", "er", "k12_rmat6"])
def test_triangle_count_closed_forms(eng, gname):
    """The bowtie (two triangles sharing a vertex), the triangle with a
    two-edge path hanging off a corner, the house (a 4-cycle with a triangle
    on one edge), the diamond with a pendant at a tip and the fan of three
    triangles and the 4-clique with an ear are counted in closed form from
    the per-edge and per-vertex triangle counts, the 4-cycles' sums of them,
    per-triangle sums of them (less twelve per 4-clique) and per-4-clique
    sums of them; against the oracle census, in a
    single-pattern set, in the 21-pattern edge-induced set (several
    edge-support launches in one replay) and in the morphed vertex-induced
    5-motif set, and the same with the triangle kernels off (enumerating
    plans instead)."""
    import paper_2012_04553_amd as pm
    g = {"rmat8": lambda: gen.rmat(8, 8, seed=31),
         "er": lambda: gen.erdos_renyi(120, 0.1, seed=32),
         "k12_rmat6": lambda: _union(gen.complete_graph(12), gen.rmat(6, 8, seed=33))}[gname]()
    vi = oracle.census(g, 5)
    ei = P.edge_induced_from_vertex_induced(5, vi)
    classes = list(P.connected_classes(5))
    gid = eng.load(g)
    try:
        eng.set_option("clique_kernel", 1)
        assert "triangle counts: bowtie" in eng.plan_describe(gid, (5, _BOWTIE, False))
        assert "triangle counts: triangle with a two-edge path" in eng.plan_describe(gid, (5, _TRIPATH, False))
        assert "triangle counts: house" in eng.plan_describe(gid, (5, _HOUSE, False))
        assert "triangle counts: diamond with a pendant" in eng.plan_describe(gid, (5, _DTAIL, False))
        assert "triangle counts: fan of three triangles" in eng.plan_describe(gid, (5, _FAN, False))
        assert "triangle counts: 4-clique with an ear" in eng.plan_describe(gid, (5, _K4EAR, False))
        for on in (True, False):
            for m in (_BOWTIE, _TRIPATH, _HOUSE, _DTAIL, _FAN, _K4EAR):
                assert _count(eng, gid, [(5, m, False)], pm.MORPH_NONE, on) == [ei[m]]
            assert _count(eng, gid, [(5, m, False) for m in classes], pm.MORPH_NONE, on) == \
                [ei[m] for m in classes]
            assert _count(eng, gid, [(5, m, True) for m in classes], pm.MORPH_NAIVE, on) == \
                [vi[m] for m in classes]
        eng.set_option("clique_kernel", 1)
        # a second replay of the same cached launch set starts from cleared
        # supports and per-vertex counts
        three = [(5, _BOWTIE, False), (5, _TRIPATH, False), (5, _HOUSE, False)]
        want = [ei[_BOWTIE], ei[_TRIPATH], ei[_HOUSE]]
        assert eng.count(gid, three, morph=pm.MORPH_NONE) == want
        # forked launch sets are not forked with the house's dense counters
        eng.set_option("fork_launches", 1)
        try:
            assert eng.count(gid, three + [(4, 0x3F, False)], morph=pm.MORPH_NONE)[:3] == want
        finally:
            eng.set_option("fork_launches", 0)
    finally:
        eng.graph_unload(gid)


def test_triangle_count_closed_forms_match_enumeration(eng):
    """On R-MAT 13 (hub roots, large triangle counts per vertex) the closed
    forms equal the enumerating plans; beside a clique with more
    out-neighbours than the triangle kernel takes (not every triangle would
    be counted per edge), no closed form is chosen."""
    import paper_2012_04553_amd as pm
    pats = [(5, m, False) for m in (_BOWTIE, _TRIPATH, _HOUSE, _DTAIL, _FAN, _K4EAR)]
    g = gen.rmat(13, 16, seed=34)
    gid = eng.load(g)
    try:
        a = _count(eng, gid, pats, pm.MORPH_NONE, True)
        b = _count(eng, gid, pats, pm.MORPH_NONE, False)
        print(f"R-MAT 13: {a}", flush=True)
        assert a == b and min(a) > 0
    finally:
        eng.set_option("clique_kernel", 1)
        eng.graph_unload(gid)
    g = _union(gen.complete_graph(1040), gen.rmat(8, 8, seed=35))
    gid = eng.load(g)
    try:
        assert eng.graph_stats(gid)["max_out_degree"] > 1024
        for p in pats:
            assert "triangle counts" not in eng.plan_describe(gid, p)
    finally:
        eng.set_option("clique_kernel", 1)
        eng.graph_unload(gid)
