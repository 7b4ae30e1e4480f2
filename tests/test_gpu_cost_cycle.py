"""GPU parity of two plan forms: cost-based alternative sets with vertex-
and edge-induced patterns mixed (Section 4.1, Table 4's queries), and the
edge-induced 5-cycle counted at its lowest vertex (cycle5_kernel) minus its
companion triangle plan.  Counts are integers: exact equality."""
from math import comb

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
    e.close()


def _c5():
    m = 0
    for i in range(5):
        m |= 1 << P.pair_bit(i, (i + 1) % 5)
    return m


@pytest.mark.parametrize("gname", ["er", "rmat8", "rmat9", "kn", "kab", "c5", "c7", "k5"])
def test_cycle5_edge_induced(eng, gname):
    import paper_2012_04553_amd as pm
    if gname == "er":
        g = gen.erdos_renyi(45, 0.25, 71)
    elif gname == "rmat8":
        g = gen.rmat(8, 16, seed=72)
    elif gname == "rmat9":
        g = gen.rmat(9, 16, seed=3)
    elif gname == "kn":
        g = gen.complete_graph(9)
    elif gname == "kab":
        g = gen.complete_bipartite(5, 7)
    elif gname == "c5":
        g = gen.cycle_graph(5)
    elif gname == "c7":
        g = gen.cycle_graph(7)
    else:
        g = gen.graph_from_mask(5, 0x3ff)
    print(f"5-cycle on {gname}", flush=True)
    gid = eng.load(g)
    try:
        got = eng.count(gid, [(5, _c5(), False)], morph=pm.MORPH_NONE)[0]
        desc = eng.plan_describe(gid, (5, _c5(), False))
    finally:
        eng.graph_unload(gid)
    assert "cycle5" in desc
    if gname == "kn":
        assert got == comb(9, 5) * 12          # 12 Hamiltonian cycles on 5 vertices
    elif gname == "kab":
        assert got == 0                         # bipartite: no odd cycle
    elif gname == "c5":
        assert got == 1
    elif gname == "c7":
        assert got == 0
    assert got == oracle.count(g, 5, _c5(), False)


def test_five_motifs_morphed_with_cycle_kernel(eng):
    """All 21 vertex-induced 5-motifs through morphing (their edge-induced
    superpatterns include the 5-cycle) equal the oracle's census."""
    import paper_2012_04553_amd as pm
    for g in (gen.rmat(8, 16, seed=73), gen.erdos_renyi(60, 0.15, 74)):
        gid = eng.load(g)
        try:
            got = eng.count(gid, [(5, m, True) for m in P.connected_classes(5)], morph=pm.MORPH_NAIVE)
        finally:
            eng.graph_unload(gid)
        want = oracle.census(g, 5)
        assert got == [want[m] for m in P.connected_classes(5)]


def test_table4_queries_all_modes(eng):
    """The queries of Table 4 on a skewed and a uniform graph: NONE, NAIVE
    and COST (whatever mixed set the cost model picks) give the oracle's
    counts."""
    import paper_2012_04553_amd as pm
    n = oracle.named_4()
    p1, p2, p3 = n["tailed_triangle"], n["cycle4"], n["diamond"]
    queries = [[(4, p1, True)], [(4, p2, True)], [(4, p2, False)], [(4, p3, True)],
               [(4, p2, False), (4, p3, False)]]
    for g in (gen.rmat(11, 16, seed=75), gen.erdos_renyi(400, 0.05, 76)):
        gid = eng.load(g)
        try:
            for q in queries:
                want = [oracle.count(g, k, m, vi) for k, m, vi in q]
                for mode in (pm.MORPH_NONE, pm.MORPH_NAIVE, pm.MORPH_COST):
                    assert eng.count(gid, q, morph=mode) == want, (q, mode)
                print(f"  {q}: COST matched {eng.last_stats()['num_alt']} patterns", flush=True)
        finally:
            eng.graph_unload(gid)
