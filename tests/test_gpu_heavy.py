"""GPU parity of the heavy-root kernels (LDS window sweeps for two-hop and
edge-core plans).  With the mass threshold at 1 every eligible root takes
the window path, on graphs the oracle counts quickly; the same counts must
come out with the path switched off."""
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
    e = pm.Engine(arena_bytes=4 << 30)
    yield e
    e.close()


def _counts(eng, g, k, induced, morph, heavy):
    eng.set_option("heavy_roots", 1 if heavy else 0)
    eng.set_option("heavy_min_mass", 1)
    gid = eng.load(g)
    try:
        return eng.count(gid, [(k, m, induced) for m in P.connected_classes(k)], morph=morph)
    finally:
        eng.graph_unload(gid)
        eng.set_option("heavy_roots", 1)
        eng.set_option("heavy_min_mass", 16384)


@pytest.mark.parametrize("scale,seed", [(9, 1), (10, 4)])
def test_heavy_roots_four_vertex(eng, scale, seed):
    import paper_2012_04553_amd as pm
    g = gen.rmat(scale, 16, seed=seed)
    print(f"R-MAT {scale} seed {seed}", flush=True)
    want_e = oracle.edge_induced_4_from_tier_c(g)
    want_e = [want_e[m] for m in P.connected_classes(4)]
    assert _counts(eng, g, 4, False, pm.MORPH_NONE, True) == want_e
    want_v = oracle.vertex_induced_4_from_tier_c(g)
    want_v = [want_v[m] for m in P.connected_classes(4)]
    assert _counts(eng, g, 4, True, pm.MORPH_NAIVE, True) == want_v
    assert _counts(eng, g, 4, True, pm.MORPH_NAIVE, False) == want_v


def test_heavy_roots_labeled(eng):
    import paper_2012_04553_amd as pm
    g = gen.erdos_renyi(120, 0.12, 7).with_labels(gen.zipf_labels(120, 3, 1.2, 8))
    names = oracle.named_4()
    eng.set_option("heavy_min_mass", 1)
    gid = eng.load(g)
    try:
        for mask in (names["cycle4"], names["diamond"]):
            for labs in ([0, 0, 0, 0], [0, 1, 0, 1], [1, 0, 2, 0]):
                want = oracle.count(g, 4, mask, False, plabels=labs)
                pats = [(4, mask, False, labs)]
                assert eng.count(gid, pats, morph=pm.MORPH_NONE) == [want], (mask, labs)
    finally:
        eng.graph_unload(gid)
        eng.set_option("heavy_min_mass", 16384)


def test_heavy_roots_five_vertex(eng):
    import paper_2012_04553_amd as pm
    g = gen.rmat(7, 8, seed=5)
    want = oracle.census(g, 5)
    want = [want[m] for m in P.connected_classes(5)]
    assert _counts(eng, g, 5, True, pm.MORPH_NAIVE, True) == want


def test_heavy_roots_wide_counters(eng):
    """The 32-bit-counter variant of the two-hop window kernel (taken on
    graphs with a degree above 16 bits) forced on small graphs: counts from
    the oracle's closed forms, and equal to the 16-bit variant."""
    import paper_2012_04553_amd as pm
    g = gen.rmat(10, 16, seed=6)
    want_e = oracle.edge_induced_4_from_tier_c(g)
    want_e = [want_e[m] for m in P.connected_classes(4)]
    want_v = oracle.vertex_induced_4_from_tier_c(g)
    want_v = [want_v[m] for m in P.connected_classes(4)]
    eng.set_option("window_counters", 32)
    try:
        assert _counts(eng, g, 4, False, pm.MORPH_NONE, True) == want_e
        assert _counts(eng, g, 4, True, pm.MORPH_NAIVE, True) == want_v
    finally:
        eng.set_option("window_counters", 16)
    assert _counts(eng, g, 4, True, pm.MORPH_NAIVE, True) == want_v
