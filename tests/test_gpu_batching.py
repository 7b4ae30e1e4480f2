"""Batching on the GPU: one multi-pattern launch, hipGraph capture/replay,
autotuned launch parameters.  Every result is compared exactly."""
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
    e.close()


def test_multi_pattern_launch_equals_separate(eng):
    import paper_2012_04553_amd as pm
    g = gen.rmat(10, 8, seed=21)
    gid = eng.load(g)
    try:
        eng.set_option("hipgraph", 0)
        pats = [(5, m, False) for m in P.connected_classes(5)]
        together = eng.count(gid, pats, morph=pm.MORPH_NONE)
        separate = [eng.count(gid, [p], morph=pm.MORPH_NONE)[0] for p in pats]
        assert together == separate
    finally:
        eng.set_option("hipgraph", 1)
        eng.graph_unload(gid)
    # oracle check of the same launch on a graph small enough for it
    h = gen.rmat(7, 8, seed=21)
    hid = eng.load(h)
    try:
        vi = oracle.census(h, 5)
        ei = P.edge_induced_from_vertex_induced(5, vi)
        got = eng.count(hid, [(5, m, False) for m in P.connected_classes(5)], morph=pm.MORPH_NONE)
        assert got == [ei[m] for m in P.connected_classes(5)]
    finally:
        eng.graph_unload(hid)


def test_graph_replay_matches_eager(eng):
    """Replays of a captured query set, with eager work and syncs between
    them, each checked against the eager result."""
    import torch
    import paper_2012_04553_amd as pm
    g = gen.rmat(10, 16, seed=22)
    gid = eng.load(g)
    try:
        pats = [(5, m, True) for m in P.connected_classes(5)]
        eng.set_option("hipgraph", 0)
        ref = eng.count(gid, pats, morph=pm.MORPH_NAIVE)
        other = [(4, m, True) for m in P.connected_classes(4)]
        ref4 = eng.count(gid, other, morph=pm.MORPH_NAIVE)
        eng.set_option("hipgraph", 1)
        for rep in range(5):
            assert eng.count(gid, pats, morph=pm.MORPH_NAIVE) == ref, rep
            eng.set_option("hipgraph", 0)
            assert eng.count(gid, other, morph=pm.MORPH_NAIVE) == ref4
            x = torch.arange(1 << 20, device="cuda").sum()
            torch.cuda.synchronize()
            assert int(x) == (1 << 20) * ((1 << 20) - 1) // 2
            eng.set_option("hipgraph", 1)
    finally:
        eng.set_option("hipgraph", 1)
        eng.graph_unload(gid)


def test_autotune(eng):
    import paper_2012_04553_amd as pm
    g = gen.rmat(11, 16, seed=23)
    gid = eng.load(g)
    try:
        pats = [(4, m, True) for m in P.connected_classes(4)]
        ref = eng.count(gid, pats, morph=pm.MORPH_NAIVE)
        cfg = eng.autotune(gid, pats, morph=pm.MORPH_NAIVE)
        assert cfg["blocks_per_cu"] in (1, 2, 4, 8)
        assert cfg["item_budget"] in (256, 1024, 4096, 16384, 65536)
        assert cfg["item_split"] in (32, 64, 512, 2048, 8192)
        assert cfg["ms"] > 0
        again = eng.autotune(gid, pats, morph=pm.MORPH_NAIVE)
        assert again == cfg            # cached
        for _ in range(3):
            assert eng.count(gid, pats, morph=pm.MORPH_NAIVE) == ref
        want = oracle.vertex_induced_4_from_tier_c(g)
        assert ref == [want[m] for m in P.connected_classes(4)]
    finally:
        eng.graph_unload(gid)
