"""GPU parity: the HIP path through the C-ABI against the oracle.

Counts are integers, so every comparison is exact equality.
"""
import itertools
import os
import sys

import numpy as np
import pytest

import gen
import oracle
from oracle import P

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def eng():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_04553_amd as pm
    e = pm.Engine(arena_bytes=12 << 30)
    yield e
    e.close()


def _patterns(k, induced):
    return [(k, m, induced) for m in P.connected_classes(k)]


def _gpu_counts(eng, g, k, induced, morph):
    import paper_2012_04553_amd as pm
    gid = eng.load(g)
    try:
        return eng.count(gid, _patterns(k, induced), morph=morph)
    finally:
        eng.graph_unload(gid)


def _oracle_counts(g, k, induced):
    return [oracle.count(g, k, m, induced) for m in P.connected_classes(k)]


@pytest.mark.parametrize("k", [3, 4, 5])
def test_five_vertex_graphs_all_masks(eng, k):
    """Every 5-vertex graph whose edge mask is a multiple of 7 (a spread
    over all 1024), every connected k-pattern, VI and EI, both modes."""
    import paper_2012_04553_amd as pm
    _say(f"five-vertex sweep k={k}")
    for mask in range(0, 1 << 10, 7):
        g = gen.graph_from_mask(5, mask)
        for induced in (False, True):
            want = _oracle_counts(g, k, induced)
            for morph in (pm.MORPH_NONE, pm.MORPH_NAIVE):
                got = _gpu_counts(eng, g, k, induced, morph)
                assert got == want, (mask, k, induced, morph)


@pytest.mark.parametrize("seed,n,p", [(1, 30, 0.3), (2, 40, 0.2), (3, 24, 0.5)])
def test_random_graphs_4_and_5(eng, seed, n, p):
    import paper_2012_04553_amd as pm
    g = gen.erdos_renyi(n, p, seed)
    for k in (4, 5):
        for induced in (False, True):
            _say(f"ER n={n} p={p} seed={seed} k={k} induced={induced}")
            want = _oracle_counts(g, k, induced)
            for morph in (pm.MORPH_NONE, pm.MORPH_NAIVE):
                assert _gpu_counts(eng, g, k, induced, morph) == want, (k, induced, morph)


@pytest.mark.parametrize("scale,seed", [(8, 3), (9, 4)])
def test_small_rmat_hubs(eng, scale, seed):
    """Skewed degrees: hubs exercise the level-1 slicing and long lists."""
    import paper_2012_04553_amd as pm
    g = gen.rmat(scale, 8, seed=seed)
    for k in (3, 4):
        for induced in (False, True):
            _say(f"rmat scale={scale} k={k} induced={induced}")
            want = _oracle_counts(g, k, induced)
            for morph in (pm.MORPH_NONE, pm.MORPH_NAIVE):
                assert _gpu_counts(eng, g, k, induced, morph) == want, (k, induced, morph)
    if scale <= 8:
        vi5 = oracle.census(g, 5)
        ei5 = P.edge_induced_from_vertex_induced(5, vi5)
        assert _gpu_counts(eng, g, 5, False, pm.MORPH_NONE) == [ei5[m] for m in P.connected_classes(5)]
        assert _gpu_counts(eng, g, 5, True, pm.MORPH_NAIVE) == [vi5[m] for m in P.connected_classes(5)]


def test_hub_slicing(eng):
    """A star-heavy graph with item_split forcing many level-1 slices."""
    import paper_2012_04553_amd as pm
    g = gen.rmat(10, 16, seed=9)
    eng.set_option("item_split", 64)
    try:
        for induced in (False, True):
            _say(f"hub slicing induced={induced}")
            want = _oracle_counts(g, 4, induced)
            got = _gpu_counts(eng, g, 4, induced, pm.MORPH_NONE)
            assert got == want
    finally:
        eng.set_option("item_split", 2048)


def test_config_er_2000(eng):
    """Plain 4-motif counting on G(2000, 0.005): direct and morphed."""
    import paper_2012_04553_amd as pm
    g = gen.erdos_renyi(2000, 0.005, 1)
    want = oracle.census(g, 4)
    want = [want[m] for m in P.connected_classes(4)]
    _say("ER(2000, 0.005) 4-MC")
    assert _gpu_counts(eng, g, 4, True, pm.MORPH_NONE) == want
    assert _gpu_counts(eng, g, 4, True, pm.MORPH_NAIVE) == want


def test_dense_k4_bearing_graph(eng):
    import paper_2012_04553_amd as pm
    g = gen.erdos_renyi(60, 0.35, 5)
    for k in (4, 5):
        want = _oracle_counts(g, k, True)
        for morph in (pm.MORPH_NONE, pm.MORPH_NAIVE):
            _say(f"dense n=60 k={k} morph={morph}")
            assert _gpu_counts(eng, g, k, True, morph) == want


def test_special_graphs(eng):
    import paper_2012_04553_amd as pm
    cases = [gen.complete_graph(7), gen.complete_bipartite(4, 6), gen.star_graph(9),
             gen.cycle_graph(11), gen.graph_from_mask(4, 0), gen.graph_from_mask(2, 1)]
    for g in cases:
        for k in (3, 4, 5):
            for induced in (False, True):
                want = _oracle_counts(g, k, induced)
                for morph in (pm.MORPH_NONE, pm.MORPH_NAIVE):
                    assert _gpu_counts(eng, g, k, induced, morph) == want, (g.name, k, induced, morph)


def test_labeled_counts(eng):
    import paper_2012_04553_amd as pm
    g = gen.erdos_renyi(40, 0.2, 7)
    g = g.with_labels(gen.zipf_labels(g.n, 3, 1.2, 8))
    gid = eng.load(g)
    try:
        rng = np.random.default_rng(3)
        for k in (3, 4):
            for m in P.connected_classes(k):
                for induced in (False, True):
                    labs = [int(x) for x in rng.integers(-1, 3, size=k)]
                    want = oracle.count(g, k, m, induced, labs)
                    for morph in (pm.MORPH_NONE, pm.MORPH_NAIVE):
                        got = eng.count(gid, [(k, m, induced, labs)], morph=morph)
                        assert got == [want], (k, m, induced, labs, morph)
    finally:
        eng.graph_unload(gid)


def test_relabel_invariance_and_mode_agreement(eng):
    import paper_2012_04553_amd as pm
    g = gen.rmat(9, 8, seed=11)
    rng = np.random.default_rng(1)
    perm = rng.permutation(g.n)
    e = g.edges()
    h = gen.from_edges(g.n, perm[e[:, 0]], perm[e[:, 1]])
    a = _gpu_counts(eng, g, 4, True, pm.MORPH_NAIVE)
    b = _gpu_counts(eng, h, 4, True, pm.MORPH_NAIVE)
    c = _gpu_counts(eng, g, 4, True, pm.MORPH_NONE)
    assert a == b == c


def test_hub_bitmaps_off_equals_on(eng):
    """Probes of hub lists answer from membership bitmaps (vertices of 64 or
    more neighbours); with the bitmaps switched off every probe is a binary
    search.  All 5-vertex classes, both ways, against the oracle's census."""
    import paper_2012_04553_amd as pm
    g = gen.rmat(8, 16, seed=21)
    vi5 = oracle.census(g, 5)
    ei5 = P.edge_induced_from_vertex_induced(5, vi5)
    want_ei = [ei5[m] for m in P.connected_classes(5)]
    want_vi = [vi5[m] for m in P.connected_classes(5)]
    for hb in (1, 0):
        eng.set_option("hub_bitmaps", hb)
        try:
            _say(f"hub bitmaps {hb}")
            assert _gpu_counts(eng, g, 5, False, pm.MORPH_NONE) == want_ei, hb
            assert _gpu_counts(eng, g, 5, True, pm.MORPH_NAIVE) == want_vi, hb
        finally:
            eng.set_option("hub_bitmaps", 1)
