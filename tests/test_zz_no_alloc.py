"""pm_count_noalloc, the allocation-free entry point, against pm_submit +
pm_wait (the entry point it varies) on the same seeded inputs, through the
C-ABI: two calls in a row, the second with a smaller input, then a labeled
and a 5-vertex query.  Counts are integers: exact equality."""
import pytest

import gen
from oracle import P

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eng():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_04553_amd as pm
    e = pm.Engine(arena_bytes=2 << 30)
    yield e
    e.close()


def _both(eng, g, pats, morph):
    gid = eng.load(g)
    try:
        want = eng.count(gid, pats, morph=morph)
        got = eng.count_noalloc(gid, pats, morph=morph)
    finally:
        eng.graph_unload(gid)
    return got, want


def test_noalloc_two_calls_second_smaller(eng):
    import paper_2012_04553_amd as pm
    big = gen.rmat(12, 16, seed=7)
    small = gen.erdos_renyi(200, 0.05, 8)
    print("R-MAT 12, 4-motifs morphed", flush=True)
    got, want = _both(eng, big, [(4, m, True) for m in P.connected_classes(4)], pm.MORPH_NAIVE)
    assert got == want
    print("ER(200, 0.05), 3-vertex edge-induced", flush=True)
    got, want = _both(eng, small, [(3, m, False) for m in P.connected_classes(3)], pm.MORPH_NONE)
    assert got == want


def test_noalloc_labeled_and_five_vertex(eng):
    import paper_2012_04553_amd as pm
    g = gen.erdos_renyi(60, 0.15, 9).with_labels(gen.zipf_labels(60, 3, 1.2, 10))
    pats = [(4, m, True, [0, 1, 0, 2]) for m in P.connected_classes(4)]
    got, want = _both(eng, g, pats, pm.MORPH_NAIVE)
    assert got == want
    g5 = gen.rmat(7, 8, seed=11)
    pats = [(5, m, True) for m in P.connected_classes(5)]
    got, want = _both(eng, g5, pats, pm.MORPH_NAIVE)
    assert got == want
    got, want = _both(eng, g5, [(5, m, False) for m in P.connected_classes(5)], pm.MORPH_NONE)
    assert got == want


def test_noalloc_rejects_oversized(eng):
    """A query beyond the static array's plan limit (64) is refused with
    PM_E_NOMEM, and the entry point keeps working afterwards."""
    from itertools import combinations_with_replacement
    import paper_2012_04553_amd as pm
    g = gen.erdos_renyi(50, 0.2, 12).with_labels(gen.zipf_labels(50, 5, 1.2, 13))
    star = (1 << 0) | (1 << 1) | (1 << 3)
    pats = [(4, star, False, [c, x, y, z]) for c in range(5)
            for x, y, z in combinations_with_replacement(range(5), 3)][:70]
    gid = eng.load(g)
    try:
        with pytest.raises(pm.PMError) as ei:
            eng.count_noalloc(gid, pats, morph=pm.MORPH_NONE)
        assert ei.value.status == -2, str(ei.value)
        want = eng.count(gid, pats[:20], morph=pm.MORPH_NONE)
        assert eng.count_noalloc(gid, pats[:20], morph=pm.MORPH_NONE) == want
    finally:
        eng.graph_unload(gid)
