"""Error paths of the C-ABI on the GPU.  Malformed graphs are rejected with
PM_E_INVAL (nothing is loaded and the context stays usable), and a count
outside int64 is reported as PM_E_OVERFLOW instead of wrapping (no result
ever leaves int64 silently)."""
from math import comb

import numpy as np
import pytest

import gen

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


def _csr(n, rows):
    rp = [0]
    col = []
    for r in rows:
        col.extend(r)
        rp.append(len(col))
    assert len(rp) == n + 1
    return np.array(rp, dtype=np.uint32), np.array(col, dtype=np.uint32)


MALFORMED = {
    # name: (n, row_ptr, col)
    "row_ptr_start": (2, np.array([1, 2, 3], dtype=np.uint32), np.array([1, 0, 0], dtype=np.uint32)),
    "row_ptr_decreasing": (3, np.array([0, 2, 1, 2], dtype=np.uint32), np.array([1, 0], dtype=np.uint32)),
    "odd_entries": (3,) + _csr(3, [[1], [0, 2], []]),
    "id_out_of_range": (4,) + _csr(4, [[1], [0], [9, 10], []]),
    "self_loop": (3,) + _csr(3, [[0, 1], [0, 1], []]),
    "unsorted": (3,) + _csr(3, [[2, 1], [0], [0]]),
    "duplicate": (3,) + _csr(3, [[1, 1], [0, 0], []]),
    "asymmetric": (3,) + _csr(3, [[1], [2], []]),
    "empty": (0, np.array([0], dtype=np.uint32), np.array([], dtype=np.uint32)),
}


@pytest.mark.parametrize("name", sorted(MALFORMED))
def test_malformed_csr_rejected(eng, name):
    import paper_2012_04553_amd as pm
    n, rp, col = MALFORMED[name]
    print(f"malformed CSR: {name}", flush=True)
    with pytest.raises(pm.PMError) as ei:
        eng.graph_load(n, rp, col)
    assert ei.value.status == -1, (name, str(ei.value))
    # the context still serves a valid graph afterwards
    g = gen.complete_graph(5)
    gid = eng.load(g)
    try:
        assert eng.count(gid, [(3, 0b111, False)], morph=pm.MORPH_NONE) == [10]
    finally:
        eng.graph_unload(gid)


def test_count_overflow_reported(eng):
    """The 5-vertex star on a star with L leaves has C(L, 4) copies:
    100,000 leaves fit int64 (exact value), 125,000 do not (about 1.02e19)."""
    import paper_2012_04553_amd as pm
    star5 = (1 << 0) | (1 << 1) | (1 << 3) | (1 << 6)   # centre 0, leaves 1..4
    star4 = (1 << 0) | (1 << 1) | (1 << 3)
    for leaves in (100_000, 125_000):
        print(f"star with {leaves} leaves", flush=True)
        gid = eng.load(gen.star_graph(leaves))
        try:
            assert eng.count(gid, [(4, star4, False)], morph=pm.MORPH_NONE) == [comb(leaves, 3)]
            want = comb(leaves, 4)
            if want <= 2 ** 63 - 1:
                assert eng.count(gid, [(5, star5, False)], morph=pm.MORPH_NONE) == [want]
            else:
                with pytest.raises(pm.PMError) as ei:
                    eng.count(gid, [(5, star5, False)], morph=pm.MORPH_NONE)
                assert ei.value.status == -3, str(ei.value)
                # the same context keeps answering
                assert eng.count(gid, [(4, star4, False)], morph=pm.MORPH_NONE) == [comb(leaves, 3)]
        finally:
            eng.graph_unload(gid)
