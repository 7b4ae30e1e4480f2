"""Host-side checks of the C-ABI library (no GPU needed)."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "pm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pm_[a-z_0-9]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    from paper_2012_04553_amd.binding import LIB_PATH, SIGNATURES
    lib = ctypes.CDLL(LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), name
        assert name in SIGNATURES, name


def test_status_strings():
    from paper_2012_04553_amd.binding import lib
    assert lib().pm_status_str(0) == b"PM_OK"
    assert lib().pm_status_str(-3) == b"PM_E_OVERFLOW"


def test_morph_plan_matches_oracle_algebra():
    """pm_morph_plan (host-only) against the oracle's Corollary 3.1."""
    import oracle
    from oracle import P
    import paper_2012_04553_amd as pm
    for k in (3, 4, 5):
        cls = P.connected_classes(k)
        pats = [(k, m, True) for m in cls]
        alts, M = pm.morph_plan(pats)
        # random edge-induced counts -> vertex-induced via both algebras
        rng = np.random.default_rng(k)
        ne = {m: int(rng.integers(0, 10 ** 6)) for m in cls}
        ora = P.vertex_induced_from_edge_induced(k, ne)
        for i, m in enumerate(cls):
            val = 0
            for j, (ak, am, avi, alab) in enumerate(alts):
                assert not avi or am == P.clique_mask(k)
                val += int(M[i, j]) * ne[P.canonical(k, am)[0]]
            assert val == ora[m], (k, m)


def test_morph_plan_labeled_rows_are_exact():
    """Labeled vertex-induced query: the conversion row applied to oracle
    edge-induced counts equals the oracle vertex-induced count."""
    import gen
    import oracle
    from oracle import P
    import paper_2012_04553_amd as pm
    g = gen.erdos_renyi(25, 0.3, 4).with_labels(gen.zipf_labels(25, 2, 1.2, 6))
    for m in P.connected_classes(4):
        labs = [0, 1, 0, 1]
        alts, M = pm.morph_plan([(4, m, True, labs)])
        val = 0
        for j, (ak, am, avi, alab) in enumerate(alts):
            val += int(M[0, j]) * oracle.count(g, ak, am, bool(avi), alab)
        assert val == oracle.count(g, 4, m, True, labs)


def test_invalid_patterns_rejected_on_host():
    from paper_2012_04553_amd.binding import PMError
    import paper_2012_04553_amd as pm
    with pytest.raises(PMError):
        pm.morph_plan([(4, 0b000011, True)])      # disconnected
    with pytest.raises(PMError):
        pm.morph_plan([(6, 0, True)])             # k out of range


def _oracle_three_edge_forms(L):
    """Canonical forms of every labeled connected pattern with 3 edges on L
    labels (the triangle, the 3-path and the 3-star; any labeling), from the
    oracle's pattern algebra."""
    from itertools import product
    from oracle import P
    forms = set()
    for k in (3, 4):
        for m in P.connected_classes(k):
            if P.edge_count(m) != 3:
                continue
            for labs in product(range(L), repeat=k):
                forms.add((k,) + P.canonical(k, m, labs))
    return forms


@pytest.mark.parametrize("L", [3, 16])
def test_fsm_slot_table_complete_and_distinct(L):
    """pm_fsm_slot enumerates every labeled 3-edge pattern exactly once:
    the slots' canonical forms are distinct and equal the oracle's set
    (85 at 3 labels, 46,768 at 16)."""
    from oracle import P
    import paper_2012_04553_amd as pm
    want = _oracle_three_edge_forms(L)
    ns = pm.fsm_num_slots(L)
    assert ns == len(want) == {3: 85, 16: 46768}[L]
    seen = set()
    for s in range(ns):
        k, mask, labs = pm.fsm_slot(L, s)
        assert P.edge_count(mask) == 3 and P.is_connected(k, mask)
        seen.add((k,) + P.canonical(k, mask, labs))
    assert len(seen) == ns
    assert seen == want
