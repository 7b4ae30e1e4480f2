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
