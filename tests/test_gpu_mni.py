"""MNI support through pm_submit (PM_AGG_MNI), direct and morphed
(Theorem 3.2), the morphed 3-edge FSM route, and level-wise FSM, against the
oracle's minimum-node-image supports (supports are integers: exact
equality)."""
import time
from itertools import product

import numpy as np
import pytest

import gen
import oracle
from oracle import P

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)


@pytest.fixture(scope="module")
def eng():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_04553_amd as pm
    e = pm.Engine(arena_bytes=8 << 30)
    yield e
    e.close()


def _graphs():
    yield "er", gen.erdos_renyi(30, 0.2, 41).with_labels(gen.zipf_labels(30, 3, 1.2, 42))
    g = gen.rmat(7, 6, seed=43)
    yield "rmat", g.with_labels(gen.zipf_labels(g.n, 3, 1.2, 44))
    yield "star", gen.star_graph(6).with_labels(np.array([0, 1, 1, 2, 0, 1, 2], dtype=np.uint8))
    yield "kn", gen.complete_graph(6).with_labels(np.array([0, 0, 1, 1, 2, 0], dtype=np.uint8))


def _patterns(k, rng):
    out = []
    for m in P.connected_classes(k):
        for induced in (False, True):
            out.append((k, m, induced, None))
            out.append((k, m, induced, [int(x) for x in rng.integers(0, 3, size=k)]))
            out.append((k, m, induced, [0] * k))
    return out


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_mni_direct_and_morphed(eng, k):
    import paper_2012_04553_amd as pm
    rng = np.random.default_rng(k)
    for gname, g in _graphs():
        _say(f"MNI k={k} on {gname}")
        pats = _patterns(k, rng)
        want = [oracle.mni_support(g, kk, m, ind, labs) for kk, m, ind, labs in pats]
        gid = eng.load(g)
        try:
            for morph in (pm.MORPH_NONE, pm.MORPH_NAIVE, pm.MORPH_COST):
                got = eng.mni(gid, [(kk, m, ind, labs) for kk, m, ind, labs in pats], morph=morph)
                for p, gv, wv in zip(pats, got, want):
                    assert gv == wv, (gname, morph, p)
        finally:
            eng.graph_unload(gid)


@pytest.mark.parametrize("gname", ["er", "rmat", "star", "kn"])
def test_fsm_morphed_all_slots(eng, gname):
    """pm_fsm through Theorem 3.2 (PM_MORPH_NAIVE) equals the direct route
    and the oracle on every slot at 3 labels."""
    import paper_2012_04553_amd as pm
    g = dict(_graphs())[gname]
    L = 3
    gid = eng.load(g)
    try:
        plain, fp = eng.fsm(gid, L, threshold=3, morph=pm.MORPH_NONE)
        morphed, fm = eng.fsm(gid, L, threshold=3, morph=pm.MORPH_NAIVE)
    finally:
        eng.graph_unload(gid)
    assert list(plain) == list(morphed)
    assert list(fp) == list(fm)
    for s in range(len(plain)):
        k, mask, labs = pm.fsm_slot(L, s)
        assert morphed[s] == oracle.mni_support(g, k, mask, False, labs), (gname, s)


def test_mni_config_scale_sampled(eng):
    """R-MAT scale 18, edge factor 8, Zipf(1.2) over 16 labels: sampled FSM
    slots through pm_submit's MNI route, direct and morphed, equal the
    direct FSM kernels and the rooted-search oracle."""
    import paper_2012_04553_amd as pm
    L = 16
    g = gen.rmat(18, 8, seed=4)
    g = g.with_labels(gen.zipf_labels(g.n, L, 1.2, 40))
    rng = np.random.default_rng(7)
    gid = eng.load(g)
    try:
        t = time.time()
        table, _ = eng.fsm(gid, L, threshold=1000, morph=pm.MORPH_NONE)
        _say(f"direct FSM, all slots: {time.time() - t:.2f}s")
        slots = [int(x) for x in rng.choice(len(table), size=10, replace=False)]
        slots += [int(i) for i in np.argsort(-table)[:4]]
        pats = [pm.fsm_slot(L, s) for s in slots]
        qs = [(k, m, False, labs) for k, m, labs in pats]
        for morph in (pm.MORPH_NONE, pm.MORPH_NAIVE):
            t = time.time()
            got = eng.mni(gid, qs, morph=morph)
            _say(f"MNI route morph={morph}, {len(qs)} slots: {time.time() - t:.2f}s")
            assert got == [int(table[s]) for s in slots], morph
    finally:
        eng.graph_unload(gid)
    for (k, m, labs), s in zip(pats[:6], slots[:6]):
        assert oracle.mni_support_rooted(g, k, m, False, labs) == table[s]


def _oracle_frequent(g, L, max_edges, threshold):
    forms = set()
    for k in range(2, 6):
        for m in P.connected_classes(k):
            if P.edge_count(m) > max_edges:
                continue
            for labs in product(range(L), repeat=k):
                forms.add((k,) + P.canonical(k, m, labs))
    out = {}
    for k, m, labs in forms:
        s = oracle.mni_support(g, k, m, False, list(labs))
        if s >= threshold:
            out[(k, m, labs)] = s
    return out


@pytest.mark.parametrize("max_edges", [3, 4])
def test_fsm_levelwise(eng, max_edges):
    """Level-wise mining with anti-monotone pruning finds exactly the
    frequent patterns a brute-force enumeration of every labeled pattern
    finds, with the same supports."""
    import paper_2012_04553_amd as pm
    L = 2
    g = gen.erdos_renyi(22, 0.22, 45).with_labels(gen.zipf_labels(22, L, 1.0, 46))
    threshold = 4
    want = _oracle_frequent(g, L, max_edges, threshold)
    gid = eng.load(g)
    try:
        for morph in (pm.MORPH_NONE, pm.MORPH_NAIVE):
            res = eng.fsm_levelwise(gid, L, max_edges, threshold, morph=morph)
            got = {}
            for k, m, labs, s in res:
                cm, cl = P.canonical(k, m, labs)
                got[(k, cm, tuple(cl))] = s
            assert len(got) == len(res)
            assert got == want, (morph, set(got) ^ set(want))
            _say(f"level-wise FSM (<= {max_edges} edges, morph={morph}): {len(got)} frequent patterns")
    finally:
        eng.graph_unload(gid)
