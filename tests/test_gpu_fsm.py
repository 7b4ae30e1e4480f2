"""Labeled 3-edge FSM with MNI support on the GPU against the oracle."""
import sys
import time

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


def _slot_pattern(L, s):
    import paper_2012_04553_amd as pm
    k, mask, labs = pm.fsm_slot(L, s)
    return k, mask, labs


@pytest.mark.parametrize("gname", ["er", "rmat", "star", "kn"])
def test_fsm_all_slots_small(eng, gname):
    L = 3
    if gname == "er":
        g = gen.erdos_renyi(40, 0.15, 31)
        g = g.with_labels(gen.zipf_labels(g.n, L, 1.2, 32))
    elif gname == "rmat":
        g = gen.rmat(7, 8, seed=33)
        g = g.with_labels(gen.zipf_labels(g.n, L, 1.2, 34))
    elif gname == "star":
        g = gen.star_graph(7)
        g = g.with_labels(np.array([0, 1, 1, 2, 0, 1, 2, 2], dtype=np.uint8))
    else:
        g = gen.complete_graph(6)
        g = g.with_labels(np.array([0, 0, 1, 1, 2, 0], dtype=np.uint8))
    gid = eng.load(g)
    try:
        sup, freq = eng.fsm(gid, L, threshold=3)
    finally:
        eng.graph_unload(gid)
    import paper_2012_04553_amd as pm
    assert len(sup) == pm.fsm_num_slots(L)
    for s in range(len(sup)):
        k, mask, labs = _slot_pattern(L, s)
        want = oracle.mni_support(g, k, mask, False, labs)
        assert sup[s] == want, (gname, s, k, mask, labs)
        assert freq[s] == (want >= 3)


def test_fsm_sixteen_labels_sampled(eng):
    L = 16
    g = gen.rmat(10, 8, seed=35)
    g = g.with_labels(gen.zipf_labels(g.n, L, 1.2, 36))
    gid = eng.load(g)
    try:
        sup, freq = eng.fsm(gid, L, threshold=10)
    finally:
        eng.graph_unload(gid)
    rng = np.random.default_rng(0)
    slots = list(rng.choice(len(sup), size=60, replace=False))
    slots += [int(i) for i in np.argsort(-sup)[:15]]
    for s in slots:
        k, mask, labs = _slot_pattern(L, int(s))
        want = oracle.mni_support_rooted(g, k, mask, False, labs)
        assert sup[s] == want, (s, k, mask, labs)


def test_fsm_sixteen_labels_every_slot(eng):
    """All 46,768 slots at 16 labels on R-MAT graphs small enough for the
    oracle to enumerate every match of each 3-edge shape once."""
    import paper_2012_04553_amd as pm
    L = 16
    for scale, seed in ((9, 37), (10, 39)):
        g = gen.rmat(scale, 8, seed=seed)
        g = g.with_labels(gen.zipf_labels(g.n, L, 1.2, seed + 1))
        gid = eng.load(g)
        try:
            sup, freq = eng.fsm(gid, L, threshold=8)
        finally:
            eng.graph_unload(gid)
        by_shape = {}
        for s in range(len(sup)):
            k, mask, labs = _slot_pattern(L, s)
            by_shape.setdefault((k, mask), []).append((s, labs))
        assert sum(len(v) for v in by_shape.values()) == 46768
        nonzero = 0
        for (k, mask), items in by_shape.items():
            want = oracle.mni_labelings(g, k, mask, False, L, [labs for _, labs in items])
            for (s, labs), w in zip(items, want):
                assert sup[s] == w, (scale, s, k, mask, labs)
                assert freq[s] == (w >= 8)
                nonzero += w > 0
        _say(f"R-MAT {scale}: every slot equal, {nonzero} with nonzero support")


def _repeated_label_slots(L, ns, rng, count):
    """Slots whose pattern repeats a label (where injectivity between
    same-labeled pattern vertices decides membership)."""
    out = []
    for s in rng.permutation(ns):
        k, mask, labs = _slot_pattern(L, int(s))
        if len(set(labs)) < k and max(labs) <= 5:
            out.append(int(s))
            if len(out) == count:
                break
    return out


def test_fsm_config_scale_sampled(eng):
    """R-MAT scale 18, edge factor 8, Zipf(1.2) over 16 labels: 260 slots
    (random, highest-support, and 200 that repeat a label) against the
    rooted-search oracle."""
    import paper_2012_04553_amd as pm
    L = 16
    g = gen.rmat(18, 8, seed=4)
    g = g.with_labels(gen.zipf_labels(g.n, L, 1.2, 40))
    gid = eng.load(g)
    try:
        t = time.time()
        sup, freq = eng.fsm(gid, L, threshold=1000)
        _say(f"fsm config scale: {time.time() - t:.2f}s, frequent {int(freq.sum())}")
    finally:
        eng.graph_unload(gid)
    rng = np.random.default_rng(1)
    slots = [int(x) for x in rng.choice(len(sup), size=40, replace=False)]
    slots += [int(i) for i in np.argsort(-sup)[:20]]
    slots += _repeated_label_slots(L, len(sup), np.random.default_rng(2), 200)
    t = time.time()
    for s in slots:
        k, mask, labs = _slot_pattern(L, s)
        want = oracle.mni_support_rooted(g, k, mask, False, labs)
        assert sup[s] == want, (s, k, mask, labs)
        assert freq[s] == (want >= 1000)
    _say(f"  {len(slots)} slots equal the oracle ({time.time() - t:.1f}s)")
