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


def test_fsm_config_scale_sampled(eng):
    """R-MAT scale 18, edge factor 8, Zipf(1.2) over 16 labels: a sample of
    slots (random and highest-support) against the rooted-search oracle."""
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
    slots = [int(x) for x in rng.choice(len(sup), size=8, replace=False)]
    slots += [int(i) for i in np.argsort(-sup)[:4]]
    for s in slots:
        k, mask, labs = _slot_pattern(L, s)
        t = time.time()
        want = oracle.mni_support_rooted(g, k, mask, False, labs)
        _say(f"  slot {s} k={k} labels={labs}: gpu {sup[s]} oracle {want} ({time.time() - t:.1f}s)")
        assert sup[s] == want
