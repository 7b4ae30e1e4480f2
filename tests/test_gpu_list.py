"""Listing (pm_list), direct and through morphing, against every match the
oracle enumerates, deduplicated into subgraphs.  A listed tuple is one of
the automorphic matches of its subgraph, so the comparison is on what is
unique: the set of subgraphs (vertex set and edge set), their number, and
that every tuple is a match."""
from itertools import product

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
    e = pm.Engine(arena_bytes=4 << 30)
    yield e
    e.close()


def _key(k, mask, tup):
    edges = frozenset(tuple(sorted((int(tup[i]), int(tup[j])))) for i, j in P.edges_of(k, mask))
    return frozenset(int(x) for x in tup), edges


def _is_match(g, k, mask, induced, labs, tup):
    adj = lambda u, v: v in set(int(x) for x in g.neighbors(u))
    if len(set(int(x) for x in tup)) != k:
        return False
    for j in range(k):
        for i in range(j):
            e = adj(int(tup[i]), int(tup[j]))
            if P.has_edge(mask, i, j) and not e:
                return False
            if induced and not P.has_edge(mask, i, j) and e:
                return False
    if labs is not None:
        return all(labs[v] < 0 or int(g.labels[int(tup[v])]) == labs[v] for v in range(k))
    return True


def _graphs():
    yield "er", gen.erdos_renyi(24, 0.25, 81).with_labels(gen.zipf_labels(24, 3, 1.2, 82))
    g = gen.rmat(6, 6, seed=83)
    yield "rmat", g.with_labels(gen.zipf_labels(g.n, 3, 1.2, 84))


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_list_direct_and_morphed(eng, k):
    import paper_2012_04553_amd as pm
    rng = np.random.default_rng(k)
    for gname, g in _graphs():
        gid = eng.load(g)
        try:
            for m in P.connected_classes(k):
                for induced in (False, True):
                    for labs in (None, [int(x) for x in rng.integers(0, 3, size=k)]):
                        want = {_key(k, m, t) for t in oracle.list_maps(g, k, m, induced, labs)}
                        assert len(want) == oracle.count(g, k, m, induced, labs)
                        for morph in (pm.MORPH_NONE, pm.MORPH_NAIVE):
                            tuples, total = eng.list(gid, (k, m, induced, labs), morph=morph)
                            assert total == len(tuples) == len(want), (gname, m, induced, labs, morph)
                            got = [_key(k, m, t) for t in tuples]
                            assert len(set(got)) == len(got)
                            assert set(got) == want
                            for t in tuples[:50]:
                                assert _is_match(g, k, m, induced, labs, t)
        finally:
            eng.graph_unload(gid)


def test_list_capacity(eng):
    """A short buffer receives the first tuples and the full count."""
    import paper_2012_04553_amd as pm
    g = gen.complete_graph(7)
    gid = eng.load(g)
    try:
        tri = (3, 0b111, False)
        tuples, total = eng.list(gid, tri, morph=pm.MORPH_NONE, capacity=5)
        assert total == 35 and len(tuples) == 5
        tuples, total = eng.list(gid, tri, morph=pm.MORPH_NONE)
        assert total == 35 and len({frozenset(t) for t in tuples}) == 35
    finally:
        eng.graph_unload(gid)
