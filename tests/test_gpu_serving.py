"""Serving loop: continuous batching over resident graphs.  Each request's
result in the mix must equal the same request alone (exact)."""
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
    e = pm.Engine(arena_bytes=16 << 30)
    yield e
    e.close()


@pytest.fixture(scope="module")
def graphs(eng):
    gs = [gen.erdos_renyi(300, 0.03, 61).with_labels(gen.zipf_labels(300, 16, 1.2, 62)),
          gen.rmat(9, 8, seed=63).with_labels(gen.zipf_labels(512, 16, 1.2, 64)),
          gen.chung_lu(2000, 2.1, 20, seed=65).with_labels(gen.zipf_labels(2000, 16, 1.2, 66))]
    ids = [eng.load(g) for g in gs]
    yield gs, ids
    for i in ids:
        eng.graph_unload(i)


def _trace(ids, n, qps, seed, k_choices=(3, 4)):
    import paper_2012_04553_amd as pm
    qs = gen.query_stream(n, qps, len(ids), seed=seed, k_choices=k_choices)
    return [(q.arrival_s, ids[q.graph], q.patterns, pm.MORPH_NAIVE) for q in qs]


def test_serving_mix_equals_alone(eng, graphs):
    import paper_2012_04553_amd as pm
    gs, ids = graphs
    reqs = _trace(ids, 120, 2000.0, seed=7)
    res, st = eng.serve(reqs, max_slots=4, max_batch=4)
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["batches"] >= 1 and st["p50_s"] <= st["p99_s"] <= st["max_s"]
    assert any(r["batch_size"] > 1 for r in res), "no batching happened"
    for (t, gid, pats, morph), r in zip(reqs, res):
        assert r["status"] == 0
        alone = eng.count(gid, pats, morph=morph)
        assert r["values"] == alone
    # oracle on a few requests of the smallest graph
    checked = 0
    for (t, gid, pats, morph), r in zip(reqs, res):
        if gid != ids[0] or checked >= 10:
            continue
        g = gs[0]
        want = [oracle.count(g, k, m, ind, labs) for (k, m, ind, labs) in pats]
        assert r["values"] == want
        checked += 1
    assert checked > 0


def test_serving_five_vertex_and_cost_mode(eng, graphs):
    """Five-vertex requests side by side (each slot fills its own edge
    supports for the triangle-count closed forms) equal the same requests
    counted alone, with the closed forms and without, and in cost mode."""
    import paper_2012_04553_amd as pm
    gs, ids = graphs
    reqs = _trace(ids[:2], 40, 1000.0, seed=8, k_choices=(5,))
    res, st = eng.serve(reqs, max_slots=3, max_batch=2)
    assert st["failed"] == 0
    for (t, gid, pats, morph), r in zip(reqs, res):
        assert r["values"] == eng.count(gid, pats, morph=morph)
    with _enumerating(eng):
        res1, st1 = eng.serve(reqs, max_slots=3, max_batch=2)
    cost = [(t, gid, pats, pm.MORPH_COST) for (t, gid, pats, m) in reqs]
    res2, st2 = eng.serve(cost, max_slots=3, max_batch=2)
    for a, b, c in zip(res, res1, res2):
        assert a["values"] == b["values"] == c["values"]


def test_serving_admission_by_budget(eng, graphs):
    """A budget that holds one batch at a time still serves everything;
    a request larger than the whole budget fails alone with PM_E_NOMEM."""
    import paper_2012_04553_amd as pm
    gs, ids = graphs
    reqs = _trace(ids[:1], 30, 3000.0, seed=9)
    one = eng.footprint(ids[0], reqs[0][2], morph=pm.MORPH_NAIVE)
    biggest = max(eng.footprint(gid, pats, morph=pm.MORPH_NAIVE) for (_, gid, pats, _) in reqs)
    res, st = eng.serve(reqs, max_slots=4, max_batch=1, budget_bytes=biggest)
    assert st["failed"] == 0 and st["completed"] == len(reqs)
    for (t, gid, pats, morph), r in zip(reqs, res):
        assert r["values"] == eng.count(gid, pats, morph=morph)
    tiny = [(0.0, ids[0], reqs[0][2], pm.MORPH_NAIVE)]
    res, st = eng.serve(tiny, max_slots=1, max_batch=1, budget_bytes=max(one // 4, 1))
    assert res[0]["status"] == -2 and st["failed"] == 1


def _heavy5():
    """The house (a 5-cycle with one chord), edge-induced: with the
    triangle-count closed forms off (edge_support 0) its plan enumerates long
    enough on R-MAT 14 to be cancelled, or to time out in a
    serving slot (a share of the GPU)."""
    return P.canonical(5, 0xED)[0]


class _enumerating:
    """Closed forms over triangle counts off for the duration."""
    def __init__(self, eng):
        self.eng = eng

    def __enter__(self):
        self.eng.set_option("edge_support", 0)

    def __exit__(self, *exc):
        self.eng.set_option("edge_support", 1)


def test_cancel_heavy_query(eng):
    """Cancellation is forced from the host: the kernels stop taking work
    items and pm_wait reports PM_E_CANCELLED; the next query is exact."""
    import time
    import paper_2012_04553_amd as pm
    from paper_2012_04553_amd.binding import PMError
    g = gen.rmat(14, 16, seed=3)
    gid = eng.load(g)
    try:
        # the edge-induced house alone, enumerated, runs for about a second here
        heavy = [(5, _heavy5(), False)]
        t = time.time()
        with _enumerating(eng):
            tk = eng.submit(gid, heavy, morph=pm.MORPH_NONE)
            time.sleep(0.2)
            eng.cancel(tk)
            with pytest.raises(PMError) as ei:
                eng.wait(tk, 1)
        assert ei.value.status == -8
        assert time.time() - t < 5.0
        pats = [(4, m, True) for m in P.connected_classes(4)]
        got = eng.count(gid, pats, morph=pm.MORPH_NAIVE)
        want = oracle.vertex_induced_4_from_tier_c(g)
        assert got == [want[m] for m in P.connected_classes(4)]
        # a morphed 5-motif query that fills edge supports, cancelled at once
        # (its kernels may stop anywhere): the next query, which reads
        # supports too, is still exact
        five = [(5, m, True) for m in P.connected_classes(5)]
        tk = eng.submit(gid, five, morph=pm.MORPH_NAIVE)
        eng.cancel(tk)
        try:
            eng.wait(tk, 1)
        except PMError as e:
            assert e.status == -8
        assert eng.count(gid, pats, morph=pm.MORPH_NAIVE) == [want[m] for m in P.connected_classes(4)]
    finally:
        eng.graph_unload(gid)


def test_serving_deadline(eng, graphs):
    import paper_2012_04553_amd as pm
    gs, ids = graphs
    heavy_g = gen.rmat(14, 16, seed=3)
    hid = eng.load(heavy_g)
    try:
        heavy = [(5, _heavy5(), False)]
        reqs = [(0.0, hid, heavy, pm.MORPH_NONE)]
        light = _trace(ids[:1], 10, 1000.0, seed=11)
        reqs += [(t + 0.01, gid, pats, m) for (t, gid, pats, m) in light]
        with _enumerating(eng):
            res, st = eng.serve(reqs, max_slots=4, max_batch=1, deadline_s=0.5)
        assert res[0]["status"] == -7
        # a light batch may wait behind the long one if their streams share a
        # hardware queue; what completes must be exact, and most must complete
        done = [(q, r) for q, r in zip(reqs[1:], res[1:]) if r["status"] == 0]
        assert all(r["status"] in (0, -7) for r in res[1:])
        assert len(done) >= 0.8 * (len(reqs) - 1)
        for (t, gid, pats, morph), r in done:
            assert r["values"] == eng.count(gid, pats, morph=morph)
    finally:
        eng.graph_unload(hid)


def test_serving_sheds_after_timeout(eng, graphs):
    """Once its class has timed out twice, a request estimated at the work of
    a batch that timed out ends at admission; cheaper requests still
    complete, exactly."""
    import paper_2012_04553_amd as pm
    gs, ids = graphs
    heavy_g = gen.rmat(14, 16, seed=3)
    hid = eng.load(heavy_g)
    try:
        heavy = [(5, _heavy5(), False)]
        reqs = [(0.0, hid, heavy, pm.MORPH_NONE)]
        light = _trace(ids[:1], 12, 10.0, seed=13)
        reqs += [(t, gid, pats, m) for (t, gid, pats, m) in light]
        reqs.append((light[-1][0] + 1.5, hid, heavy, pm.MORPH_NONE))
        reqs.append((light[-1][0] + 3.0, hid, heavy, pm.MORPH_NONE))
        reqs.sort(key=lambda q: q[0])
        with _enumerating(eng):
            res, st = eng.serve(reqs, max_slots=4, max_batch=4, deadline_s=0.5)
        heavy_idx = [i for i, q in enumerate(reqs) if q[1] == hid]
        assert [res[i]["status"] for i in heavy_idx] == [-7, -7, -7]
        assert st["shed"] >= 1
        # the second heavy request ran to its deadline (one timeout is not
        # enough); the third never ran: it ended at admission
        assert res[heavy_idx[1]]["service_s"] > 0.0
        assert res[heavy_idx[2]]["service_s"] == 0.0
        for q, r in zip(reqs, res):
            if q[1] == hid:
                continue
            assert r["status"] == 0
            assert r["values"] == eng.count(q[1], q[2], morph=q[3])
    finally:
        eng.graph_unload(hid)
