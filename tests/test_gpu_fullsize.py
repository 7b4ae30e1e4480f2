"""GPU parity at the full benchmark size: 4-vertex counts of R-MAT scale 20
(edge factor 16, seed 2) in the launch configuration the benchmark times,
against the oracle's counts stored in tests/golden/rmat20_4mc.txt (written
by tests/golden/make_rmat20_4mc.py, which calls only the oracle)."""
import os
import sys

import pytest

import gen
import oracle

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "rmat20_4mc.txt")
NAMES = ["star3", "path4", "tailed_triangle", "cycle4", "diamond", "clique4"]


def _golden():
    out = {"EI": {}, "VI": {}}
    with open(GOLDEN) as f:
        for line in f:
            w = line.split()
            if not w or w[0].startswith("#"):
                continue
            if w[0] in ("EI", "VI"):
                out[w[0]][w[1]] = int(w[2])
            else:
                out[w[0]] = w[1]
    return out


def test_rmat20_counts_match_oracle():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2012_04553_amd as pm

    want = _golden()
    print("generating R-MAT scale 20 (seed 2)", flush=True)
    g = gen.rmat(20, 16, 0.57, 0.19, 0.19, 0.05, seed=2)
    assert gen.sha256_of(g) == want["sha256"], "generator output changed; rerun make_rmat20_4mc.py"
    names = oracle.named_4()  # pattern masks by name
    eng = pm.Engine(arena_bytes=48 << 30)
    try:
        gid = eng.load(g)
        print("morphed vertex-induced 4-MC", flush=True)
        got_vi = eng.count(gid, [(4, names[n], True) for n in NAMES], morph=pm.MORPH_NAIVE)
        assert got_vi == [want["VI"][n] for n in NAMES]
        print("edge-induced patterns matched directly", flush=True)
        got_ei = eng.count(gid, [(4, names[n], False) for n in NAMES], morph=pm.MORPH_NONE)
        assert got_ei == [want["EI"][n] for n in NAMES]
        print("cost-based morphing", flush=True)
        got_cost = eng.count(gid, [(4, names[n], True) for n in NAMES], morph=pm.MORPH_COST)
        assert got_cost == got_vi
    finally:
        eng.close()
