"""Write rmat20_4mc.txt: the exact 4-vertex counts of the R-MAT scale-20
benchmark graph (edge factor 16, (a,b,c,d) = (0.57, 0.19, 0.19, 0.05),
seed 2), computed by the oracle alone.

Edge-induced counts come from the oracle's closed forms over per-vertex
degrees and per-edge common-neighbour counts (3-star, 3-path, tailed
triangle, diamond), its co-degree 4-cycle count and its 4-clique
enumeration; vertex-induced counts follow by Corollary 3.1.  The graph is
identified by the sha256 of its CSR so a test can tell that it regenerated
the same graph.

    python tests/golden/make_rmat20_4mc.py      (about 2-3 minutes)
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import gen  # noqa: E402
import oracle  # noqa: E402

NAMES = ["star3", "path4", "tailed_triangle", "cycle4", "diamond", "clique4"]


def main():
    g = gen.rmat(20, 16, 0.57, 0.19, 0.19, 0.05, seed=2)
    names = oracle.named_4()
    ei = oracle.edge_induced_4_from_tier_c(g)
    vi = oracle.P.vertex_induced_from_edge_induced(4, ei)
    out = os.path.join(HERE, "rmat20_4mc.txt")
    with open(out, "w") as f:
        f.write("# Exact 4-vertex counts of R-MAT scale 20, edge factor 16, (0.57,0.19,0.19,0.05), seed 2.\n")
        f.write("# Written by make_rmat20_4mc.py from the oracle only (closed forms + 4-cycle co-degrees\n")
        f.write("# + 4-clique enumeration; vertex-induced by Corollary 3.1).\n")
        f.write(f"sha256 {gen.sha256_of(g)}\n")
        f.write(f"n {g.n}\nm {g.m}\n")
        for nm in NAMES:
            f.write(f"EI {nm} {ei[names[nm]]}\n")
        for nm in NAMES:
            f.write(f"VI {nm} {vi[names[nm]]}\n")
    print(f"wrote {out}")


if __name__ == "__main__":
    main()
