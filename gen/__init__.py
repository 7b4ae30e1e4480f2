"""Seeded synthetic inputs shared by the oracle and the GPU path.

This package only draws random graphs, vertex labels and query streams and
writes them as plain simple-undirected CSR arrays.  It holds none of the
pattern-counting arithmetic: neither side of a parity test can borrow a
counting step from here.
"""
from .graphs import (  # noqa: F401
    Graph,
    erdos_renyi,
    rmat,
    chung_lu,
    zipf_labels,
    from_edges,
    complete_graph,
    complete_bipartite,
    star_graph,
    cycle_graph,
    graph_from_mask,
    sha256_of,
)
from .queries import Query, connected_masks, query_stream  # noqa: F401
