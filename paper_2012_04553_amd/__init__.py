"""MI355X-native pattern-morphing subgraph counting.

The engine is the HIP/C++ library ``libpm.so`` behind the C-ABI in
``include/pm.h``; this package is its thin Python binding.
"""
from .binding import (  # noqa: F401
    AGG_COUNT,
    AGG_MNI,
    EDGE_INDUCED,
    MORPH_COST,
    MORPH_NAIVE,
    MORPH_NONE,
    VERTEX_INDUCED,
    Engine,
    PMError,
    lib,
    make_pattern,
    fsm_num_slots,
    fsm_slot,
    morph_plan,
    morph_plan_costs,
)
