// Kernel-side argument block shared by the runtime and the HIP kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace pm {

struct KGraph {
    const uint32_t* rp;   // row offsets, n+1 (degree-ordered ids)
    const uint32_t* col;  // sorted adjacency
    const uint32_t* split;  // per vertex: index of the first neighbour above it
    const uint8_t* lab;   // labels or null
    uint32_t n;
};

// A work item: roots [r0, r1) of one plan; for a single high-degree root,
// the slice [s0, s1) of its level-1 candidates.
struct KItem {
    uint32_t r0, r1, s0, s1;
};

struct KArgs {
    KGraph g;
    const DPlan* plans;
    int32_t nplans;
    uint32_t nitems;          // items per plan (the item list is shared)
    const KItem* items;
    uint64_t* counters;       // 2 x u64 (lo, hi) per plan
    uint32_t* head;           // work-queue head
    uint32_t* scratch;        // per-wave level buffers: KMAX * buf_stride each
    uint64_t buf_stride;
    uint32_t* aggcnt;         // per-wave dense counters (n each), zeroed
    uint32_t* aggtouch;       // per-wave touched lists (n each)
    uint64_t* bytes;          // algorithmic bytes (counting launch only)
    uint32_t* rootbm;         // per-wave root adjacency bitmaps (bm_words each), zeroed
    uint64_t bm_words;
    // two-hop plans whose aggregation is the first level: the heaviest roots
    // run in two launches over one shared counter array per (plan, root):
    // agg_mode 1 adds the paths of a slice of the root's bridges, agg_mode 2
    // evaluates a range of targets.  0 = every other launch.
    uint32_t agg_mode;
    uint32_t heavy_k;         // heavy roots (arrays per plan)
    uint32_t* heavy;          // (plan * heavy_k + h) * n counters, zeroed
    const int* cancel;        // host-visible cancel flag or null
};

int launch_match(const KArgs& a, int grid, int block, bool count_bytes, hipStream_t s);
// Clears `words` 32-bit words (used instead of memset nodes inside graphs).
int launch_zero(uint32_t* p, uint64_t words, hipStream_t s);

}  // namespace pm
