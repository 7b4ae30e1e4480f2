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
    // membership bitmaps (n bits, hub_words words each) of the vertices
    // hub0 .. n-1, the highest degrees; null when the graph has none
    const uint32_t* hubbm;
    uint32_t hub0, hub_words;
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
    // heavy two-hop roots (agg_window_kernel): per block, a cursor and an
    // end position for each bridge of the current root
    uint32_t* wscr;           // blocks * (2 + EW_TERMS) * wscr_stride
    uint64_t wscr_stride;
    const int* cancel;        // host-visible cancel flag or null
    uint32_t* support;        // per out-list position: triangles on that edge, or null
    uint32_t wide;            // 1: agg_window_kernel keeps 32-bit counters even
                              //    when every degree fits 16 bits
    uint64_t* vtri;           // per vertex: the supports of its edges summed
                              // (twice its triangles), zeroed; or null
    uint32_t mirror;          // 1: vtri_kernel also writes every support at
                              //    the lower end's entry in the higher end's
                              //    list
};

int launch_match(const KArgs& a, int grid, int block, bool count_bytes, hipStream_t s);
// Heavy roots of first-level two-hop plans: large workgroups (1024 threads
// and 142 KB of LDS by default), one root or root slice at a time, items
// {root, 0, slice, slices}; `grid` should not exceed the CU count times
// agg_window_cu_blocks(), the workgroups one CU holds.
int launch_agg_window(const KArgs& a, int grid, bool count_bytes, hipStream_t s);
// Fills the membership bitmaps of vertices hub0 .. n-1 (bm: (n - hub0) *
// words zeroed words).
int launch_hub_bitmaps(const KGraph& g, uint32_t* bm, uint32_t hub0, uint32_t words, hipStream_t s);
int agg_window_cu_blocks();
// Heavy roots of edge-core plans (edge_window_ok): one workgroup per root.
int launch_edge_window(const KArgs& a, int grid, bool count_bytes, hipStream_t s);
// Triangle-core plans (clique_ok), at most CQ_PLANS per launch: one
// wavefront per item {r0, r1, i0, i1} (roots [r0, r1), rows [i0, i1) of
// N+(r)).
int launch_clique(const KArgs& a, int grid, bool count_bytes, hipStream_t s);
// Edge-support plans (support_ok) and triangle-count closed forms (tagg)
// over a support array filled by a launch_clique with a.support set (and,
// for the closed forms, a.vtri filled by launch_vtri).
int launch_support(const KArgs& a, int grid, bool count_bytes, hipStream_t s);
// Per-vertex sums of the supports (a.vtri, zeroed beforehand): one thread
// per vertex over its out-list, one atomic per edge for the far end.
int launch_vtri(const KArgs& a, int grid, bool count_bytes, hipStream_t s);
// The house's 4-cycle support sums (TAGG_HOUSE plans) over the root items,
// one wavefront per item with its dense counter array (aggcnt/aggtouch),
// over supports mirrored by launch_vtri.
int launch_house(const KArgs& a, int grid, bool count_bytes, hipStream_t s);
// Per-triangle closed forms (TAGG_DTAIL, TAGG_FAN plans, at most CQ_PLANS
// a launch) over the triangle items {r0, r1, i0, i1}, reading the supports
// a launch_clique with a.support filled.
int launch_trisup(const KArgs& a, int grid, bool count_bytes, hipStream_t s);
// The K4 with an ear (one TAGG_K4EAR plan a launch) over the 4-clique items
// of `mode` (as launch_clique4), reading complete supports.
int launch_k4ear(const KArgs& a, int grid, int mode, bool count_bytes, hipStream_t s);
// Ordered 4-clique plans (clique4_ok), at most CQ_PLANS per launch: one
// wavefront (mode 0: up to C4_LIGHT_MAX out-neighbours) or one workgroup
// (mode 1: up to C4_HEAVY_MAX, mode 2: up to C4_ROOT_MAX) per root of the
// items {r0, r1, 0, 0}.
int launch_clique4(const KArgs& a, int grid, int mode, bool count_bytes, hipStream_t s);
// Edge-induced 5-cycle pair sums (plans with cyc5) over the root items,
// one wavefront per root with its dense counter array (aggcnt/aggtouch).
int launch_cycle5(const KArgs& a, int grid, bool count_bytes, hipStream_t s);
// Clears `words` 32-bit words (used instead of memset nodes inside graphs).
int launch_zero(uint32_t* p, uint64_t words, hipStream_t s);

}  // namespace pm
