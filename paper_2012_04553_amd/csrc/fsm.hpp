// Device arguments of the labeled 3-edge FSM kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

constexpr int FSM_LMAX = 16;                    // labels supported
constexpr int FSM_SCRATCH_WORDS = FSM_LMAX * 12;  // per-thread 64-bit words (three 256-bit sets per label)
#ifndef PM_FSM_HUB
#define PM_FSM_HUB 32
#endif
constexpr uint32_t FSM_HUB = PM_FSM_HUB;  // vertices with this many neighbours or more: one wavefront each

struct FsmArgs {
    const uint32_t* rp;
    const uint32_t* col;
    const uint8_t* lab;
    uint32_t n;
    int L;
    uint32_t* hist;     // n * FSM_LMAX neighbour-label counts
    uint32_t* pres;     // n * 3: labels with count >= 1, >= 2, >= 3
    uint8_t* bcnt;      // n * FSM_LMAX^2 (saturating)
    uint8_t* bfrag;     // n * FSM_LMAX^2 (saturating)
    uint32_t* bmask;    // n * FSM_LMAX
    const int32_t* tricode;  // sorted label triple -> slot
    const int32_t* p4code;   // ordered label 4-tuple -> slot<<2 | reversed<<1 | palindrome
    const int32_t* s3code;   // (centre, sorted leaf triple) -> slot
    uint32_t* counts;   // nslots * 4 domain sizes
    uint64_t* scratch;  // per thread FSM_SCRATCH_WORDS
    const uint32_t* order;  // n vertices sorted by label
    const uint32_t* split;  // per vertex: index of the first neighbour above it
    unsigned long long* tri;  // n * 4: label pairs of the triangles at each vertex
    uint32_t hub0;      // first id of degree >= FSM_HUB (ids ascend with degree), or n
};

// The five FSM kernels in order (fsm_hist, fsm_tri, fsm_btab, fsm_main for
// vertices below FSM_HUB neighbours, fsm_hub for the others); with `ev`
// (6 events), ev[i] is recorded before kernel i and ev[5] after the last.
int launch_fsm(const FsmArgs& a, int grid, hipStream_t s, hipEvent_t* ev = nullptr);

}  // namespace pm
