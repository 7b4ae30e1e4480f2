// Device arguments of the minimum-node-image (MNI) domain kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace pm {

// One domain column: the data vertices x for which some match of a pattern
// maps the column's pattern vertex to x.  Found by an existence search
// rooted at x: step 0 is the column vertex, every later step a pattern
// vertex adjacent to an earlier one.
struct MTask {
    uint8_t k;               // search steps (pattern vertices)
    uint8_t adj[KMAX];       // step j: earlier steps its image is adjacent to
    uint8_t anti[KMAX];      // step j: earlier steps its image is not adjacent to
    int8_t label[KMAX];      // step j: label, -1 = any
    uint32_t pos_b, pos_e;   // candidate roots: positions [pos_b, pos_e) of the root order
};

constexpr uint32_t MNI_CHUNK = 16;   // roots per work item

struct MArgs {
    KGraph g;
    const uint32_t* order;     // root order (vertices by label), or null = identity
    const MTask* tasks;
    const uint64_t* prefix;    // work items before each task (ntasks + 1)
    uint32_t ntasks;
    uint32_t* dom;             // ntasks bitmaps of `words` u32, zeroed
    uint64_t words;
    uint32_t* head;            // work-queue head, zeroed
    const int* cancel;         // host-visible cancel flag or null
};

// A column of a query pattern: the union of `count` task bitmaps whose
// indices are list[first .. first + count).
struct MOut {
    uint32_t first, count;
};

// Listing: every distinct matched subgraph once.  The searches of the
// route patterns (the pattern itself, or every p + S read vertex-induced)
// enumerate all their matches from every root; a match is kept when it is
// the lexicographically smallest of its images under the listed pattern's
// automorphisms (one per subgraph) and written, in pattern-vertex order,
// at the next position of `out` while `cap` allows (`count` counts all).
struct LArgs {
    KGraph g;
    const uint32_t* order;     // root order (vertices by label), or null = identity
    const MTask* tasks;
    const uint8_t* steps;      // per task: the pattern vertex of each step (KMAX bytes)
    const uint64_t* prefix;    // work items before each task (ntasks + 1)
    uint32_t ntasks;
    const uint8_t* aut;        // automorphisms of the listed pattern, naut x KMAX
    uint32_t naut;
    uint32_t k;
    uint32_t* out;             // cap tuples of k vertex ids
    uint64_t cap;
    unsigned long long* count; // matches kept (also beyond cap), zeroed
    uint32_t* head;            // work-queue head, zeroed
};

int launch_mni(const MArgs& a, int grid, hipStream_t s);
int launch_list(const LArgs& a, int grid, hipStream_t s);
// counts[o] = popcount of the union of output o's bitmaps (counts zeroed)
int launch_mni_union(const uint32_t* dom, uint64_t words, const uint32_t* list, const MOut* outs,
                     uint32_t nout, unsigned long long* counts, int grid, hipStream_t s);

}  // namespace pm
