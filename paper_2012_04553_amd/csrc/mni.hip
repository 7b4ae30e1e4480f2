// Minimum-node-image domains on gfx950.
//
// The MNI support of a pattern is the size of its smallest domain, the
// domain of a pattern vertex v being every data vertex some match maps v to
// (Preliminaries, FSM).  A domain column is computed by existence searches:
// for every candidate root x (the roots carrying v's label, a contiguous
// range of the label-sorted vertex order) a wavefront asks whether some
// match maps v to x.  The 64 lanes take 64 of x's neighbours at a time as
// the second pattern vertex and each continues the search depth first over
// the remaining (at most three) pattern vertices, every step drawing its
// candidates from the shortest adjacency list of its already-mapped pattern
// neighbours and testing the others (and, for vertex-induced patterns, the
// non-neighbours) by binary search, the labels and injectivity.  The wave
// stops at the first lane that completes a match (ballot) and sets x's bit.
//
// Domains of morphed patterns are unions of the domains of other patterns'
// columns (Theorem 3.2); mni_union_kernel ORs those bitmaps word by word and
// counts the bits.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "mni.hpp"

namespace pm {

namespace {

__device__ __forceinline__ bool adjacent(const KGraph& g, uint32_t u, uint32_t x) {
    uint32_t lo = g.rp[u], hi = g.rp[u + 1];
    const uint32_t end = hi;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (g.col[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < end && g.col[lo] == x;
}

// Candidate x for step j of task T, given the images img[0 .. j-1] and the
// driver step d (x is already a neighbour of img[d]).
__device__ __forceinline__ bool step_ok(const KGraph& g, const MTask& T, const uint32_t* img, int j, int d,
                                        uint32_t x) {
    if (T.label[j] >= 0 && g.lab[x] != (uint8_t)T.label[j]) return false;
    for (int i = 0; i < j; ++i)
        if (img[i] == x) return false;
    for (int i = 0; i < j; ++i) {
        if (i == d) continue;
        if ((T.adj[j] >> i) & 1) {
            if (!adjacent(g, img[i], x)) return false;
        } else if ((T.anti[j] >> i) & 1) {
            if (adjacent(g, img[i], x)) return false;
        }
    }
    return true;
}

// The shortest adjacency list among step j's mapped pattern neighbours.
__device__ __forceinline__ int driver(const KGraph& g, const MTask& T, const uint32_t* img, int j, uint32_t& b,
                                      uint32_t& e) {
    int best = -1;
    uint32_t len = 0xffffffffu;
    for (int i = 0; i < j; ++i) {
        if (!((T.adj[j] >> i) & 1)) continue;
        const uint32_t s = g.rp[img[i]], t = g.rp[img[i] + 1];
        if (t - s < len) {
            len = t - s;
            best = i;
            b = s;
            e = t;
        }
    }
    return best;
}

// Depth-first completion of a match whose steps 0 and 1 are mapped: true
// when some assignment of steps 2 .. k-1 satisfies every constraint.
__device__ bool lane_complete(const KGraph& g, const MTask& T, uint32_t* img) {
    if (T.k <= 2) return true;
    uint32_t pos[KMAX], end[KMAX];
    int drv[KMAX];
    int j = 2;
    drv[j] = driver(g, T, img, j, pos[j], end[j]);
    for (;;) {
        if (pos[j] >= end[j]) {
            if (--j < 2) return false;
            continue;
        }
        const uint32_t x = g.col[pos[j]++];
        if (!step_ok(g, T, img, j, drv[j], x)) continue;
        img[j] = x;
        if (j == T.k - 1) return true;
        ++j;
        drv[j] = driver(g, T, img, j, pos[j], end[j]);
    }
}

__global__ void __launch_bounds__(256) mni_kernel(MArgs a) {
    const int lane = __lane_id();
    const uint64_t total = a.prefix[a.ntasks];
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(a.head, 1u);
        it = __builtin_amdgcn_readfirstlane(it);
        if (it >= total) break;
        if (a.cancel) {
            uint32_t stop = 0;
            if (lane == 0) stop = (uint32_t)__atomic_load_n(a.cancel, __ATOMIC_RELAXED);
            if (__builtin_amdgcn_readfirstlane(stop)) break;
        }
        // the task holding item `it`: the last t with prefix[t] <= it
        uint32_t lo = 0, hi = a.ntasks;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.prefix[mid] <= it) lo = mid;
            else hi = mid;
        }
        const uint32_t t = lo;
        const MTask T = a.tasks[t];
        const uint64_t c0 = (uint64_t)T.pos_b + (it - a.prefix[t]) * (uint64_t)MNI_CHUNK;
        const uint64_t c1 = min(c0 + MNI_CHUNK, (uint64_t)T.pos_e);
        for (uint64_t p = c0; p < c1; ++p) {
            const uint32_t x = a.order ? a.order[p] : (uint32_t)p;
            if (T.label[0] >= 0 && a.g.lab[x] != (uint8_t)T.label[0]) continue;
            const uint32_t b = a.g.rp[x], e = a.g.rp[x + 1];
            bool found = false;
            for (uint32_t base = b; base < e && !found; base += 64) {
                const uint32_t q = base + lane;
                bool ok = q < e;
                uint32_t img[KMAX];
                img[0] = x;
                if (ok) {
                    const uint32_t y = a.g.col[q];
                    img[1] = y;
                    ok = T.label[1] < 0 || a.g.lab[y] == (uint8_t)T.label[1];
                    if (ok) ok = lane_complete(a.g, T, img);
                }
                found = __ballot(ok) != 0ull;
            }
            if (found && lane == 0) atomicOr(&a.dom[(uint64_t)t * a.words + (x >> 5)], 1u << (x & 31));
        }
    }
}

__global__ void __launch_bounds__(256) mni_union_kernel(const uint32_t* __restrict__ dom, uint64_t words,
                                                        const uint32_t* __restrict__ list,
                                                        const MOut* __restrict__ outs, uint32_t nout,
                                                        unsigned long long* counts) {
    for (uint32_t o = blockIdx.x; o < nout; o += gridDim.x) {
        const MOut O = outs[o];
        unsigned long long cnt = 0;
        for (uint64_t w = threadIdx.x; w < words; w += blockDim.x) {
            uint32_t v = 0;
            for (uint32_t i = 0; i < O.count; ++i) v |= dom[(uint64_t)list[O.first + i] * words + w];
            cnt += (unsigned long long)__popc(v);
        }
        for (int off = 32; off >= 1; off >>= 1) cnt += __shfl_xor(cnt, off);
        if (__lane_id() == 0 && cnt) atomicAdd(&counts[o], cnt);
    }
}

// Whether match m (images in pattern-vertex order) is the smallest of its
// images m o g under the automorphisms g.
__device__ __forceinline__ bool aut_minimal(const uint32_t* m, uint32_t k, const uint8_t* aut, uint32_t naut) {
    for (uint32_t t = 0; t < naut; ++t) {
        const uint8_t* gp = aut + (uint64_t)t * KMAX;
        for (uint32_t v = 0; v < k; ++v) {
            const uint32_t x = m[gp[v]], y = m[v];
            if (x < y) return false;
            if (x > y) break;
        }
    }
    return true;
}

__device__ __forceinline__ void list_emit(const LArgs& a, const uint8_t* st, const uint32_t* img) {
    uint32_t m[KMAX];
    for (uint32_t j = 0; j < a.k; ++j) m[st[j]] = img[j];
    if (!aut_minimal(m, a.k, a.aut, a.naut)) return;
    const unsigned long long idx = atomicAdd(a.count, 1ull);
    if (idx < a.cap)
        for (uint32_t v = 0; v < a.k; ++v) a.out[idx * a.k + v] = m[v];
}

// Every completion of a match whose steps 0 and 1 are mapped.
__device__ void lane_list(const LArgs& a, const MTask& T, const uint8_t* st, uint32_t* img) {
    const KGraph& g = a.g;
    if (T.k <= 2) {
        list_emit(a, st, img);
        return;
    }
    uint32_t pos[KMAX], end[KMAX];
    int drv[KMAX];
    int j = 2;
    drv[j] = driver(g, T, img, j, pos[j], end[j]);
    for (;;) {
        if (pos[j] >= end[j]) {
            if (--j < 2) return;
            continue;
        }
        const uint32_t x = g.col[pos[j]++];
        if (!step_ok(g, T, img, j, drv[j], x)) continue;
        img[j] = x;
        if (j == T.k - 1) {
            list_emit(a, st, img);
            continue;
        }
        ++j;
        drv[j] = driver(g, T, img, j, pos[j], end[j]);
    }
}

__global__ void __launch_bounds__(256) list_kernel(LArgs a) {
    const int lane = __lane_id();
    const uint64_t total = a.prefix[a.ntasks];
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(a.head, 1u);
        it = __builtin_amdgcn_readfirstlane(it);
        if (it >= total) break;
        uint32_t lo = 0, hi = a.ntasks;
        while (hi - lo > 1) {
            const uint32_t mid = (lo + hi) >> 1;
            if (a.prefix[mid] <= it) lo = mid;
            else hi = mid;
        }
        const uint32_t t = lo;
        const MTask T = a.tasks[t];
        const uint8_t* st = a.steps + (uint64_t)t * KMAX;
        const uint64_t c0 = (uint64_t)T.pos_b + (it - a.prefix[t]) * (uint64_t)MNI_CHUNK;
        const uint64_t c1 = min(c0 + MNI_CHUNK, (uint64_t)T.pos_e);
        for (uint64_t p = c0; p < c1; ++p) {
            const uint32_t x = a.order ? a.order[p] : (uint32_t)p;
            if (T.label[0] >= 0 && a.g.lab[x] != (uint8_t)T.label[0]) continue;
            const uint32_t b = a.g.rp[x], e = a.g.rp[x + 1];
            for (uint32_t q = b + lane; q < e; q += 64) {
                const uint32_t y = a.g.col[q];
                if (T.label[1] >= 0 && a.g.lab[y] != (uint8_t)T.label[1]) continue;
                uint32_t img[KMAX];
                img[0] = x;
                img[1] = y;
                lane_list(a, T, st, img);
            }
        }
    }
}

}  // namespace

int launch_list(const LArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(list_kernel, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mni(const MArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(mni_kernel, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_mni_union(const uint32_t* dom, uint64_t words, const uint32_t* list, const MOut* outs, uint32_t nout,
                     unsigned long long* counts, int grid, hipStream_t s) {
    if (nout == 0) return 0;
    hipLaunchKernelGGL(mni_union_kernel, dim3(grid), dim3(256), 0, s, dom, words, list, outs, nout, counts);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pm
