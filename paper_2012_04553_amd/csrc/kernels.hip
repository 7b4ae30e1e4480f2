// Matching kernels for gfx950 (wave64).
//
// One wavefront works on one work item at a time, taken from an atomic
// queue: a range of roots (vertices in degree order) of one plan, or a
// slice of the level-1 candidates of a single high-degree root.  From a
// root the wave extends partial matches level by level (the core of the
// plan).  The candidates of a level are produced cooperatively: the 64
// lanes stream 64 consecutive entries of the shortest bounded driver list
// (a neighbour list, or an earlier level's candidate buffer that contains
// this level's), each lane tests its entry against the other neighbour
// lists of the level (binary search: membership for edges, non-membership
// for anti-edges), against the symmetry-breaking bounds, injectivity and the
// label, and a ballot + popcount either counts the survivors or compacts
// them in order into the level buffer.  At a full core match the tail
// polynomial over set sizes gives the number of injective leaf extensions
// (see the plan compiler); when every tail term is a plain range count the
// lanes evaluate it for 64 last-level candidates in parallel.  A plan whose
// last core vertex is reached only through bridge leaves aggregates
// two-hop multiplicities in a per-wave dense counter array.
//
// Counts accumulate per lane in 128 bits, are reduced across the wave and
// added to a 128-bit global counter per plan (two 64-bit atomics with
// carry); the host divides by the plan's divisor.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.hpp"

namespace pm {

typedef unsigned __int128 u128;
typedef __int128 i128;

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* __restrict__ a, uint32_t lo,
                                                     uint32_t hi, uint32_t x) {
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool contains(const uint32_t* __restrict__ col, uint32_t lo, uint32_t hi,
                                         uint32_t x) {
    uint32_t p = lower_bound_u32(col, lo, hi, x);
    return p < hi && col[p] == x;
}

__device__ __forceinline__ int wave_lane() { return __lane_id(); }

__device__ __forceinline__ uint32_t bcast(uint32_t x) {
    return __builtin_amdgcn_readfirstlane(x);
}

struct Ctx {
    const KArgs* a;
    const DPlan* P;
    uint32_t v[KMAX];       // core vertices matched so far (wave-uniform)
    uint32_t* buf;          // per-wave level buffers
    uint64_t stride;
    uint32_t size[KMAX];    // candidates per level buffer
    uint64_t bytes;         // algorithmic bytes (when counting)
};

// Bounds [lo, hi) implied by gt/lt masks over the matched core vertices.
__device__ __forceinline__ void bounds_of(const Ctx& c, uint8_t gt, uint8_t lt, uint32_t& lo,
                                          uint32_t& hi) {
    lo = 0;
    hi = 0xffffffffu;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if ((gt >> i) & 1) lo = max(lo, c.v[i] + 1);
        if ((lt >> i) & 1) hi = min(hi, c.v[i]);
    }
}

// Generic filter over a driver range.  MODE 0: count, 1: compact into out.
// Returns the number of survivors (wave-uniform).
template <int MODE, bool BYTES>
__device__ uint32_t filter_range(Ctx& c, const uint32_t* __restrict__ drv, uint32_t b, uint32_t e,
                                 uint8_t chk_adj, uint8_t anti, uint8_t neq, int8_t label,
                                 uint32_t lo, uint32_t hi, uint32_t* __restrict__ out) {
    const uint32_t* __restrict__ rp = c.a->g.rp;
    const uint32_t* __restrict__ col = c.a->g.col;
    const uint8_t* __restrict__ lab = c.a->g.lab;
    const int lane = wave_lane();
    // neighbour-list ranges of the lists to probe, restricted to [lo, hi)
    uint32_t pb[KMAX], pe[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        pb[i] = pe[i] = 0;
        if (((chk_adj | anti) >> i) & 1) {
            uint32_t s = rp[c.v[i]], t = rp[c.v[i] + 1];
            pb[i] = lo ? lower_bound_u32(col, s, t, lo) : s;
            pe[i] = hi != 0xffffffffu ? lower_bound_u32(col, pb[i], t, hi) : t;
            if (BYTES) c.bytes += 8 + 4ull * (pe[i] - pb[i]);
        }
    }
    if (BYTES) c.bytes += 4ull * (e - b);
    uint32_t total = 0;
    for (uint32_t base = b; base < e; base += 64) {
        uint32_t idx = base + lane;
        bool ok = idx < e;
        uint32_t x = ok ? drv[idx] : 0;
        if (ok && label >= 0) ok = lab[x] == (uint8_t)label;
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (ok && ((neq >> i) & 1)) ok = x != c.v[i];
        }
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (ok && ((chk_adj >> i) & 1)) ok = contains(col, pb[i], pe[i], x);
            if (ok && ((anti >> i) & 1)) ok = !contains(col, pb[i], pe[i], x);
        }
        uint64_t m = __ballot(ok);
        if (MODE == 1) {
            uint32_t pos = total + (uint32_t)__builtin_amdgcn_mbcnt_hi(
                                       (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
            if (ok) out[pos] = x;
        }
        total += (uint32_t)__popcll(m);
    }
    return total;
}

// Candidate set of core level j (MODE 1 compacts into the level buffer).
template <int MODE, bool BYTES>
__device__ uint32_t level_set(Ctx& c, int j) {
    const DLevel L = c.P->lev[j];
    const uint32_t* __restrict__ rp = c.a->g.rp;
    const uint32_t* __restrict__ col = c.a->g.col;
    uint32_t lo, hi;
    bounds_of(c, L.gt, L.lt, lo, hi);
    uint32_t* out = c.buf + (uint64_t)j * c.stride;
    if (lo >= hi) return 0;
    const uint32_t* drv;
    uint32_t b, e;
    uint8_t chk = L.adj;
    if (L.base != 0xff) {
        const uint32_t* bb = c.buf + (uint64_t)L.base * c.stride;
        uint32_t n = c.size[L.base];
        b = lo ? lower_bound_u32(bb, 0, n, lo) : 0;
        e = hi != 0xffffffffu ? lower_bound_u32(bb, b, n, hi) : n;
        drv = bb;
        chk &= (uint8_t)~c.P->lev[L.base].adj;
    } else {
        // shortest bounded adjacency list drives
        uint32_t best = 0xffffffffu;
        int bi = 0;
        b = e = 0;
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (!((L.adj >> i) & 1)) continue;
            uint32_t s = rp[c.v[i]], t = rp[c.v[i] + 1];
            uint32_t sb = lo ? lower_bound_u32(col, s, t, lo) : s;
            uint32_t se = hi != 0xffffffffu ? lower_bound_u32(col, sb, t, hi) : t;
            if (se - sb < best) {
                best = se - sb;
                bi = i;
                b = sb;
                e = se;
            }
        }
        drv = col;
        chk &= (uint8_t)~(1u << bi);
        if (BYTES) c.bytes += 8;
    }
    uint8_t anti = L.anti;
    if (L.base != 0xff) anti &= (uint8_t)~c.P->lev[L.base].anti;
    return filter_range<MODE, BYTES>(c, drv, b, e, chk, anti, L.neq, L.label, lo, hi, out);
}

// ---- tail terms --------------------------------------------------------

// Range count for a cheap term: |N(v_a) within bounds| minus matched core
// vertices that lie in that range (injectivity).  Per lane, v_last given.
__device__ __forceinline__ uint64_t cheap_term(const Ctx& c, const DTerm& t, const uint32_t* vv) {
    const uint32_t* __restrict__ rp = c.a->g.rp;
    const uint32_t* __restrict__ col = c.a->g.col;
    uint32_t lo = 0, hi = 0xffffffffu;
    int a = 0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if ((t.gt >> i) & 1) lo = max(lo, vv[i] + 1);
        if ((t.lt >> i) & 1) hi = min(hi, vv[i]);
        if ((t.adj >> i) & 1) a = i;
    }
    if (lo >= hi) return 0;
    uint32_t s = rp[vv[a]], e = rp[vv[a] + 1];
    uint32_t b = lo ? lower_bound_u32(col, s, e, lo) : s;
    uint32_t f = hi != 0xffffffffu ? lower_bound_u32(col, b, e, hi) : e;
    uint64_t cnt = f - b;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if (!((t.neq >> i) & 1)) continue;
        uint32_t y = vv[i];
        if (y >= lo && y < hi && contains(col, b, f, y)) --cnt;
    }
    return cnt;
}

__device__ __forceinline__ u128 poly_eval(const DPlan* P, const uint64_t* tv) {
    i128 s = 0;
    for (int m = 0; m < P->nmono; ++m) {
        const DMono M = P->mono[m];
        i128 prod = (i128)M.coef;
        for (int f = 0; f < M.nf; ++f) prod *= (i128)tv[M.f[f]];
        s += prod;
    }
    return s > 0 ? (u128)s : (u128)0;
}

// Lane-parallel tail: all terms cheap (or the aggregation multiplicity).
template <bool BYTES>
__device__ __forceinline__ u128 tail_lane(Ctx& c, const uint32_t* vv, uint64_t aggm) {
    uint64_t tv[MAX_TERMS];
    const int nt = c.P->nterm;
    for (int q = 0; q < nt; ++q) {
        const DTerm t = c.P->term[q];
        tv[q] = t.agg ? aggm : cheap_term(c, t, vv);
        if (BYTES && !t.agg) c.bytes += 8;
    }
    return poly_eval(c.P, tv);
}

// Wave-cooperative tail for one full core match (c.v complete).
template <bool BYTES>
__device__ u128 tail_wave(Ctx& c) {
    uint64_t tv[MAX_TERMS];
    const uint32_t* __restrict__ rp = c.a->g.rp;
    const uint32_t* __restrict__ col = c.a->g.col;
    const int nt = c.P->nterm;
    for (int q = 0; q < nt; ++q) {
        const DTerm t = c.P->term[q];
        if (t.cheap) {
            tv[q] = cheap_term(c, t, c.v);
            if (BYTES) c.bytes += 8;
            continue;
        }
        uint32_t lo, hi;
        bounds_of(c, t.gt, t.lt, lo, hi);
        if (lo >= hi) {
            tv[q] = 0;
            continue;
        }
        uint32_t best = 0xffffffffu, b = 0, e = 0;
        int bi = 0;
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (!((t.adj >> i) & 1)) continue;
            uint32_t s = rp[c.v[i]], f = rp[c.v[i] + 1];
            uint32_t sb = lo ? lower_bound_u32(col, s, f, lo) : s;
            uint32_t se = hi != 0xffffffffu ? lower_bound_u32(col, sb, f, hi) : f;
            if (se - sb < best) {
                best = se - sb;
                bi = i;
                b = sb;
                e = se;
            }
        }
        if (BYTES) c.bytes += 8;
        tv[q] = filter_range<0, BYTES>(c, col, b, e, (uint8_t)(t.adj & ~(1u << bi)), t.anti, t.neq,
                                        t.label, lo, hi, nullptr);
    }
    return poly_eval(c.P, tv);
}

// ---- last core level ---------------------------------------------------

template <bool BYTES>
__device__ void last_level(Ctx& c, int j, uint32_t s0, uint32_t s1, u128& acc) {
    const DPlan* P = c.P;
    const int lane = wave_lane();
    if (P->nterm == 0) {
        if (P->mult == 0) return;
        uint32_t n;
        if (j == 1 && (s0 != 0 || s1 != 0xffffffffu)) {
            n = level_set<1, BYTES>(c, j);
            uint32_t e = min(s1, n);
            n = e > s0 ? e - s0 : 0;
        } else {
            n = level_set<0, BYTES>(c, j);
        }
        if (lane == 0) acc += (u128)n * (u128)(uint32_t)P->mult;
        return;
    }
    uint32_t n = level_set<1, BYTES>(c, j);
    const uint32_t* bj = c.buf + (uint64_t)j * c.stride;
    uint32_t b = 0, e = n;
    if (j == 1) {
        b = min(s0, n);
        e = min(s1, n);
    }
    if (P->lane_par) {
        uint32_t vv[KMAX];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) vv[i] = c.v[i];
        for (uint32_t base = b; base < e; base += 64) {
            uint32_t idx = base + lane;
            if (idx < e) {
                vv[j] = bj[idx];
                acc += tail_lane<BYTES>(c, vv, 0);
            }
        }
    } else {
        for (uint32_t idx = b; idx < e; ++idx) {
            c.v[j] = bj[idx];
            u128 r = tail_wave<BYTES>(c);
            if (lane == 0) acc += r;
        }
    }
}

// Two-hop aggregation for the last core level j: targets x reached from
// bridges y in N(v_src) (bridge bounds and label), counted in a per-wave
// dense array; then every touched target is evaluated lane-parallel with
// its multiplicity.
template <bool BYTES>
__device__ void agg_level(Ctx& c, int j, uint32_t wid, u128& acc) {
    const DPlan* P = c.P;
    const DLevel L = P->lev[j];
    const uint32_t* __restrict__ rp = c.a->g.rp;
    const uint32_t* __restrict__ col = c.a->g.col;
    const uint8_t* __restrict__ lab = c.a->g.lab;
    const int lane = wave_lane();
    uint32_t* cnt = c.a->aggcnt + (uint64_t)wid * c.a->g.n;
    uint32_t* touched = c.a->aggtouch + (uint64_t)wid * c.a->g.n;
    uint32_t blo, bhi;
    bounds_of(c, P->bridge_gt, P->bridge_lt, blo, bhi);
    uint32_t lo, hi;
    bounds_of(c, L.gt, L.lt, lo, hi);
    if (blo >= bhi || lo >= hi) return;
    const uint32_t src = c.v[P->bridge_src];
    uint32_t s = rp[src], t = rp[src + 1];
    uint32_t bb = blo ? lower_bound_u32(col, s, t, blo) : s;
    uint32_t be = bhi != 0xffffffffu ? lower_bound_u32(col, bb, t, bhi) : t;
    if (BYTES) c.bytes += 8 + 4ull * (be - bb);
    uint32_t ntouch = 0;
    for (uint32_t p = bb; p < be; ++p) {
        uint32_t y = col[p];
        if (P->bridge_label >= 0 && lab[y] != (uint8_t)P->bridge_label) continue;
        bool core = false;
        for (int i = 0; i < j; ++i) core |= (y == c.v[i]);
        if (core) continue;
        uint32_t ys = rp[y], ye = rp[y + 1];
        uint32_t yb = lo ? lower_bound_u32(col, ys, ye, lo) : ys;
        uint32_t yf = hi != 0xffffffffu ? lower_bound_u32(col, yb, ye, hi) : ye;
        if (BYTES) c.bytes += 8 + 4ull * (yf - yb);
        for (uint32_t base = yb; base < yf; base += 64) {
            uint32_t idx = base + lane;
            bool ok = idx < yf;
            uint32_t x = ok ? col[idx] : 0;
            if (ok && L.label >= 0) ok = lab[x] == (uint8_t)L.label;
#pragma unroll
            for (int i = 0; i < KMAX; ++i)
                if (ok && ((L.neq >> i) & 1)) ok = x != c.v[i];
            bool fresh = false;
            if (ok) fresh = atomicAdd(&cnt[x], 1u) == 0u;
            uint64_t m = __ballot(fresh);
            uint32_t pos = ntouch + (uint32_t)__builtin_amdgcn_mbcnt_hi(
                                        (uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
            if (fresh) touched[pos] = x;
            ntouch += (uint32_t)__popcll(m);
        }
    }
    __threadfence_block();
    uint32_t vv[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) vv[i] = c.v[i];
    for (uint32_t base = 0; base < ntouch; base += 64) {
        uint32_t idx = base + lane;
        if (idx < ntouch) {
            uint32_t x = touched[idx];
            uint32_t m = cnt[x];
            cnt[x] = 0;
            vv[j] = x;
            acc += tail_lane<BYTES>(c, vv, m);
        }
    }
    __threadfence_block();
}

// ---- wave reduction and flush -------------------------------------------

__device__ __forceinline__ void flush(const KArgs& a, int plan, u128 acc) {
    uint64_t lo = (uint64_t)acc, hi = (uint64_t)(acc >> 64);
    // wave-wide 128-bit sum: reduce as four 32-bit limbs carried in 64 bits
    uint64_t l0 = lo & 0xffffffffu, l1 = lo >> 32, l2 = hi & 0xffffffffu, l3 = hi >> 32;
    for (int off = 32; off >= 1; off >>= 1) {
        l0 += __shfl_xor(l0, off);
        l1 += __shfl_xor(l1, off);
        l2 += __shfl_xor(l2, off);
        l3 += __shfl_xor(l3, off);
    }
    if (wave_lane() == 0) {
        l1 += l0 >> 32;
        l2 += l1 >> 32;
        l3 += l2 >> 32;
        uint64_t rlo = (l0 & 0xffffffffu) | (l1 << 32);
        uint64_t rhi = (l2 & 0xffffffffu) | (l3 << 32);
        if (rlo | rhi) {
            unsigned long long* ctr = (unsigned long long*)(a.counters + 2 * plan);
            unsigned long long old = atomicAdd(&ctr[0], (unsigned long long)rlo);
            unsigned long long carry = (old + rlo < old) ? 1ull : 0ull;
            if (rhi + carry) atomicAdd(&ctr[1], (unsigned long long)(rhi + carry));
        }
    }
}

template <bool BYTES>
__global__ void __launch_bounds__(256) match_kernel(KArgs a) {
    const int lane = wave_lane();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    Ctx c;
    c.a = &a;
    c.stride = a.buf_stride;
    c.buf = a.scratch + (uint64_t)wid * (uint64_t)KMAX * a.buf_stride;
    c.bytes = 0;
    int cur = -1;
    u128 acc = 0;
    const uint64_t total = (uint64_t)a.nplans * a.nitems;
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(a.head, 1u);
        it = bcast(it);
        if (it >= total) break;
        if (a.cancel && *(volatile int*)a.cancel) break;
        const int pi = (int)(it / a.nitems);
        const KItem item = a.items[it % a.nitems];
        if (pi != cur) {
            if (cur >= 0) flush(a, cur, acc);
            acc = 0;
            cur = pi;
        }
        const DPlan* P = a.plans + pi;
        c.P = P;
        const int nc = P->ncore;
        const int8_t rl = P->lev[0].label;
        if (nc == 1) {
            if (item.s0 != 0) continue;
            if (P->nterm == 0) {
                // single-vertex pattern: unsupported by the planner (k >= 2)
                continue;
            }
            if (P->lane_par) {
                for (uint32_t base = item.r0; base < item.r1; base += 64) {
                    uint32_t r = base + lane;
                    if (r < item.r1 && (rl < 0 || a.g.lab[r] == (uint8_t)rl)) {
                        uint32_t vv[KMAX] = {r, 0, 0, 0, 0};
                        acc += tail_lane<BYTES>(c, vv, 0);
                    }
                }
            } else {
                for (uint32_t r = item.r0; r < item.r1; ++r) {
                    if (rl >= 0 && a.g.lab[r] != (uint8_t)rl) continue;
                    c.v[0] = r;
                    u128 t = tail_wave<BYTES>(c);
                    if (lane == 0) acc += t;
                }
            }
            continue;
        }
        for (uint32_t r = item.r0; r < item.r1; ++r) {
            if (rl >= 0 && a.g.lab[r] != (uint8_t)rl) continue;
            c.v[0] = r;
            if (nc == 2) {
                if (P->agg_last) {
                    if (item.s0 == 0) agg_level<BYTES>(c, 1, wid, acc);
                } else {
                    last_level<BYTES>(c, 1, item.s0, item.s1, acc);
                }
                continue;
            }
            // levels 1 .. nc-2 enumerated, level nc-1 handled by last_level
            uint32_t pos[KMAX], end[KMAX];
            int j = 1;
            c.size[1] = level_set<1, BYTES>(c, 1);
            pos[1] = min(item.s0, c.size[1]);
            end[1] = min(item.s1, c.size[1]);
            while (j >= 1) {
                if (pos[j] >= end[j]) {
                    --j;
                    continue;
                }
                c.v[j] = c.buf[(uint64_t)j * c.stride + pos[j]];
                ++pos[j];
                if (j + 1 == nc - 1) {
                    if (P->agg_last) agg_level<BYTES>(c, j + 1, wid, acc);
                    else last_level<BYTES>(c, j + 1, 0, 0xffffffffu, acc);
                    continue;
                }
                ++j;
                c.size[j] = level_set<1, BYTES>(c, j);
                pos[j] = 0;
                end[j] = c.size[j];
            }
        }
    }
    if (cur >= 0) flush(a, cur, acc);
    if (BYTES) {
        unsigned long long bsum = c.bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (lane == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

int launch_match(const KArgs& a, int grid, int block, bool count_bytes, hipStream_t s) {
    if (count_bytes)
        hipLaunchKernelGGL(match_kernel<true>, dim3(grid), dim3(block), 0, s, a);
    else
        hipLaunchKernelGGL(match_kernel<false>, dim3(grid), dim3(block), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pm
