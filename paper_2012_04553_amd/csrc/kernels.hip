// Matching kernel for gfx950 (wave64).
//
// One wavefront takes one work item at a time from an atomic queue: a
// range of roots (vertex ids ascend with degree, so a range holds roots of
// similar degree) of one plan, or a slice of the level-1 candidates of one
// high-degree root.  Core levels are enumerated depth first.  Upper levels
// are wave-cooperative: the 64 lanes stream 64 consecutive entries of the
// shortest bounded driver list (a neighbour list, or the buffer of an
// earlier level that contains this level's candidates), each lane tests its
// entry against the other lists of the level (binary search: membership
// for pattern edges, non-membership for anti-edges), the symmetry-breaking
// bounds, injectivity and the label, and ballot + mbcnt compact the
// survivors in order into the level buffer.  The candidates of the
// second-to-last core level are then spread over the lanes: every lane
// finishes its own partial match - counting the last level, or walking it
// and evaluating the tail polynomial over leaf-set sizes - with sequential
// set operations, so one wave keeps 64 independent memory streams in flight
// on the short (degree-oriented) lists that dominate power-law graphs.
// A plan whose last core vertex is reached only through bridge leaves
// aggregates two-hop multiplicities in a per-wave dense counter array, the
// lanes scanning different bridges.
//
// Counts accumulate per lane in 128 bits, are reduced across the wave and
// added to a 128-bit global counter per plan (two 64-bit atomics with
// carry); the host divides by the plan's divisor.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

#include "kernels.hpp"

namespace pm {

typedef unsigned __int128 u128;
typedef __int128 i128;

constexpr uint32_t NOB = 0xffffffffu;  // "no upper bound"

__device__ __forceinline__ uint32_t lower_bound_u32(const uint32_t* __restrict__ a, uint32_t lo,
                                                     uint32_t hi, uint32_t x) {
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ bool in_sorted(const uint32_t* __restrict__ a, uint32_t lo, uint32_t hi,
                                          uint32_t x) {
    uint32_t p = lower_bound_u32(a, lo, hi, x);
    return p < hi && a[p] == x;
}

// Entries of N(v) within [lo, hi): the split index (first neighbour above
// v) answers the common bounds lo = v+1 and hi = v without a search.
__device__ __forceinline__ void list_range(const KGraph& g, uint32_t v, uint32_t lo, uint32_t hi,
                                           uint32_t& b, uint32_t& e) {
    const uint32_t s = g.rp[v], t = g.rp[v + 1], sp = g.split[v];
    if (lo == 0) b = s;
    else if (lo == v + 1) b = sp;
    else if (lo > v) b = lower_bound_u32(g.col, sp, t, lo);
    else b = lower_bound_u32(g.col, s, sp, lo);
    if (hi == NOB) e = t;
    else if (hi == v) e = sp;
    else if (hi > v) e = lower_bound_u32(g.col, b > sp ? b : sp, t, hi);
    else e = lower_bound_u32(g.col, b, sp, hi);
    if (e < b) e = b;
}

__device__ __forceinline__ int wave_lane() { return __lane_id(); }

__device__ __forceinline__ uint32_t bcast(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint32_t lane_prefix(uint64_t m) {
    return (uint32_t)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
}

struct Ctx {
    KGraph g;
    const DPlan* P;
    uint32_t v[KMAX];        // wave-uniform prefix of the core match
    uint32_t* buf;           // per-wave level buffers
    uint64_t stride;
    uint32_t size[KMAX];     // entries in each level buffer
    uint64_t bytes;          // algorithmic bytes (counting build only)
};

__device__ __forceinline__ void bounds_of(const uint32_t* vv, uint8_t gt, uint8_t lt, uint32_t& lo,
                                          uint32_t& hi) {
    lo = 0;
    hi = NOB;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if ((gt >> i) & 1) lo = max(lo, vv[i] + 1);
        if ((lt >> i) & 1) hi = min(hi, vv[i]);
    }
}

// Shortest bounded adjacency list among `adj` (per lane when vv differs).
__device__ __forceinline__ int pick_driver(const KGraph& g, const uint32_t* vv, uint8_t adj, uint32_t lo,
                                           uint32_t hi, uint32_t& b, uint32_t& e) {
    uint32_t best = NOB;
    int bi = 0;
    b = e = 0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if (!((adj >> i) & 1)) continue;
        uint32_t sb, se;
        list_range(g, vv[i], lo, hi, sb, se);
        if (se - sb < best) {
            best = se - sb;
            bi = i;
            b = sb;
            e = se;
        }
    }
    return bi;
}

// Per-candidate test against probe lists, injectivity and label.
struct Probe {
    uint32_t pb[KMAX], pe[KMAX];
    uint8_t adj, anti, neq;
    int8_t label;
};

__device__ __forceinline__ uint64_t make_probe(const KGraph& g, const uint32_t* vv, uint8_t adj, uint8_t anti,
                                               uint8_t neq, int8_t label, uint32_t lo, uint32_t hi,
                                               Probe& pr) {
    uint64_t bytes = 0;
    pr.adj = adj;
    pr.anti = anti;
    pr.neq = neq;
    pr.label = label;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        pr.pb[i] = pr.pe[i] = 0;
        if (((adj | anti) >> i) & 1) {
            list_range(g, vv[i], lo, hi, pr.pb[i], pr.pe[i]);
            bytes += 8 + 4ull * (pr.pe[i] - pr.pb[i]);
        }
    }
    return bytes;
}

__device__ __forceinline__ bool probe_ok(const KGraph& g, const uint32_t* vv, const Probe& pr, uint32_t x) {
    if (pr.label >= 0 && g.lab[x] != (uint8_t)pr.label) return false;
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
        if (((pr.neq >> i) & 1) && x == vv[i]) return false;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if (((pr.adj >> i) & 1) && !in_sorted(g.col, pr.pb[i], pr.pe[i], x)) return false;
        if (((pr.anti >> i) & 1) && in_sorted(g.col, pr.pb[i], pr.pe[i], x)) return false;
    }
    return true;
}

// ---------------------------------------------------------------- wave-cooperative level

// Materialise the candidates of core level j (wave-uniform prefix c.v).
template <bool BYTES>
__device__ uint32_t wave_level(Ctx& c, int j) {
    const DLevel L = c.P->lev[j];
    const int lane = wave_lane();
    uint32_t lo, hi;
    bounds_of(c.v, L.gt, L.lt, lo, hi);
    uint32_t* out = c.buf + (uint64_t)j * c.stride;
    if (lo >= hi) return 0;
    const uint32_t* drv;
    uint32_t b, e;
    uint8_t chk = L.adj, anti = L.anti;
    if (L.base != 0xff) {
        const uint32_t* bb = c.buf + (uint64_t)L.base * c.stride;
        uint32_t n = c.size[L.base];
        b = lo ? lower_bound_u32(bb, 0, n, lo) : 0;
        e = hi != NOB ? lower_bound_u32(bb, b, n, hi) : n;
        drv = bb;
        chk &= (uint8_t)~c.P->lev[L.base].adj;
        anti &= (uint8_t)~c.P->lev[L.base].anti;
    } else {
        int bi = pick_driver(c.g, c.v, L.adj, lo, hi, b, e);
        drv = c.g.col;
        chk &= (uint8_t)~(1u << bi);
        if (BYTES && lane == 0) c.bytes += 8;
    }
    Probe pr;
    uint64_t pbytes = make_probe(c.g, c.v, chk, anti, L.neq, L.label, lo, hi, pr);
    if (BYTES && lane == 0) c.bytes += pbytes + 4ull * (e - b);
    uint32_t total = 0;
    for (uint32_t base = b; base < e; base += 64) {
        uint32_t idx = base + lane;
        bool ok = idx < e;
        uint32_t x = ok ? drv[idx] : 0;
        ok = ok && probe_ok(c.g, c.v, pr, x);
        uint64_t m = __ballot(ok);
        if (ok) out[total + lane_prefix(m)] = x;
        total += (uint32_t)__popcll(m);
    }
    return total;
}

// ---------------------------------------------------------------- per-lane work

// Per-lane filter over level j (prefix vv complete below j).  MODE 0 counts;
// MODE 1 evaluates the tail for every survivor and returns it in `sum`.
template <int MODE, bool BYTES>
__device__ uint64_t lane_level(Ctx& c, uint32_t* vv, int j, u128& sum);

__device__ __forceinline__ u128 poly_eval(const DPlan* P, const uint64_t* tv) {
    i128 s = 0;
    const int nm = P->nmono;
    for (int m = 0; m < nm; ++m) {
        const DMono M = P->mono[m];
        i128 prod = (i128)M.coef;
        for (int f = 0; f < M.nf; ++f) prod *= (i128)tv[M.f[f]];
        s += prod;
    }
    return s > 0 ? (u128)s : (u128)0;
}

// One tail term for the full core match vv (per lane).
template <bool BYTES>
__device__ __forceinline__ uint64_t lane_term(Ctx& c, const uint32_t* vv, const DTerm& t, uint64_t aggm) {
    if (t.agg) return aggm;
    uint32_t lo, hi;
    bounds_of(vv, t.gt, t.lt, lo, hi);
    if (lo >= hi) return 0;
    if (t.cheap) {
        int a = __builtin_ctz((uint32_t)t.adj);
        uint32_t b, e;
        list_range(c.g, vv[a], lo, hi, b, e);
        uint64_t cnt = e - b;
#pragma unroll
        for (int i = 0; i < KMAX; ++i) {
            if (!((t.neq >> i) & 1)) continue;
            uint32_t y = vv[i];
            if (y >= lo && y < hi && (((t.sure >> i) & 1) || in_sorted(c.g.col, b, e, y))) --cnt;
        }
        if (BYTES) c.bytes += 8;
        return cnt;
    }
    uint32_t b, e;
    int bi = pick_driver(c.g, vv, t.adj, lo, hi, b, e);
    Probe pr;
    uint64_t pbytes = make_probe(c.g, vv, (uint8_t)(t.adj & ~(1u << bi)), t.anti, t.neq, t.label, lo, hi, pr);
    if (BYTES) c.bytes += 8 + pbytes + 4ull * (e - b);
    uint64_t cnt = 0;
    for (uint32_t p = b; p < e; ++p)
        if (probe_ok(c.g, vv, pr, c.g.col[p])) ++cnt;
    return cnt;
}

template <bool BYTES>
__device__ __forceinline__ u128 lane_tail(Ctx& c, const uint32_t* vv, uint64_t aggm) {
    uint64_t tv[MAX_TERMS];
    const int nt = c.P->nterm;
    for (int q = 0; q < nt; ++q) tv[q] = lane_term<BYTES>(c, vv, c.P->term[q], aggm);
    return poly_eval(c.P, tv);
}

template <int MODE, bool BYTES>
__device__ uint64_t lane_level(Ctx& c, uint32_t* vv, int j, u128& sum) {
    const DLevel L = c.P->lev[j];
    uint32_t lo, hi;
    bounds_of(vv, L.gt, L.lt, lo, hi);
    if (lo >= hi) return 0;
    const uint32_t* drv;
    uint32_t b, e;
    uint8_t chk = L.adj, anti = L.anti;
    if (L.base != 0xff) {
        const uint32_t* bb = c.buf + (uint64_t)L.base * c.stride;
        uint32_t n = c.size[L.base];
        b = lo ? lower_bound_u32(bb, 0, n, lo) : 0;
        e = hi != NOB ? lower_bound_u32(bb, b, n, hi) : n;
        drv = bb;
        chk &= (uint8_t)~c.P->lev[L.base].adj;
        anti &= (uint8_t)~c.P->lev[L.base].anti;
    } else {
        int bi = pick_driver(c.g, vv, L.adj, lo, hi, b, e);
        drv = c.g.col;
        chk &= (uint8_t)~(1u << bi);
        if (BYTES) c.bytes += 8;
    }
    Probe pr;
    uint64_t pbytes = make_probe(c.g, vv, chk, anti, L.neq, L.label, lo, hi, pr);
    if (BYTES) c.bytes += pbytes + 4ull * (e - b);
    uint64_t cnt = 0;
    for (uint32_t p = b; p < e; ++p) {
        uint32_t x = drv[p];
        if (!probe_ok(c.g, vv, pr, x)) continue;
        if (MODE == 0) {
            ++cnt;
        } else {
            vv[j] = x;
            sum += lane_tail<BYTES>(c, vv, 0);
        }
    }
    return cnt;
}

// ---------------------------------------------------------------- aggregation

// Two-hop aggregation for the last core level j: targets x reached from
// bridges y in N(v_src) (bridge bounds and label) are counted in a per-wave
// dense array; every touched target is then evaluated lane-parallel with
// its multiplicity as the bridge term.
template <bool BYTES>
__device__ void agg_level(Ctx& c, int j, uint32_t wid, uint32_t* s_touch, const KArgs& a, u128& acc) {
    const DPlan* P = c.P;
    const DLevel L = P->lev[j];
    const int lane = wave_lane();
    uint32_t* cnt = a.aggcnt + (uint64_t)wid * c.g.n;
    uint32_t* touched = a.aggtouch + (uint64_t)wid * c.g.n;
    uint32_t blo, bhi, lo, hi;
    bounds_of(c.v, P->bridge_gt, P->bridge_lt, blo, bhi);
    bounds_of(c.v, L.gt, L.lt, lo, hi);
    if (blo >= bhi || lo >= hi) return;
    uint32_t bb, be;
    list_range(c.g, c.v[P->bridge_src], blo, bhi, bb, be);
    if (BYTES && lane == 0) c.bytes += 8 + 4ull * (be - bb);
    if (lane == 0) *s_touch = 0;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t base = bb; base < be; base += 64) {
        uint32_t idx = base + lane;
        if (idx >= be) continue;
        uint32_t y = c.g.col[idx];
        if (P->bridge_label >= 0 && c.g.lab[y] != (uint8_t)P->bridge_label) continue;
        bool core = false;
        for (int i = 0; i < j; ++i) core |= (y == c.v[i]);
        if (core) continue;
        uint32_t yb, yf;
        list_range(c.g, y, lo, hi, yb, yf);
        if (BYTES) c.bytes += 8 + 4ull * (yf - yb);
        for (uint32_t p = yb; p < yf; ++p) {
            uint32_t x = c.g.col[p];
            if (L.label >= 0 && c.g.lab[x] != (uint8_t)L.label) continue;
            bool skip = false;
#pragma unroll
            for (int i = 0; i < KMAX; ++i)
                if (((L.neq >> i) & 1) && x == c.v[i]) skip = true;
            if (skip) continue;
            if (atomicAdd(&cnt[x], 1u) == 0u) touched[atomicAdd(s_touch, 1u)] = x;
        }
    }
    __builtin_amdgcn_wave_barrier();
    __threadfence_block();
    const uint32_t ntouch = bcast(*(volatile uint32_t*)s_touch);
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
            acc += lane_tail<BYTES>(c, vv, m);
        }
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- bitmap cliques

// Cliques with a total order live in the out-neighbourhood C of the root:
// lanes build one bitmap row per member x of C (bit j set when C[j] is an
// out-neighbour of x, by a merge of the two sorted lists), then count the
// deeper levels with word-wise AND and popcount over the rows.
template <bool BYTES>
__device__ void local_clique(Ctx& c, uint32_t s0, uint32_t s1, u128& acc) {
    const int lane = wave_lane();
    const int nc = c.P->ncore;
    const uint32_t v0 = c.v[0];
    const uint32_t b = c.g.split[v0], e = c.g.rp[v0 + 1];
    const uint32_t s = e - b;
    if (BYTES && lane == 0) c.bytes += 8 + 4ull * s;
    if (s < (uint32_t)(nc - 1) || s0 >= s) return;
    const uint32_t W = (s + 63) >> 6;
    uint64_t* rows = (uint64_t*)c.buf;
    const uint32_t* C1 = c.g.col + b;
    for (uint32_t i = lane; i < s; i += 64) {
        const uint32_t x = C1[i];
        uint32_t p = c.g.split[x];
        const uint32_t pe = c.g.rp[x + 1];
        if (BYTES) c.bytes += 8 + 4ull * (pe - p) + 4ull * (s - i - 1);
        uint64_t* row = rows + (uint64_t)i * W;
        uint32_t q = i + 1;
        uint32_t cw = q >> 6;
        for (uint32_t w = 0; w < cw && w < W; ++w) row[w] = 0;
        uint64_t bits = 0;
        while (q < s && p < pe) {
            const uint32_t a = C1[q], y = c.g.col[p];
            if (a == y) bits |= 1ull << (q & 63);
            if (y <= a) ++p;
            if (a <= y) {
                ++q;
                if ((q >> 6) != cw) {
                    row[cw] = bits;
                    bits = 0;
                    ++cw;
                }
            }
        }
        if (cw < W) row[cw++] = bits;
        for (; cw < W; ++cw) row[cw] = 0;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    const uint32_t ie = min(s, s1);
    for (uint32_t i = s0 + lane; i < ie; i += 64) {
        const uint64_t* ri = rows + (uint64_t)i * W;
        uint64_t cnt = 0;
        if (nc == 3) {
            for (uint32_t w = 0; w < W; ++w) cnt += __popcll(ri[w]);
        } else {
            for (uint32_t w = 0; w < W; ++w) {
                uint64_t m = ri[w];
                while (m) {
                    const uint32_t j = (w << 6) + __builtin_ctzll(m);
                    m &= m - 1;
                    const uint64_t* rj = rows + (uint64_t)j * W;
                    if (nc == 4) {
                        for (uint32_t w2 = j >> 6; w2 < W; ++w2) cnt += __popcll(ri[w2] & rj[w2]);
                    } else {
                        for (uint32_t w2 = j >> 6; w2 < W; ++w2) {
                            uint64_t t = ri[w2] & rj[w2];
                            while (t) {
                                const uint32_t k = (w2 << 6) + __builtin_ctzll(t);
                                t &= t - 1;
                                const uint64_t* rk = rows + (uint64_t)k * W;
                                for (uint32_t w3 = k >> 6; w3 < W; ++w3) cnt += __popcll(ri[w3] & rj[w3] & rk[w3]);
                            }
                        }
                    }
                }
            }
        }
        acc += (u128)cnt;
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------- flush

__device__ __forceinline__ void flush(const KArgs& a, int plan, u128 acc) {
    uint64_t lo = (uint64_t)acc, hi = (uint64_t)(acc >> 64);
    // wave-wide 128-bit sum as four 32-bit limbs carried in 64 bits
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

// ---------------------------------------------------------------- kernel

// Lanes take the entries [b, e) of the level-j buffer as v_j and finish
// the match (j = ncore - 2).
template <bool BYTES>
__device__ __forceinline__ void lanes_finish(Ctx& c, int j, uint32_t b, uint32_t e, u128& acc) {
    const DPlan* P = c.P;
    const int lane = wave_lane();
    const int last = P->ncore - 1;
    const uint32_t* bj = c.buf + (uint64_t)j * c.stride;
    for (uint32_t base = b; base < e; base += 64) {
        uint32_t idx = base + lane;
        if (idx >= e) continue;
        uint32_t vv[KMAX];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) vv[i] = c.v[i];
        vv[j] = bj[idx];
        if (P->nterm == 0) {
            u128 dummy = 0;
            acc += (u128)lane_level<0, BYTES>(c, vv, last, dummy) * (u128)(uint32_t)P->mult;
        } else {
            lane_level<1, BYTES>(c, vv, last, acc);
        }
    }
}

// Cancellation: the host sets a coherent flag; lane 0 reads it every 16th
// call (root or level-1 step), so an abandoned item ends within a few of its
// iterations.  Wave-uniform.
__device__ __forceinline__ bool should_stop(const KArgs& a, uint32_t& tick) {
    if (!a.cancel || ((++tick) & 15u)) return false;
    uint32_t stop = 0;
    if (wave_lane() == 0) stop = (uint32_t)__atomic_load_n(a.cancel, __ATOMIC_RELAXED);
    return bcast(stop) != 0;
}

template <bool BYTES>
__global__ void __launch_bounds__(256) match_kernel(KArgs a) {
    __shared__ uint32_t s_touch[4];
    const int lane = wave_lane();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    uint32_t* my_touch = &s_touch[threadIdx.x >> 6];
    Ctx c;
    c.g = a.g;
    c.stride = a.buf_stride;
    c.buf = a.scratch + (uint64_t)wid * (uint64_t)KMAX * a.buf_stride;
    c.bytes = 0;
    int cur = -1;
    u128 acc = 0;
    uint32_t tick = 0;
    bool stopped = false;
    const uint64_t total = (uint64_t)a.nplans * a.nitems;
    for (;;) {
        if (stopped) break;
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(a.head, 1u);
        it = bcast(it);
        if (it >= total) break;
        if (a.cancel) {
            // host-visible flag: one read per work item, by one lane
            uint32_t stop = 0;
            if (lane == 0) stop = (uint32_t)__atomic_load_n(a.cancel, __ATOMIC_RELAXED);
            if (bcast(stop)) break;
        }
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
            // lanes take roots; every tail term is evaluated per lane
            if (item.s0 != 0 || P->nterm == 0) continue;
            for (uint32_t base = item.r0; base < item.r1; base += 64) {
                uint32_t r = base + lane;
                if (r < item.r1 && (rl < 0 || a.g.lab[r] == (uint8_t)rl)) {
                    uint32_t vv[KMAX] = {r, 0, 0, 0, 0};
                    acc += lane_tail<BYTES>(c, vv, 0);
                }
            }
            continue;
        }
        for (uint32_t r = item.r0; r < item.r1; ++r) {
            if (stopped || should_stop(a, tick)) {
                stopped = true;
                break;
            }
            if (rl >= 0 && a.g.lab[r] != (uint8_t)rl) continue;
            c.v[0] = r;
            if (P->local) {
                local_clique<BYTES>(c, item.s0, item.s1, acc);
                continue;
            }
            if (nc == 2) {
                if (P->agg_last) {
                    if (item.s0 == 0) agg_level<BYTES>(c, 1, wid, my_touch, a, acc);
                    continue;
                }
                uint32_t n = wave_level<BYTES>(c, 1);
                uint32_t b = min(item.s0, n), e = min(item.s1, n);
                if (P->nterm == 0) {
                    if (lane == 0 && e > b) acc += (u128)(e - b) * (u128)(uint32_t)P->mult;
                    continue;
                }
                const uint32_t* b1 = c.buf + c.stride;
                for (uint32_t base = b; base < e; base += 64) {
                    uint32_t idx = base + lane;
                    if (idx >= e) continue;
                    uint32_t vv[KMAX] = {r, b1[idx], 0, 0, 0};
                    acc += lane_tail<BYTES>(c, vv, 0);
                }
                continue;
            }
            // nc >= 3: levels 1 .. nc-2 materialised, lanes finish
            const int pen = nc - 2;
            uint32_t pos[KMAX], end[KMAX];
            c.size[1] = wave_level<BYTES>(c, 1);
            pos[1] = min(item.s0, c.size[1]);
            end[1] = min(item.s1, c.size[1]);
            if (pen == 1) {
                if (P->agg_last) {
                    for (uint32_t q = pos[1]; q < end[1]; ++q) {
                        if (should_stop(a, tick)) {
                            stopped = true;
                            break;
                        }
                        c.v[1] = c.buf[c.stride + q];
                        agg_level<BYTES>(c, 2, wid, my_touch, a, acc);
                    }
                } else {
                    lanes_finish<BYTES>(c, 1, pos[1], end[1], acc);
                }
                continue;
            }
            int j = 1;
            while (j >= 1) {
                if (pos[j] >= end[j]) {
                    --j;
                    continue;
                }
                if (j == 1 && should_stop(a, tick)) {
                    stopped = true;
                    break;
                }
                c.v[j] = c.buf[(uint64_t)j * c.stride + pos[j]];
                ++pos[j];
                ++j;
                c.size[j] = wave_level<BYTES>(c, j);
                if (j == pen) {
                    if (P->agg_last) {
                        for (uint32_t q = 0; q < c.size[j]; ++q) {
                            c.v[j] = c.buf[(uint64_t)j * c.stride + q];
                            agg_level<BYTES>(c, j + 1, wid, my_touch, a, acc);
                        }
                    } else {
                        lanes_finish<BYTES>(c, j, 0, c.size[j], acc);
                    }
                    --j;
                    continue;
                }
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

__global__ void zero_kernel(uint32_t* p, uint64_t words) {
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = 0u;
}

int launch_zero(uint32_t* p, uint64_t words, hipStream_t s) {
    int grid = (int)std::min<uint64_t>(1024, (words + 255) / 256);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(256), 0, s, p, words);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_match(const KArgs& a, int grid, int block, bool count_bytes, hipStream_t s) {
    if (count_bytes)
        hipLaunchKernelGGL(match_kernel<true>, dim3(grid), dim3(block), 0, s, a);
    else
        hipLaunchKernelGGL(match_kernel<false>, dim3(grid), dim3(block), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pm
