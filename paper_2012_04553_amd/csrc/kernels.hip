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
// survivors in order into the level buffer.
//
// The candidates of the second-to-last core level are then spread over the
// lanes, one partial match per lane.  Everything a lane still has to do for
// its match - the last level, the set-size terms of the leaves, the bridge
// lists of a two-hop level - is a set of driver ranges, one per lane, of
// very different lengths on power-law graphs.  These are processed
// flattened: a wave prefix sum over the range lengths numbers all entries
// of all lanes, every lane takes the next unprocessed entry in that order
// (so a long range is streamed by the whole wave, coalesced) and fetches
// the owning lane's match and probe with cross-lane reads; per-owner counts
// come back through ballot masks over each owner's stretch of entries.
//
// Membership in the root's list N(v0), which every partial match of a root
// shares, can use a per-wave bitmap of N(v0) (built once per root by plain
// stores, one writer per word) instead of a binary search.
//
// A plan whose last core vertex is reached only through bridge leaves
// aggregates two-hop multiplicities in a per-wave dense counter array.
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

// Graph arrays, level buffers and bitmaps live in global memory.  Device
// code reaches them through pointers typed with the global address space, so
// loads compile as global (not flat) accesses even inside functions that
// receive the matching context by reference: a flat load also counts against
// the LDS wait counter, which would make every LDS or cross-lane wait drain
// the wave's outstanding memory loads.
#define PM_GLOBAL __attribute__((address_space(1)))
template <class T> using gcp = const PM_GLOBAL T*;
template <class T> using gp = PM_GLOBAL T*;

struct DGraph {
    gcp<uint32_t> rp, col, split;
    gcp<uint8_t> lab;
    uint32_t n;
    gcp<uint32_t> hubbm;
    uint32_t hub0, hub_words;
};

// Copy of a plan record (plain words) out of global memory.
template <class T>
__device__ __forceinline__ T gload(const PM_GLOBAL T* p) {
    static_assert(sizeof(T) % 4 == 0, "plan records are whole words");
    T out;
    uint32_t* o = (uint32_t*)&out;
    const PM_GLOBAL uint32_t* w = (const PM_GLOBAL uint32_t*)p;
#pragma unroll
    for (uint32_t i = 0; i < sizeof(T) / 4; ++i) o[i] = w[i];
    return out;
}

__device__ __forceinline__ DGraph dgraph(const KGraph& g) {
    return DGraph{(gcp<uint32_t>)g.rp, (gcp<uint32_t>)g.col,   (gcp<uint32_t>)g.split,
                  (gcp<uint8_t>)g.lab, g.n, (gcp<uint32_t>)g.hubbm, g.hub0, g.hub_words};
}

template <class P>
__device__ __forceinline__ uint32_t lower_bound_u32(P a, uint32_t lo, uint32_t hi, uint32_t x) {
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// First position in a[lo, hi) holding a value >= x, searching outward from
// lo (cheap when the answer is near lo).
template <class P>
__device__ __forceinline__ uint32_t gallop_u32(P a, uint32_t lo, uint32_t hi, uint32_t x) {
    uint32_t step = 1, b = lo;
    while (b < hi && a[b] < x) {
        lo = b + 1;
        b = lo + step;
        step <<= 1;
    }
    return lower_bound_u32(a, lo, b < hi ? b : hi, x);
}

template <class P>
__device__ __forceinline__ bool in_sorted(P a, uint32_t lo, uint32_t hi, uint32_t x) {
    uint32_t p = lower_bound_u32(a, lo, hi, x);
    return p < hi && a[p] == x;
}

// Entries of N(v) within [lo, hi): the split index (first neighbour above
// v) answers the common bounds lo = v+1 and hi = v without a search.
template <class GR>
__device__ __forceinline__ void list_range(const GR& g, uint32_t v, uint32_t lo, uint32_t hi,
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
    DGraph g;
    gcp<DPlan> P;
    uint32_t v[KMAX];        // wave-uniform prefix of the core match
    gp<uint32_t> buf;        // per-wave level buffers
    uint64_t stride;
    uint32_t size[KMAX];     // entries in each level buffer
    uint64_t bytes;          // algorithmic bytes (counting build only)
    gp<uint32_t> bmw;        // this wave's root bitmap (n bits) or null
    gcp<uint32_t> bm;        // bmw while it holds N(v0), else null
    const int* cancel = nullptr;   // host-visible cancel flag (matching kernel) or null
    uint32_t ctick = 0;            // inner steps since the flag was last read
    uint32_t stopped = 0;          // the flag was seen set: inner loops end early
};

// ---------------------------------------------------------------- wave helpers

// Cancellation inside long inner loops (a flattened filter chunk, a batch of
// 64 finishing candidates): lane 0 reads the host flag every 64th step; once
// it is seen set every inner loop ends at its next step, and the results are
// discarded with the query.  Wave-uniform.
__device__ __forceinline__ bool ctx_stop(Ctx& c) {
    if (c.stopped) return true;
    if (!c.cancel || ((++c.ctick) & 63u)) return false;
    uint32_t f = 0;
    if (__lane_id() == 0) f = (uint32_t)__atomic_load_n(c.cancel, __ATOMIC_RELAXED);
    c.stopped = __builtin_amdgcn_readfirstlane(f) != 0 ? 1u : 0u;
    return c.stopped != 0;
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t x) {
    const int lane = wave_lane();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x;
}

// Lane owning flattened entry t: the number of lanes whose inclusive
// prefix is <= t (prefixes are non-decreasing over the lanes).  Every lane
// must execute it (cross-lane reads).
__device__ __forceinline__ int owner_of(uint32_t incl, uint32_t t) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
        uint32_t v = __shfl(incl, lo + step - 1);
        if (v <= t) lo += step;
    }
    return lo;
}

// Bits [a, b) of a 64-bit mask (0 <= a < b <= 64).
__device__ __forceinline__ uint64_t range_mask(uint32_t a, uint32_t b) {
    uint64_t m = (b - a >= 64) ? ~0ull : ((1ull << (b - a)) - 1ull);
    return m << a;
}

template <class P>
__device__ __forceinline__ bool bm_test(P bm, uint32_t x) {
    return (bm[x >> 5] >> (x & 31)) & 1u;
}

// Root bitmap of N(r): the lane holding the first entry of each 32-id word
// assembles the word from the following entries (the list is sorted) and
// stores it, so no two lanes write one word.  The bitmap is all zero before.
__device__ void bm_build(Ctx& c, uint32_t r) {
    const int lane = wave_lane();
    const uint32_t b = c.g.rp[r], e = c.g.rp[r + 1];
    for (uint32_t p = b + lane; p < e; p += 64) {
        const uint32_t x = c.g.col[p];
        const uint32_t w = x >> 5;
        if (p == b || (c.g.col[p - 1] >> 5) != w) {
            uint32_t bits = 0;
            for (uint32_t q = p; q < e; ++q) {
                const uint32_t y = c.g.col[q];
                if ((y >> 5) != w) break;
                bits |= 1u << (y & 31);
            }
            c.bmw[w] = bits;
        }
    }
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    c.bm = c.bmw;
}

__device__ void bm_clear(Ctx& c, uint32_t r) {
    const int lane = wave_lane();
    const uint32_t b = c.g.rp[r], e = c.g.rp[r + 1];
    // every lane has finished its probes of the bitmap
    __builtin_amdgcn_wave_barrier();
    for (uint32_t p = b + lane; p < e; p += 64) c.bmw[c.g.col[p] >> 5] = 0u;
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    c.bm = nullptr;
}

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
template <class GR>
__device__ __forceinline__ int pick_driver(const GR& g, const uint32_t* vv, uint8_t adj, uint32_t lo,
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

// Per-candidate test against probe lists, injectivity and label.  With a
// root bitmap, list 0 is tested on the bitmap; every candidate handed to a
// probe lies inside the probe's id bounds, so membership in all of N(v0)
// equals membership in its bounded range.
struct Probe {
    uint32_t pb[KMAX], pe[KMAX];
    uint8_t adj, anti, neq, bm;
    int8_t label;
};

__device__ __forceinline__ void clear_probe(Probe& pr, uint8_t neq, int8_t label) {
#pragma unroll
    for (int i = 0; i < KMAX; ++i) pr.pb[i] = pr.pe[i] = 0;
    pr.adj = pr.anti = pr.bm = 0;
    pr.neq = neq;
    pr.label = label;
}

template <bool BYTES>
__device__ __forceinline__ uint64_t make_probe(const Ctx& c, const uint32_t* vv, uint8_t adj, uint8_t anti,
                                               uint8_t neq, int8_t label, uint32_t lo, uint32_t hi,
                                               Probe& pr) {
    uint64_t bytes = 0;
    pr.adj = adj;
    pr.anti = anti;
    pr.neq = neq;
    pr.label = label;
    pr.bm = (c.bm != nullptr && ((adj | anti) & 1u)) ? 1 : 0;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        pr.pb[i] = pr.pe[i] = 0;
        if (((adj | anti) >> i) & 1) {
            if (i == 0 && pr.bm && !BYTES) continue;
            list_range(c.g, vv[i], lo, hi, pr.pb[i], pr.pe[i]);
            bytes += 8 + 4ull * (pr.pe[i] - pr.pb[i]);
        }
    }
    return bytes;
}

__device__ __forceinline__ bool probe_ok(const Ctx& c, const uint32_t* vv, const Probe& pr, uint32_t x) {
    if (pr.label >= 0 && c.g.lab[x] != (uint8_t)pr.label) return false;
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
        if (((pr.neq >> i) & 1) && x == vv[i]) return false;
    if (pr.bm && ((pr.adj | pr.anti) & 1u)) {
        const bool in0 = bm_test(c.bm, x);
        if ((pr.adj & 1u) && !in0) return false;
        if ((pr.anti & 1u) && in0) return false;
    }
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        if (i == 0 && pr.bm) continue;
        if (!(((pr.adj | pr.anti) >> i) & 1)) continue;
        // x lies inside the bounds the list was cut to, so membership in the
        // cut list is membership in N(v_i): a hub answers from its bitmap
        // with one load, any other list by binary search
        const uint32_t v = vv[i];
        const bool in = (c.g.hubbm && v >= c.g.hub0)
                            ? (c.g.hubbm[(uint64_t)(v - c.g.hub0) * c.g.hub_words + (x >> 5)] >> (x & 31)) & 1u
                            : in_sorted(c.g.col, pr.pb[i], pr.pe[i], x);
        if (((pr.adj >> i) & 1) && !in) return false;
        if (((pr.anti >> i) & 1) && in) return false;
    }
    return true;
}

// The probe of lane o (lists: union of the list bits any lane may probe).
__device__ __forceinline__ void fetch_probe(const Probe& pr, int o, uint8_t lists, Probe& q) {
    const uint32_t packed = __shfl((uint32_t)pr.adj | ((uint32_t)pr.anti << 8) | ((uint32_t)pr.bm << 16), o);
    q.adj = (uint8_t)packed;
    q.anti = (uint8_t)(packed >> 8);
    q.bm = (uint8_t)(packed >> 16);
    q.neq = pr.neq;
    q.label = pr.label;
#pragma unroll
    for (int i = 0; i < KMAX; ++i) {
        q.pb[i] = q.pe[i] = 0;
        if ((lists >> i) & 1) {
            q.pb[i] = __shfl(pr.pb[i], o);
            q.pe[i] = __shfl(pr.pe[i], o);
        }
    }
}

// ---------------------------------------------------------------- wave-cooperative level

// Label and injectivity of a candidate already known to lie in every list.
__device__ __forceinline__ bool merge_ok(const Ctx& c, const uint32_t* vv, const Probe& pr, uint32_t x) {
    if (pr.label >= 0 && c.g.lab[x] != (uint8_t)pr.label) return false;
#pragma unroll
    for (int i = 0; i < KMAX; ++i)
        if (((pr.neq >> i) & 1) && x == vv[i]) return false;
    return true;
}

// Sorted intersection of two bounded lists of similar length by merge path:
// the merged sequence of A and B (equal entries: A first) is cut into 64
// stretches of equal length and lane l merges stretch l, its start found by
// a binary search along its diagonal.  An entry of A is a match when the B
// cursor stands on an equal entry as it is taken.  The lanes count their
// matches, a wave prefix sum places them, and a second merge writes them,
// so the output is sorted.  Every read stays inside A[0, la) and B[0, lb).
__device__ uint32_t merge_level(const Ctx& c, gcp<uint32_t> A, uint32_t la, gcp<uint32_t> B, uint32_t lb,
                                const Probe& pr, gp<uint32_t> out) {
    const uint32_t lane = (uint32_t)wave_lane();
    const uint32_t total = la + lb;
    const uint32_t len = (total + 63) / 64;
    const uint32_t d0 = min(total, lane * len), d1 = min(total, d0 + len);
    uint32_t lo = d0 > lb ? d0 - lb : 0, hi = min(d0, la);
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (A[mid] <= B[d0 - mid - 1]) lo = mid + 1;
        else hi = mid;
    }
    const uint32_t i0 = lo, j0 = d0 - lo;
    uint32_t cnt = 0;
    {
        uint32_t i = i0, jb = j0;
        for (uint32_t st = d0; st < d1; ++st) {
            if (i < la && (jb >= lb || A[i] <= B[jb])) {
                const uint32_t x = A[i];
                if (jb < lb && B[jb] == x && merge_ok(c, c.v, pr, x)) ++cnt;
                ++i;
            } else {
                ++jb;
            }
        }
    }
    const uint32_t incl = wave_incl_scan(cnt);
    const uint32_t tot = __shfl(incl, 63);
    if (cnt) {
        uint32_t o = incl - cnt;
        uint32_t i = i0, jb = j0;
        for (uint32_t st = d0; st < d1; ++st) {
            if (i < la && (jb >= lb || A[i] <= B[jb])) {
                const uint32_t x = A[i];
                if (jb < lb && B[jb] == x && merge_ok(c, c.v, pr, x)) out[o++] = x;
                ++i;
            } else {
                ++jb;
            }
        }
    }
    return tot;
}

// Materialise the candidates of core level j (wave-uniform prefix c.v).
// Two adjacency lists of similar length (the driver and one probe list, no
// anti-edge) are intersected by merge path; otherwise the lanes stream the
// driver and test each entry against the probe lists by binary search.
template <bool BYTES>
__device__ uint32_t wave_level(Ctx& c, int j) {
    const DLevel L = gload(&c.P->lev[j]);
    const int lane = wave_lane();
    uint32_t lo, hi;
    bounds_of(c.v, L.gt, L.lt, lo, hi);
    gp<uint32_t> out = c.buf + (uint64_t)j * c.stride;
    if (lo >= hi) return 0;
    gcp<uint32_t> drv;
    uint32_t b, e;
    uint8_t chk = L.adj, anti = L.anti;
    if (L.base != 0xff) {
        gcp<uint32_t> bb = c.buf + (uint64_t)L.base * c.stride;
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
    uint64_t pbytes = make_probe<BYTES>(c, c.v, chk, anti, L.neq, L.label, lo, hi, pr);
    if (BYTES && lane == 0) c.bytes += pbytes + 4ull * (e - b);
    uint32_t total = 0;
    if (L.base == 0xff && !anti && !pr.bm && chk && !(chk & (chk - 1))) {
        const int pi = __builtin_ctz((uint32_t)chk);
        const uint32_t la = e - b, lb = pr.pe[pi] - pr.pb[pi];
        if (la + lb >= 256 && lb <= 4 * la) {
            total = merge_level(c, drv + b, la, c.g.col + pr.pb[pi], lb, pr, out);
            __threadfence_block();
            __builtin_amdgcn_wave_barrier();
            return total;
        }
    }
    for (uint32_t base = b; base < e; base += 64) {
        uint32_t idx = base + lane;
        bool ok = idx < e;
        uint32_t x = ok ? drv[idx] : 0;
        ok = ok && probe_ok(c, c.v, pr, x);
        uint64_t m = __ballot(ok);
        if (ok) out[total + lane_prefix(m)] = x;
        total += (uint32_t)__popcll(m);
    }
    // other lanes read the buffer next
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
    return total;
}

// ---------------------------------------------------------------- per-lane work
//
// Every function below is called by all 64 lanes together (it reads other
// lanes); `valid` marks the lanes that hold a partial match.

template <bool BYTES, bool SMALL = false>
__device__ u128 lanes_tail(Ctx& c, const uint32_t* vv, bool valid, uint64_t aggm);

__device__ __forceinline__ u128 poly_eval(gcp<DPlan> P, const uint64_t* tv) {
    i128 s = 0;
    const int nm = P->nmono;
    for (int m = 0; m < nm; ++m) {
        const DMono M = gload(&P->mono[m]);
        i128 prod = (i128)M.coef;
        for (int f = 0; f < M.nf; ++f) prod *= (i128)tv[M.f[f]];
        s += prod;
    }
    return s > 0 ? (u128)s : (u128)0;
}

// A cheap tail term (one adjacency list, range count with injectivity
// corrections) or the aggregation multiplicity; per lane.
template <bool BYTES>
__device__ __forceinline__ uint64_t cheap_term(Ctx& c, const uint32_t* vv, const DTerm& t, uint64_t aggm) {
    if (t.agg) return aggm;
    uint32_t lo, hi;
    bounds_of(vv, t.gt, t.lt, lo, hi);
    if (lo >= hi) return 0;
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

// Flattened filter: lane l owns drv[b_l, b_l + len_l) and the probe pr_l of
// its match vv_l.  MODE 0 returns, per owner, the number of entries that
// pass; MODE 1 (level j) extends every passing entry x to the match
// vv_owner + {v_j = x} and adds its tail to `acc` (on the lane that tested
// x); the return value is then 0.
template <int MODE, bool BYTES>
__device__ uint64_t flat_filter(Ctx& c, const uint32_t* vv, gcp<uint32_t> drv, uint32_t b, uint32_t len,
                                const Probe& pr, uint8_t lists, int j, u128& acc) {
    const int lane = wave_lane();
    const uint32_t incl = wave_incl_scan(len);
    const uint32_t total = __shfl(incl, 63);
    const uint32_t excl = incl - len;
    const uint8_t nl = (uint8_t)(lists & (c.bm ? 0xfe : 0xff));
    uint64_t cnt = 0;
    for (uint32_t base = 0; base < total; base += 64) {
        if (ctx_stop(c)) break;
        const uint32_t t = base + lane;
        const bool act = t < total;
        const int o = owner_of(incl, act ? t : total - 1);
        const uint32_t src = __shfl(b, o) + (t - __shfl(excl, o));
        Probe q;
        fetch_probe(pr, o, nl, q);
        uint32_t vo[KMAX];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) vo[i] = __shfl(vv[i], o);
        uint32_t x = act ? drv[src] : 0u;
        const bool ok = act && probe_ok(c, vo, q, x);
        if (MODE == 0) {
            const uint64_t m = __ballot(ok);
            const uint32_t s = max(excl, base), f = min(incl, base + 64);
            if (s < f) cnt += (uint64_t)__popcll(m & range_mask(s - base, f - base));
        } else {
            vo[j] = x;
            acc += lanes_tail<BYTES>(c, vo, ok, 0);
        }
    }
    return cnt;
}

// A tail term that needs a set operation, for every lane's match.
template <bool BYTES>
__device__ uint64_t flat_term(Ctx& c, const uint32_t* vv, bool valid, const DTerm& t) {
    uint32_t lo, hi, b = 0, e = 0;
    Probe pr;
    clear_probe(pr, t.neq, t.label);
    bounds_of(vv, t.gt, t.lt, lo, hi);
    if (valid && lo < hi) {
        int bi = pick_driver(c.g, vv, t.adj, lo, hi, b, e);
        uint64_t pbytes =
            make_probe<BYTES>(c, vv, (uint8_t)(t.adj & ~(1u << bi)), t.anti, t.neq, t.label, lo, hi, pr);
        if (BYTES) c.bytes += 8 + pbytes + 4ull * (e - b);
    }
    u128 dummy = 0;
    return flat_filter<0, BYTES>(c, vv, c.g.col, b, e - b, pr, (uint8_t)(t.adj | t.anti), 0, dummy);
}

// Tails of at most SMALL_TERMS terms (the common case) keep the term values
// in registers: a dynamically indexed array would live in per-lane scratch
// memory, whose traffic goes through the L2 for every evaluated match.
constexpr int SMALL_TERMS = 4;

__device__ __forceinline__ uint64_t pick4(uint32_t i, uint64_t t0, uint64_t t1, uint64_t t2, uint64_t t3) {
    return i == 0 ? t0 : (i == 1 ? t1 : (i == 2 ? t2 : t3));
}

template <bool BYTES>
__device__ __forceinline__ uint64_t term_value(Ctx& c, const uint32_t* vv, bool valid, const DTerm& t,
                                               uint64_t aggm) {
    if (t.agg || t.cheap) return valid ? cheap_term<BYTES>(c, vv, t, aggm) : 0;
    return flat_term<BYTES>(c, vv, valid, t);
}

template <bool BYTES, bool SMALL>
__device__ u128 lanes_tail(Ctx& c, const uint32_t* vv, bool valid, uint64_t aggm) {
    const int nt = c.P->nterm;
    if (SMALL && nt <= SMALL_TERMS) {
        uint64_t t0 = 0, t1 = 0, t2 = 0, t3 = 0;
        if (nt > 0) t0 = term_value<BYTES>(c, vv, valid, gload(&c.P->term[0]), aggm);
        if (nt > 1) t1 = term_value<BYTES>(c, vv, valid, gload(&c.P->term[1]), aggm);
        if (nt > 2) t2 = term_value<BYTES>(c, vv, valid, gload(&c.P->term[2]), aggm);
        if (nt > 3) t3 = term_value<BYTES>(c, vv, valid, gload(&c.P->term[3]), aggm);
        if (!valid) return 0;
        i128 s = 0;
        const int nm = c.P->nmono;
        for (int m = 0; m < nm; ++m) {
            const DMono M = gload(&c.P->mono[m]);
            // set sizes are below 2^32, so two factors multiply exactly in
            // 64 bits and the coefficient needs one 64 x 64 -> 128 product
            const uint64_t f0 = M.nf > 0 ? pick4(M.f[0], t0, t1, t2, t3) : 1u;
            const uint64_t f1 = M.nf > 1 ? pick4(M.f[1], t0, t1, t2, t3) : 1u;
            i128 prod = (i128)M.coef * (i128)(f0 * f1);
            if (M.nf > 2) {
#pragma unroll
                for (int f = 2; f < MAX_FAC; ++f)
                    if (f < M.nf) prod *= (i128)pick4(M.f[f], t0, t1, t2, t3);
            }
            s += prod;
        }
        return s > 0 ? (u128)s : (u128)0;
    }
    uint64_t tv[MAX_TERMS];
    for (int q = 0; q < nt; ++q) {
        const DTerm t = gload(&c.P->term[q]);
        if (t.agg || t.cheap) tv[q] = valid ? cheap_term<BYTES>(c, vv, t, aggm) : 0;
        else tv[q] = flat_term<BYTES>(c, vv, valid, t);
    }
    return valid ? poly_eval(c.P, tv) : (u128)0;
}

// Level j for every lane's match vv (complete below j): MODE 0 counts the
// candidates (times the plan multiplier), MODE 1 evaluates the tail of
// every extension.
template <int MODE, bool BYTES>
__device__ void lanes_level(Ctx& c, const uint32_t* vv, bool valid, int j, u128& acc) {
    const DLevel L = gload(&c.P->lev[j]);
    uint32_t lo, hi, b = 0, e = 0;
    bounds_of(vv, L.gt, L.lt, lo, hi);
    const bool on = valid && lo < hi;
    gcp<uint32_t> drv = c.g.col;
    uint8_t chk = L.adj, anti = L.anti;
    Probe pr;
    clear_probe(pr, L.neq, L.label);
    if (L.base != 0xff) {
        gcp<uint32_t> bb = c.buf + (uint64_t)L.base * c.stride;
        chk &= (uint8_t)~c.P->lev[L.base].adj;
        anti &= (uint8_t)~c.P->lev[L.base].anti;
        drv = bb;
        if (on) {
            const uint32_t n = c.size[L.base];
            b = lo ? lower_bound_u32(bb, 0, n, lo) : 0;
            e = hi != NOB ? lower_bound_u32(bb, b, n, hi) : n;
        }
    }
    const uint8_t lists = (uint8_t)(chk | anti);
    if (on) {
        uint8_t pc = chk;
        if (L.base == 0xff) {
            int bi = pick_driver(c.g, vv, L.adj, lo, hi, b, e);
            pc &= (uint8_t)~(1u << bi);
            if (BYTES) c.bytes += 8;
        }
        uint64_t pbytes = make_probe<BYTES>(c, vv, pc, anti, L.neq, L.label, lo, hi, pr);
        if (BYTES) c.bytes += pbytes + 4ull * (e - b);
    }
    const uint64_t cnt = flat_filter<MODE, BYTES>(c, vv, drv, b, e - b, pr, lists, j, acc);
    if (MODE == 0) acc += (u128)cnt * (u128)(uint32_t)c.P->mult;
}

// ---------------------------------------------------------------- aggregation

// A wave's private counter array is touched by that wave only, so its
// read-modify-writes need workgroup scope: they complete in the L2 of the
// wave's own XCD instead of travelling to memory as device-scope atomics.
// Every access to such an array goes through these two.
__device__ __forceinline__ uint32_t wave_add(uint32_t* p) {
    return __hip_atomic_fetch_add(p, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t wave_take(uint32_t* p) {
    return __hip_atomic_exchange(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Two-hop aggregation for the last core level j: targets x reached from
// bridges y in N(v_src) (bridge bounds and label) are counted in a per-wave
// dense array; the bridges' lists are streamed flattened, 64 bridges at a
// time.  Every touched target is then evaluated lane-parallel with its
// multiplicity as the bridge term.
//
// A high-degree root (j = 1) is split over several work items by target id:
// slice [s0, s1) of the root's degree d takes the targets in the matching
// fraction of the bounded id range, so each target still collects its full
// multiplicity inside one wave.
template <bool BYTES>
__device__ void agg_level(Ctx& c, int j, uint32_t wid, uint32_t* s_touch, const KArgs& a, u128& acc,
                          uint32_t s0 = 0, uint32_t s1 = 0xffffffffu) {
    gcp<DPlan> P = c.P;
    const DLevel L = gload(&P->lev[j]);
    const int lane = wave_lane();
    uint32_t* cnt = a.aggcnt + (uint64_t)wid * c.g.n;
    uint32_t* touched = a.aggtouch + (uint64_t)wid * c.g.n;
    uint32_t blo, bhi, lo, hi;
    bounds_of(c.v, P->bridge_gt, P->bridge_lt, blo, bhi);
    bounds_of(c.v, L.gt, L.lt, lo, hi);
    if (blo >= bhi || lo >= hi) return;
    if (s0 != 0 || s1 != 0xffffffffu) {
        const uint32_t r = c.v[0];
        const uint64_t d = c.g.rp[r + 1] - c.g.rp[r];
        const uint64_t top = hi == NOB ? (uint64_t)c.g.n : (uint64_t)hi;
        const uint64_t span = top > lo ? top - lo : 0;
        const uint32_t nlo = (uint32_t)(lo + span * min((uint64_t)s0, d) / d);
        const uint32_t nhi = s1 >= d ? hi : (uint32_t)(lo + span * (uint64_t)s1 / d);
        lo = nlo;
        hi = nhi;
        if (lo >= hi) return;
    }
    uint32_t bb, be;
    list_range(c.g, c.v[P->bridge_src], blo, bhi, bb, be);
    if (BYTES && lane == 0) c.bytes += 8 + 4ull * (be - bb);
    if (lane == 0) *s_touch = 0;
    __builtin_amdgcn_wave_barrier();
    for (uint32_t base = bb; base < be; base += 64) {
        const uint32_t idx = base + lane;
        bool valid = idx < be;
        const uint32_t y = valid ? c.g.col[idx] : 0u;
        if (valid && P->bridge_label >= 0 && c.g.lab[y] != (uint8_t)P->bridge_label) valid = false;
        for (int i = 0; i < j; ++i) valid = valid && (y != c.v[i]);
        uint32_t yb = 0, yf = 0;
        if (valid) {
            list_range(c.g, y, lo, hi, yb, yf);
            if (BYTES) c.bytes += 8 + 4ull * (yf - yb);
        }
        const uint32_t len = yf - yb;
        const uint32_t incl = wave_incl_scan(len);
        const uint32_t total = __shfl(incl, 63);
        const uint32_t excl = incl - len;
        for (uint32_t tb = 0; tb < total; tb += 64) {
            const uint32_t t = tb + lane;
            const bool act = t < total;
            const int o = owner_of(incl, act ? t : total - 1);
            const uint32_t src = __shfl(yb, o) + (t - __shfl(excl, o));
            if (!act) continue;
            const uint32_t x = c.g.col[src];
            if (L.label >= 0 && c.g.lab[x] != (uint8_t)L.label) continue;
            bool skip = false;
#pragma unroll
            for (int i = 0; i < KMAX; ++i)
                if (((L.neq >> i) & 1) && x == c.v[i]) skip = true;
            if (skip) continue;
            if (wave_add(&cnt[x]) == 0u) touched[atomicAdd(s_touch, 1u)] = x;
        }
    }
    __builtin_amdgcn_wave_barrier();
    __threadfence_block();
    const uint32_t ntouch = bcast(*(volatile uint32_t*)s_touch);
    uint32_t vv[KMAX];
#pragma unroll
    for (int i = 0; i < KMAX; ++i) vv[i] = c.v[i];
    for (uint32_t base = 0; base < ntouch; base += 64) {
        const uint32_t idx = base + lane;
        const bool valid = idx < ntouch;
        uint32_t m = 0;
        if (valid) {
            const uint32_t x = touched[idx];
            m = wave_take(&cnt[x]);
            vv[j] = x;
        }
        acc += lanes_tail<BYTES, true>(c, vv, valid, m);
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
    gp<uint64_t> rows = (gp<uint64_t>)c.buf;
    gcp<uint32_t> C1 = c.g.col + b;
    for (uint32_t i = lane; i < s; i += 64) {
        const uint32_t x = C1[i];
        uint32_t p = c.g.split[x];
        const uint32_t pe = c.g.rp[x + 1];
        if (BYTES) c.bytes += 8 + 4ull * (pe - p) + 4ull * (s - i - 1);
        gp<uint64_t> row = rows + (uint64_t)i * W;
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
        gcp<uint64_t> ri = rows + (uint64_t)i * W;
        uint64_t cnt = 0;
        if (nc == 3) {
            for (uint32_t w = 0; w < W; ++w) cnt += __popcll(ri[w]);
        } else {
            for (uint32_t w = 0; w < W; ++w) {
                uint64_t m = ri[w];
                while (m) {
                    const uint32_t j = (w << 6) + __builtin_ctzll(m);
                    m &= m - 1;
                    gcp<uint64_t> rj = rows + (uint64_t)j * W;
                    if (nc == 4) {
                        for (uint32_t w2 = j >> 6; w2 < W; ++w2) cnt += __popcll(ri[w2] & rj[w2]);
                    } else {
                        for (uint32_t w2 = j >> 6; w2 < W; ++w2) {
                            uint64_t t = ri[w2] & rj[w2];
                            while (t) {
                                const uint32_t k = (w2 << 6) + __builtin_ctzll(t);
                                t &= t - 1;
                                gcp<uint64_t> rk = rows + (uint64_t)k * W;
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
    gcp<DPlan> P = c.P;
    const int lane = wave_lane();
    const int last = P->ncore - 1;
    gcp<uint32_t> bj = c.buf + (uint64_t)j * c.stride;
    for (uint32_t base = b; base < e; base += 64) {
        if (ctx_stop(c)) break;
        const uint32_t idx = base + lane;
        const bool valid = idx < e;
        uint32_t vv[KMAX];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) vv[i] = c.v[i];
        vv[j] = valid ? bj[idx] : 0u;
        if (P->nterm == 0) lanes_level<0, BYTES>(c, vv, valid, last, acc);
        else lanes_level<1, BYTES>(c, vv, valid, last, acc);
    }
}

// Cancellation: the host sets a coherent flag; lane 0 reads it once the
// calls since the last read (a root, a step at any materialised level, a
// penultimate-level aggregation, a batch of 64 level-1 candidates) weigh 16,
// a root weighing one plus its degree over 64, so an abandoned item ends
// within a few of its innermost iterations even on hub roots.  Wave-uniform.
__device__ __forceinline__ bool should_stop(const KArgs& a, uint32_t& tick, uint32_t weight = 1) {
    if (!a.cancel) return false;
    tick += weight;
    if (tick < 16u) return false;
    tick = 0;
    uint32_t stop = 0;
    if (wave_lane() == 0) stop = (uint32_t)__atomic_load_n(a.cancel, __ATOMIC_RELAXED);
    return bcast(stop) != 0;
}

template <bool BYTES>
#ifdef PM_MATCH_WPE
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(PM_MATCH_WPE))) match_kernel(KArgs a) {
#else
__global__ void __launch_bounds__(256) match_kernel(KArgs a) {
#endif
    __shared__ uint32_t s_touch[4];
    const int lane = wave_lane();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    uint32_t* my_touch = &s_touch[threadIdx.x >> 6];
    Ctx c;
    c.g = dgraph(a.g);
    c.stride = a.buf_stride;
    c.buf = (gp<uint32_t>)(a.scratch + (uint64_t)wid * (uint64_t)KMAX * a.buf_stride);
    c.bytes = 0;
    c.bmw = a.rootbm ? (gp<uint32_t>)(a.rootbm + (uint64_t)wid * a.bm_words) : nullptr;
    c.bm = nullptr;
    c.cancel = a.cancel;
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
        gcp<DPlan> P = (gcp<DPlan>)a.plans + pi;
        c.P = P;
        const int nc = P->ncore;
        const int8_t rl = P->lev[0].label;
        if (nc == 1) {
            // lanes take roots; every tail term is evaluated per lane
            if (item.s0 != 0 || P->nterm == 0) continue;
            for (uint32_t base = item.r0; base < item.r1; base += 64) {
                const uint32_t r = base + lane;
                const bool valid = r < item.r1 && (rl < 0 || a.g.lab[r] == (uint8_t)rl);
                uint32_t vv[KMAX] = {valid ? r : 0u, 0, 0, 0, 0};
                acc += lanes_tail<BYTES>(c, vv, valid, 0);
            }
            continue;
        }
        for (uint32_t r = item.r0; r < item.r1; ++r) {
            if (stopped || c.stopped || should_stop(a, tick, 1u + ((a.g.rp[r + 1] - a.g.rp[r]) >> 6))) {
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
                    agg_level<BYTES>(c, 1, wid, my_touch, a, acc, item.s0, item.s1);
                    continue;
                }
                uint32_t n = wave_level<BYTES>(c, 1);
                uint32_t b = min(item.s0, n), e = min(item.s1, n);
                if (P->nterm == 0) {
                    if (lane == 0 && e > b) acc += (u128)(e - b) * (u128)(uint32_t)P->mult;
                    continue;
                }
                gcp<uint32_t> b1 = c.buf + c.stride;
                const bool usebm = P->bm0 && c.bmw && e > b;
                if (usebm) bm_build(c, r);
                for (uint32_t base = b; base < e; base += 64) {
                    if (should_stop(a, tick)) {
                        stopped = true;
                        break;
                    }
                    const uint32_t idx = base + lane;
                    const bool valid = idx < e;
                    uint32_t vv[KMAX] = {r, valid ? b1[idx] : 0u, 0, 0, 0};
                    acc += lanes_tail<BYTES>(c, vv, valid, 0);
                }
                if (usebm) bm_clear(c, r);
                continue;
            }
            // nc >= 3: levels 1 .. nc-2 materialised, lanes finish
            const int pen = nc - 2;
            uint32_t pos[KMAX], end[KMAX];
            c.size[1] = wave_level<BYTES>(c, 1);
            pos[1] = min(item.s0, c.size[1]);
            end[1] = min(item.s1, c.size[1]);
            const bool usebm = P->bm0 && c.bmw && end[1] > pos[1];
            if (usebm) bm_build(c, r);
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
                if (usebm) bm_clear(c, r);
                continue;
            }
            int j = 1;
            while (j >= 1) {
                if (pos[j] >= end[j]) {
                    --j;
                    continue;
                }
                if (c.stopped || should_stop(a, tick)) {
                    stopped = true;
                    break;
                }
                c.v[j] = c.buf[(uint64_t)j * c.stride + pos[j]];
                ++pos[j];
                ++j;
                c.size[j] = wave_level<BYTES>(c, j);
                if (j == pen) {
                    if (P->agg_last) {
                        for (uint32_t q = 0; q < c.size[j] && !stopped; ++q) {
                            if (should_stop(a, tick)) {
                                stopped = true;
                                break;
                            }
                            c.v[j] = c.buf[(uint64_t)j * c.stride + q];
                            agg_level<BYTES>(c, j + 1, wid, my_touch, a, acc);
                        }
                    } else {
                        lanes_finish<BYTES>(c, j, 0, c.size[j], acc);
                    }
                    if (stopped || c.stopped) {
                        stopped = true;
                        break;
                    }
                    --j;
                    continue;
                }
                pos[j] = 0;
                end[j] = c.size[j];
            }
            if (usebm) bm_clear(c, r);
        }
    }
    if (cur >= 0) flush(a, cur, acc);
    if (BYTES) {
        unsigned long long bsum = c.bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (lane == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

// ---------------------------------------------------------------- edge-induced 5-cycles

__device__ __forceinline__ uint32_t wave_or(uint32_t* p, uint32_t v) {
    return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
// A counter the wave's atomics (performed in the L2) have updated: read at
// agent scope, past the compute unit's L1, which may still hold the line
// from an earlier root.
__device__ __forceinline__ uint32_t wave_peek(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Every 5-cycle once, at its lowest vertex a (degree-order ids).  For the
// targets t > a, A(t) counts the out-neighbours b of a (b > a) adjacent to
// t, filled in the wave's dense counter array by streaming N(b) above a for
// every out-neighbour b, flattened over the lanes; bit 31 of a counter marks
// t as an out-neighbour of a itself, f(t).  A cycle a-b-x-y-e-a with x < y
// is one edge {x, y} opposite a (y in N+(x): the short out-list) and one
// pair of bridges b in N(a) n N(x), e in N(a) n N(y), both above a, with
// b != y, e != x and b != e.  The wave sums, over the touched x and every y
// in N+(x), (A(x) - f(y)) (A(y) - f(x)): the corrections remove b = y and
// e = x (y is a bridge of x exactly when f(y)); b = e is left in, and its
// total is subtracted on the host (the companion triangle plan).  A target
// with A = 0 contributes nothing: f(y) = 1 would make y a bridge of x.
template <bool BYTES>
__global__ void __launch_bounds__(256) cycle5_kernel(KArgs a) {
    __shared__ uint32_t s_touch[4];
    constexpr uint32_t FLAG = 0x80000000u;
    const int lane = wave_lane();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    uint32_t* my_touch = &s_touch[threadIdx.x >> 6];
    uint32_t* cnt = a.aggcnt + (uint64_t)wid * a.g.n;
    uint32_t* touched = a.aggtouch + (uint64_t)wid * a.g.n;
    const KGraph& g = a.g;
    u128 acc = 0;
    uint64_t bytes = 0;
    int cur = -1;
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
        // a hub's level-1 slices: the first slice takes the whole root
        if (item.s0 != 0) continue;
        for (uint32_t r = item.r0; r < item.r1; ++r) {
            if (should_stop(a, tick)) {
                stopped = true;
                break;
            }
            // a root with one out-neighbour has no 5-cycle, but its pairs with
            // both bridges equal enter the companion plan's total: keep it
            const uint32_t bb = g.split[r], be = g.rp[r + 1];
            if (be == bb) continue;
            if (BYTES && lane == 0) bytes += 8 + 4ull * (be - bb);
            if (lane == 0) *my_touch = 0;
            __builtin_amdgcn_wave_barrier();
            // fill: the targets above r of every out-neighbour
            for (uint32_t base = bb; base < be; base += 64) {
                const uint32_t k = base + lane;
                uint32_t yb = 0, yf = 0;
                if (k < be) {
                    list_range(g, g.col[k], r + 1, NOB, yb, yf);
                    if (BYTES) bytes += 8 + 4ull * (yf - yb);
                }
                const uint32_t len = yf - yb;
                const uint32_t incl = wave_incl_scan(len);
                const uint32_t tot = __shfl(incl, 63);
                const uint32_t excl = incl - len;
                for (uint32_t tb = 0; tb < tot; tb += 64) {
                    const uint32_t t = tb + lane;
                    const bool act = t < tot;
                    const int o = owner_of(incl, act ? t : tot - 1);
                    const uint32_t src = __shfl(yb, o) + (t - __shfl(excl, o));
                    if (!act) continue;
                    const uint32_t x = g.col[src];
                    if (wave_add(&cnt[x]) == 0u) touched[atomicAdd(my_touch, 1u)] = x;
                }
            }
            __threadfence_block();
            __builtin_amdgcn_wave_barrier();
            // mark the out-neighbours themselves
            for (uint32_t k = bb + lane; k < be; k += 64) {
                const uint32_t y = g.col[k];
                if (wave_or(&cnt[y], FLAG) == 0u) touched[atomicAdd(my_touch, 1u)] = y;
            }
            __threadfence_block();
            __builtin_amdgcn_wave_barrier();
            const uint32_t nt = bcast(*(volatile uint32_t*)my_touch);
            // pairs: every touched x with A(x) > 0, every y in N+(x)
            for (uint32_t base = 0; base < nt; base += 64) {
                const uint32_t idx = base + lane;
                uint32_t ax = 0, fx = 0, pb = 0, pe = 0;
                if (idx < nt) {
                    const uint32_t x = touched[idx];
                    const uint32_t v = wave_peek(&cnt[x]);
                    ax = v & ~FLAG;
                    fx = v >> 31;
                    if (ax) {
                        pb = g.split[x];
                        pe = g.rp[x + 1];
                        if (BYTES) bytes += 8 + 8ull * (pe - pb);
                    }
                }
                const uint32_t len = pe - pb;
                const uint32_t incl = wave_incl_scan(len);
                const uint32_t tot = __shfl(incl, 63);
                const uint32_t excl = incl - len;
                for (uint32_t tb = 0; tb < tot; tb += 64) {
                    const uint32_t t = tb + lane;
                    const bool act = t < tot;
                    const int o = owner_of(incl, act ? t : tot - 1);
                    const uint32_t src = __shfl(pb, o) + (t - __shfl(excl, o));
                    const uint32_t oax = __shfl(ax, o), ofx = __shfl(fx, o);
                    if (!act) continue;
                    const uint32_t v = wave_peek(&cnt[g.col[src]]);
                    const uint32_t ay = v & ~FLAG;
                    if (ay) {
                        const int64_t p = ((int64_t)oax - (int64_t)(v >> 31)) * ((int64_t)ay - (int64_t)ofx);
                        acc += (u128)(i128)p;
                    }
                }
            }
            __threadfence_block();
            __builtin_amdgcn_wave_barrier();
            // every counter back to zero
            for (uint32_t i = lane; i < nt; i += 64) wave_take(&cnt[touched[i]]);
            __threadfence_block();
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (cur >= 0) flush(a, cur, acc);
    if (BYTES) {
        unsigned long long bsum = bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (lane == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

// ---------------------------------------------------------------- house: 4-cycle support sums

// The sum over all 4-cycles of the triangle counts of their four edges.
// Every 4-cycle is met once, at its highest vertex x (degree-order ids),
// through the pair (x, y) with y its opposite vertex: the cycle's other two
// vertices are two of the c(x, y) common neighbours a < x (the bridges), so
// the pair contributes (c - 1) times the sum over its bridges of
// t(x, a) + t(a, y).  A wave takes one root x (or one slice of its target
// ids: a hub's work item cuts N(x) at its own neighbours' ids) and streams
// the bridges' lists below x twice, flattened over the lanes: first every
// target's c into the wave's dense counter array, then every wedge
// x - a - y adds (c(x, y) - 1)(t(x, a) + t(a, y)).  The supports are read
// at both ends of an edge: vtri_kernel mirrors each edge's count into the
// position of its lower end's entry in the higher end's list.
template <bool BYTES>
__global__ void __launch_bounds__(256) house_kernel(KArgs a) {
    __shared__ uint32_t s_touch[4];
    const int lane = wave_lane();
    const uint32_t wid = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    uint32_t* my_touch = &s_touch[threadIdx.x >> 6];
    uint32_t* cnt = a.aggcnt + (uint64_t)wid * a.g.n;
    uint32_t* touched = a.aggtouch + (uint64_t)wid * a.g.n;
    const KGraph& g = a.g;
    const uint32_t* sup = a.support;
    u128 acc = 0;
    uint64_t bytes = 0;
    int cur = -1;
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
        for (uint32_t x = item.r0; x < item.r1; ++x) {
            if (should_stop(a, tick)) {
                stopped = true;
                break;
            }
            const uint32_t xs = g.rp[x], xb = g.split[x], dx = g.rp[x + 1] - xs;
            if (xb - xs < 2) continue;
            // targets [lo, hi): the whole range below x, or the ids between
            // the neighbours at the slice's two ends
            const uint32_t lo = item.s0 == 0 ? 0u : g.col[xs + item.s0];
            const uint32_t hi = item.s1 >= dx ? x : min(g.col[xs + item.s1], x);
            if (lo >= hi) continue;
            if (BYTES && lane == 0) bytes += 8 + 4ull * (xb - xs);
            if (lane == 0) *my_touch = 0;
            __builtin_amdgcn_wave_barrier();
#pragma unroll 1
            for (int pass = 0; pass < 2; ++pass) {
                for (uint32_t base = xs; base < xb; base += 64) {
                    const uint32_t k = base + lane;
                    uint32_t yb = 0, yf = 0, txa = 0;
                    if (k < xb) {
                        list_range(g, g.col[k], lo, hi, yb, yf);
                        if (pass) txa = sup[k];
                        if (BYTES) bytes += (pass ? 12 : 8) + (pass ? 8ull : 4ull) * (yf - yb);
                    }
                    const uint32_t len = yf - yb;
                    const uint32_t incl = wave_incl_scan(len);
                    const uint32_t tot = __shfl(incl, 63);
                    const uint32_t excl = incl - len;
                    for (uint32_t tb = 0; tb < tot; tb += 64) {
                        const uint32_t t = tb + lane;
                        const bool act = t < tot;
                        const int o = owner_of(incl, act ? t : tot - 1);
                        const uint32_t src = __shfl(yb, o) + (t - __shfl(excl, o));
                        const uint32_t ot = __shfl(txa, o);
                        if (!act) continue;
                        const uint32_t y = g.col[src];
                        if (pass == 0) {
                            if (wave_add(&cnt[y]) == 0u) touched[atomicAdd(my_touch, 1u)] = y;
                        } else {
                            const uint32_t c = wave_peek(&cnt[y]);
                            if (c > 1) acc += (u128)((uint64_t)(c - 1) * ((uint64_t)ot + sup[src]));
                        }
                    }
                }
                __threadfence_block();
                __builtin_amdgcn_wave_barrier();
            }
            // every counter back to zero
            const uint32_t nt = bcast(*(volatile uint32_t*)my_touch);
            for (uint32_t i = lane; i < nt; i += 64) wave_take(&cnt[touched[i]]);
            __threadfence_block();
            __builtin_amdgcn_wave_barrier();
        }
    }
    if (cur >= 0) flush(a, cur, acc);
    if (BYTES) {
        unsigned long long bsum = bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (lane == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

// ---------------------------------------------------------------- heavy two-hop roots

// Roots of a plan whose first level is the aggregation level and whose
// two-hop mass is large: one workgroup, alone on its CU, takes one root (or
// one slice of its target ids) and counts the paths r - y - x to each target
// x in an LDS window of consecutive target ids.  LDS atomics run in the CU,
// so the sweep is bounded by reading the bridges' lists; the window is as
// large as the CU's LDS allows (128 KB of counters), so a bridge's list is
// cut into few pieces and most of its cache lines are read once.
//
// Every bridge keeps a cursor, the end of its list and its next target (in
// global scratch owned by the workgroup): a bridge without a target in the
// current window costs one read of that state.  Each window starts at the
// smallest pending target, so empty id ranges are never visited.  Waves take
// 64 bridges at a time from a shared counter, find each bridge's targets in
// the window by galloping from its cursor, and stream them flattened.  The
// first touch of a target marks its 64-id group; after the window is
// filled, the waves walk the marked groups, clear their counters, compact
// the touched targets into a per-wave queue and evaluate the tail 64
// targets at a time.
#ifndef PM_AW_THREADS
#define PM_AW_THREADS 1024
#endif
#ifndef PM_AW_WORDS
#define PM_AW_WORDS 32768
#endif
#ifndef PM_AW_UNROLL
#define PM_AW_UNROLL 4
#endif
constexpr uint32_t AW_THREADS = PM_AW_THREADS;
constexpr uint32_t AW_WAVES = AW_THREADS / 64;
constexpr uint32_t AW_WORDS = PM_AW_WORDS;   // counter words (128 KB by default)
constexpr uint32_t AW_QCAP = 128;            // per-wave queue of touched targets
constexpr int AW_UNROLL = PM_AW_UNROLL;
#ifndef PM_AW_LONG
#define PM_AW_LONG 64
#endif
constexpr uint32_t AW_LONG = PM_AW_LONG;     // a segment this long is streamed by the whole wave
constexpr uint32_t AW_CHUNK = 512;           // long segments are queued in chunks this long
constexpr uint32_t AW_CQCAP = 2048;          // chunk queue capacity
// workgroups of this kernel that fit one CU's 160 KB of LDS
constexpr int AW_CU_BLOCKS = (int)(160u * 1024u / (AW_WORDS * 4u + AW_WAVES * AW_QCAP * 6u + AW_CQCAP * 6u + 4096u));
static_assert(AW_CU_BLOCKS >= 1, "window does not fit the LDS");

// With H16 (a graph whose degrees fit 16 bits, so does every path count)
// two counters share a word and the window covers twice as many ids.
template <bool BYTES, bool H16>
__global__ void __launch_bounds__(AW_THREADS) agg_window_kernel(KArgs a) {
    constexpr uint32_t WIN_IDS = H16 ? 2 * AW_WORDS : AW_WORDS;
    constexpr uint32_t NGROUPS = WIN_IDS / 64;
    __shared__ uint32_t win[AW_WORDS];
    __shared__ uint32_t gbits[NGROUPS / 32];
    __shared__ uint16_t glist[NGROUPS];
    __shared__ uint16_t qoff[AW_WAVES][AW_QCAP];
    __shared__ uint32_t qm[AW_WAVES][AW_QCAP];
    __shared__ uint32_t cq_q[AW_CQCAP];    // queued chunks of long segments: start
    __shared__ uint16_t cq_n[AW_CQCAP];    //                                 length
    __shared__ uint32_t s_item, s_next[2], s_ng[2], s_batch, s_nck, s_ckhead;
    const int lane = wave_lane();
    const uint32_t tid = threadIdx.x;
    const uint32_t w = tid >> 6;
    // the sweep reads the graph through this copy, which never leaves
    // registers, so its loads compile as global (not flat) accesses; the
    // tail evaluation gets the graph through the context
    const KGraph G = a.g;
    Ctx c;
    c.g = dgraph(a.g);
    c.stride = 0;
    c.buf = nullptr;   // tails need no level buffers
    c.bytes = 0;
    c.bmw = nullptr;
    c.bm = nullptr;
    // per bridge: cursor, end of its list, next target
    uint32_t* cur = a.wscr + (uint64_t)blockIdx.x * (2 + EW_TERMS) * a.wscr_stride;
    uint32_t* fin = cur + a.wscr_stride;
    uint32_t* nxt = fin + a.wscr_stride;
    uint32_t* lst = nxt + a.wscr_stride;   // last target of the bridge below `top`
    for (uint32_t i = tid; i < AW_WORDS; i += AW_THREADS) win[i] = 0;
    for (uint32_t i = tid; i < NGROUPS / 32; i += AW_THREADS) gbits[i] = 0;
    int curp = -1;
    u128 acc = 0;
    const uint64_t total = (uint64_t)a.nplans * a.nitems;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            uint32_t it = atomicAdd(a.head, 1u);
            if (a.cancel && __atomic_load_n(a.cancel, __ATOMIC_RELAXED)) it = 0xffffffffu;
            s_item = it;
            s_next[0] = s_next[1] = NOB;
            s_ng[0] = s_ng[1] = 0;
            s_batch = 0;
            s_nck = s_ckhead = 0;
        }
        __syncthreads();
        const uint32_t it = s_item;
        if (it >= total) break;
        const int pi = (int)(it / a.nitems);
        const KItem item = a.items[it % a.nitems];
        if (pi != curp) {
            if (curp >= 0) flush(a, curp, acc);
            acc = 0;
            curp = pi;
        }
        gcp<DPlan> P = (gcp<DPlan>)a.plans + pi;
        c.P = P;
        const DLevel L = gload(&P->lev[1]);
        const uint32_t r = item.r0;
        if (P->lev[0].label >= 0 && G.lab[r] != (uint8_t)P->lev[0].label) continue;
        c.v[0] = r;
        uint32_t blo, bhi, lo, hi;
        bounds_of(c.v, P->bridge_gt, P->bridge_lt, blo, bhi);
        bounds_of(c.v, L.gt, L.lt, lo, hi);
        if (blo >= bhi || lo >= hi) continue;
        // item slice s0 of s1: the matching fraction of the target id range
        {
            const uint64_t t0 = lo, t1 = hi == NOB ? (uint64_t)a.g.n : (uint64_t)hi, span = t1 - t0;
            const uint64_t ns = max(item.s1, 1u);
            lo = (uint32_t)(t0 + span * item.s0 / ns);
            hi = (uint32_t)(t0 + span * (item.s0 + 1) / ns);
            if (lo >= hi) continue;
        }
        const uint32_t top = hi;
        uint32_t bb, be;
        list_range(G, r, blo, bhi, bb, be);
        const uint32_t nb = be - bb;
        if (BYTES && tid == 0 && item.s0 == 0) c.bytes += 8 + 4ull * nb;
        // bridge set-up: the cursor starts at the first target >= lo; the
        // end is the end of the list (targets at or above `top` end the
        // bridge when they come up as its next target)
        uint32_t mine = NOB;
        for (uint32_t k = tid; k < nb; k += AW_THREADS) {
            const uint32_t y = G.col[bb + k];
            const bool ok = y != r && (P->bridge_label < 0 || G.lab[y] == (uint8_t)P->bridge_label);
            uint32_t yb = 0, yf = 0, x = NOB, xl = 0;
            if (ok) {
                const uint32_t s = G.rp[y];
                yf = G.rp[y + 1];
                yb = lo == 0 ? s : lower_bound_u32(G.col, s, yf, lo);
                if (yb < yf) {
                    x = G.col[yb];
                    xl = G.col[yf - 1];
                    if (x >= top) x = NOB;
                }
                if (BYTES) c.bytes += 8 + 4ull * (lower_bound_u32(G.col, yb, yf, top) - yb);
            }
            cur[k] = yb;
            fin[k] = yf;
            nxt[k] = x;
            lst[k] = xl;
            mine = min(mine, x);
        }
        for (int off = 32; off >= 1; off >>= 1) mine = min(mine, (uint32_t)__shfl_xor(mine, off));
        if (lane == 0 && mine != NOB) atomicMin(&s_next[0], mine);
        __syncthreads();
        uint32_t vv[KMAX];
#pragma unroll
        for (int i = 0; i < KMAX; ++i) vv[i] = c.v[i];
        int ph = 0;
        for (;;) {
            const uint32_t wlo = s_next[ph];
            if (wlo == NOB || wlo >= top) break;
            const uint32_t whi = (uint32_t)min((uint64_t)top, (uint64_t)wlo + WIN_IDS);
            // a window target: count it; its first touch marks its group
            auto take = [&](uint32_t x) {
                if ((L.label >= 0 && G.lab[x] != (uint8_t)L.label) || ((L.neq & 1) && x == r)) return;
                const uint32_t off = x - wlo;
                bool first;
                if (H16) {
                    const uint32_t sh = (off & 1u) * 16;
                    first = ((atomicAdd(&win[off >> 1], 1u << sh) >> sh) & 0xffffu) == 0u;
                } else {
                    first = atomicAdd(&win[off], 1u) == 0u;
                }
                if (first) {
                    const uint32_t g = off >> 6, bit = 1u << (g & 31);
                    if (!(gbits[g >> 5] & bit) && !(atomicOr(&gbits[g >> 5], bit) & bit))
                        glist[atomicAdd(&s_ng[ph], 1u)] = (uint16_t)g;
                }
            };
            // fill
            mine = NOB;
            for (;;) {
                uint32_t kb = 0;
                if (lane == 0) kb = atomicAdd(&s_batch, 64u);
                kb = __shfl(kb, 0);
                if (kb >= nb) break;
                const uint32_t k = kb + lane;
                const bool valid = k < nb;
                const uint32_t x0 = valid ? nxt[k] : NOB;
                const uint32_t q = valid ? cur[k] : 0u, qe = valid ? fin[k] : 0u;
                // the whole rest of the list lies in the window when its last
                // entry does; else gallop to the window's end
                const uint32_t qend = x0 >= whi ? q : (lst[k] < whi ? qe : gallop_u32(G.col, q, qe, whi));
                const uint32_t len = qend - q;
                // long segments (most of the entries: hub bridges) are cut
                // into chunks that every wave of the workgroup streams after
                // the batches are taken, each chunk by a whole wave with
                // coalesced reads and no search for an entry's owner; when
                // the chunk queue is full the wave streams them itself
                uint64_t longm = __ballot(len >= AW_LONG);
                if (longm) {
                    const uint32_t nck = len >= AW_LONG ? (len + AW_CHUNK - 1) / AW_CHUNK : 0u;
                    const uint32_t cincl = wave_incl_scan(nck);
                    const uint32_t ctot = __shfl(cincl, 63);
                    uint32_t cbase = 0;
                    if (lane == 0) cbase = atomicAdd(&s_nck, ctot);
                    cbase = __shfl(cbase, 0);
                    if (cbase + ctot <= AW_CQCAP) {
                        for (uint32_t i = 0; i < nck; ++i) {
                            const uint32_t slot = cbase + cincl - nck + i;
                            cq_q[slot] = q + i * AW_CHUNK;
                            cq_n[slot] = (uint16_t)min(AW_CHUNK, len - i * AW_CHUNK);
                        }
                        longm = 0;
                    } else {
                        for (uint32_t i = lane; i < ctot && cbase + i < AW_CQCAP; i += 64) cq_n[cbase + i] = 0;
                    }
                }
                while (longm) {
                    const int o = __builtin_ctzll(longm);
                    longm &= longm - 1;
                    const uint32_t qo = __builtin_amdgcn_readlane(q, o), lo_len = __builtin_amdgcn_readlane(len, o);
                    for (uint32_t tb = 0; tb < lo_len; tb += 64 * AW_UNROLL) {
                        // every lane loads (a clamped index past the end
                        // re-reads the last entry), so no load is predicated
                        uint32_t xs[AW_UNROLL];
#pragma unroll
                        for (int u = 0; u < AW_UNROLL; ++u)
                            xs[u] = G.col[qo + min(tb + (uint32_t)(u * 64) + lane, lo_len - 1u)];
#pragma unroll
                        for (int u = 0; u < AW_UNROLL; ++u)
                            if (tb + (uint32_t)(u * 64) + lane < lo_len) take(xs[u]);
                    }
                }
                // short segments: flattened over the lanes
                const uint32_t slen = len >= AW_LONG ? 0u : len;
                const uint32_t incl = wave_incl_scan(slen);
                const uint32_t tot = __shfl(incl, 63);
                const uint32_t excl = incl - slen;
                for (uint32_t tb = 0; tb < tot; tb += 64 * AW_UNROLL) {
                    uint32_t xs[AW_UNROLL];
#pragma unroll
                    for (int u = 0; u < AW_UNROLL; ++u) {
                        const uint32_t t = tb + (uint32_t)(u * 64) + lane;
                        const bool act = t < tot;
                        const int o = owner_of(incl, act ? t : tot - 1);
                        const uint32_t src = __shfl(q, o) + (t - __shfl(excl, o));
                        xs[u] = act ? G.col[src] : NOB;
                    }
#pragma unroll
                    for (int u = 0; u < AW_UNROLL; ++u)
                        if (xs[u] != NOB) take(xs[u]);
                }
                if (valid) {
                    uint32_t xn = !len ? x0 : (qend < qe ? G.col[qend] : NOB);
                    if (xn >= top) xn = NOB;
                    if (len) {
                        cur[k] = qend;
                        nxt[k] = xn;
                    }
                    mine = min(mine, xn);
                }
            }
            for (int off = 32; off >= 1; off >>= 1) mine = min(mine, (uint32_t)__shfl_xor(mine, off));
            if (lane == 0 && mine != NOB) atomicMin(&s_next[ph ^ 1], mine);
            __syncthreads();
            // every wave streams queued chunks until none is left
            {
                const uint32_t nck = min(s_nck, AW_CQCAP);
                for (;;) {
                    uint32_t ci = 0;
                    if (lane == 0) ci = atomicAdd(&s_ckhead, 1u);
                    ci = __shfl(ci, 0);
                    if (ci >= nck) break;
                    const uint32_t qo = cq_q[ci], cn = cq_n[ci];
                    for (uint32_t tb = 0; tb < cn; tb += 64 * AW_UNROLL) {
                        uint32_t xs[AW_UNROLL];
#pragma unroll
                        for (int u = 0; u < AW_UNROLL; ++u)
                            xs[u] = G.col[qo + min(tb + (uint32_t)(u * 64) + lane, cn - 1u)];
#pragma unroll
                        for (int u = 0; u < AW_UNROLL; ++u)
                            if (tb + (uint32_t)(u * 64) + lane < cn) take(xs[u]);
                    }
                }
            }
            __syncthreads();
            const uint32_t ng = s_ng[ph];
            if (tid == 0) {
                s_next[ph] = NOB;   // read by every thread before the barrier
                s_ng[ph ^ 1] = 0;   // next window's group count; last read a window ago
                s_batch = 0;        // every wave has left the fill
                s_nck = s_ckhead = 0;
            }
            for (uint32_t i = tid; i < NGROUPS / 32; i += AW_THREADS) gbits[i] = 0;
            // evaluate: walk the marked groups, clear their counters, queue
            // the touched targets, evaluate 64 at a time
            uint32_t qn = 0;
            for (uint32_t gi = w; gi < ng; gi += AW_WAVES) {
                const uint32_t off = ((uint32_t)glist[gi] << 6) + (uint32_t)lane;
                uint32_t m;
                if (H16) {
                    m = (win[off >> 1] >> ((off & 1u) * 16)) & 0xffffu;
                    __builtin_amdgcn_wave_barrier();
                    if (!(off & 1u)) win[off >> 1] = 0u;
                } else {
                    m = win[off];
                    win[off] = 0u;
                }
                const uint64_t mask = __ballot(m != 0u);
                if (m) {
                    const uint32_t pos = qn + lane_prefix(mask);
                    qoff[w][pos] = (uint16_t)off;
                    qm[w][pos] = m;
                }
                qn += (uint32_t)__popcll(mask);
                if (qn >= 64) {
                    __builtin_amdgcn_wave_barrier();
                    const uint32_t eo = qoff[w][lane], em = qm[w][lane];
                    const uint32_t rest = qn - 64;
                    uint32_t ro = 0, rm = 0;
                    if ((uint32_t)lane < rest) {
                        ro = qoff[w][64 + lane];
                        rm = qm[w][64 + lane];
                    }
                    __builtin_amdgcn_wave_barrier();
                    if ((uint32_t)lane < rest) {
                        qoff[w][lane] = (uint16_t)ro;
                        qm[w][lane] = rm;
                    }
                    qn = rest;
                    vv[1] = wlo + eo;
                    acc += lanes_tail<BYTES, true>(c, vv, true, em);
                }
            }
            if (qn) {
                __builtin_amdgcn_wave_barrier();
                const bool act = (uint32_t)lane < qn;
                const uint32_t eo = act ? qoff[w][lane] : 0u, em = act ? qm[w][lane] : 0u;
                vv[1] = wlo + eo;
                acc += lanes_tail<BYTES, true>(c, vv, act, em);
            }
            __syncthreads();
            ph ^= 1;
        }
    }
    if (curp >= 0) flush(a, curp, acc);
    if (BYTES) {
        unsigned long long bsum = c.bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (lane == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

// ---------------------------------------------------------------- heavy edge-core roots

// Plans with an edge core (v1 in N(v0)) whose set-size terms all intersect
// N(v0) and N(v1) (the diamond's t = |N(v0) n N(v1)|).  For a root with a
// large two-hop mass one workgroup takes the root: threads own level-1
// candidates v1 and walk N(v1) with a cursor while the workgroup sweeps
// N(v0) in windows of EW_BITS ids held as an LDS bitmap; every hit is
// checked against each term's bounds, label and exclusions and counted per
// candidate.  Each thread then evaluates the tail of its own candidates.
// Scratch per block: cursor, end and EW_TERMS counters per candidate.
constexpr uint32_t EW_BITS = 262144;
constexpr uint32_t EW_WORDS = EW_BITS / 32;

template <bool BYTES>
__global__ void __launch_bounds__(256) edge_window_kernel(KArgs a) {
    __shared__ uint32_t bits[EW_WORDS];
    __shared__ uint32_t s_item;
    const int lane = wave_lane();
    const uint32_t tid = threadIdx.x;
    Ctx c;
    c.g = dgraph(a.g);
    c.stride = a.buf_stride;
    c.buf = nullptr;
    c.bytes = 0;
    c.bmw = nullptr;
    c.bm = nullptr;
    const uint64_t ws = a.wscr_stride;
    uint32_t* ccur = a.wscr + (uint64_t)blockIdx.x * (2 + EW_TERMS) * ws;
    uint32_t* cend = ccur + ws;
    uint32_t* ccnt = cend + ws;   // EW_TERMS * ws, candidate-major
    for (uint32_t i = tid; i < EW_WORDS; i += blockDim.x) bits[i] = 0;
    int curp = -1;
    u128 acc = 0;
    const uint64_t total = (uint64_t)a.nplans * a.nitems;
    for (;;) {
        __syncthreads();
        if (tid == 0) {
            uint32_t it = atomicAdd(a.head, 1u);
            if (a.cancel && __atomic_load_n(a.cancel, __ATOMIC_RELAXED)) it = 0xffffffffu;
            s_item = it;
        }
        __syncthreads();
        const uint32_t it = s_item;
        if (it >= total) break;
        const int pi = (int)(it / a.nitems);
        const KItem item = a.items[it % a.nitems];
        if (pi != curp) {
            if (curp >= 0) flush(a, curp, acc);
            acc = 0;
            curp = pi;
        }
        gcp<DPlan> P = (gcp<DPlan>)a.plans + pi;
        c.P = P;
        const DLevel L1 = gload(&P->lev[1]);
        const uint32_t r = item.r0;
        if (P->lev[0].label >= 0 && a.g.lab[r] != (uint8_t)P->lev[0].label) continue;
        c.v[0] = r;
        uint32_t lo1, hi1, cb, ce;
        bounds_of(c.v, L1.gt, L1.lt, lo1, hi1);
        if (lo1 >= hi1) continue;
        list_range(c.g, r, lo1, hi1, cb, ce);
        // item: candidates [s0, s1) of the root's level-1 range
        if (item.s0 >= ce - cb) continue;
        ce = min(ce, cb + item.s1);
        cb += item.s0;
        const uint32_t nb = ce - cb;
        // non-cheap terms of the plan, in order (at most EW_TERMS)
        int tq[EW_TERMS];
        int nt = 0;
        for (int q = 0; q < P->nterm; ++q)
            if (!P->term[q].cheap && !P->term[q].agg && nt < (int)EW_TERMS) tq[nt++] = q;
        if (BYTES && tid == 0) c.bytes += 8 + 4ull * nb;
        for (uint32_t k = tid; k < nb; k += blockDim.x) {
            const uint32_t v1 = c.g.col[cb + k];
            const bool ok = L1.label < 0 || c.g.lab[v1] == (uint8_t)L1.label;
            ccur[k] = ok ? c.g.rp[v1] : 0u;
            cend[k] = ok ? c.g.rp[v1 + 1] : 0u;
            for (int i = 0; i < nt; ++i) ccnt[(uint64_t)k * EW_TERMS + i] = 0;
            if (BYTES && ok) c.bytes += (uint64_t)nt * (8 + 4ull * (c.g.rp[v1 + 1] - c.g.rp[v1]) + 4ull * (c.g.rp[r + 1] - c.g.rp[r]));
        }
        // windows over N(v0)
        uint32_t pos = c.g.rp[r];
        const uint32_t pend_all = c.g.rp[r + 1];
        while (pos < pend_all) {
            const uint32_t wlo = c.g.col[pos];
            const uint32_t whi = (uint32_t)min((uint64_t)c.g.n, (uint64_t)wlo + EW_BITS);
            const uint32_t pend = lower_bound_u32(c.g.col, pos, pend_all, whi);
            for (uint32_t i = pos + tid; i < pend; i += blockDim.x) {
                const uint32_t o = c.g.col[i] - wlo;
                atomicOr(&bits[o >> 5], 1u << (o & 31));
            }
            __syncthreads();
            // each wave takes 64 candidates at a time and streams their
            // entries inside the window flattened; per-owner counts per term
            // come back through ballot masks
            for (uint32_t kb = (tid & ~63u); kb < nb; kb += blockDim.x) {
                const uint32_t k = kb + lane;
                const uint32_t q = k < nb ? ccur[k] : 0u, qe = k < nb ? cend[k] : 0u;
                const uint32_t v1 = k < nb ? c.g.col[cb + k] : 0u;
                const uint32_t qs = q < qe ? gallop_u32(c.g.col, q, qe, wlo) : q;
                const uint32_t qend = qs < qe ? gallop_u32(c.g.col, qs, qe, whi) : qs;
                const uint32_t len = qend - qs;
                const uint32_t incl = wave_incl_scan(len);
                const uint32_t tot = __shfl(incl, 63);
                const uint32_t excl = incl - len;
                uint32_t add[EW_TERMS] = {0, 0, 0, 0};
                for (uint32_t tb = 0; tb < tot; tb += 64) {
                    const uint32_t t = tb + lane;
                    const bool act = t < tot;
                    const int o = owner_of(incl, act ? t : tot - 1);
                    const uint32_t src = __shfl(qs, o) + (t - __shfl(excl, o));
                    const uint32_t w1 = __shfl(v1, o);
                    const uint32_t x = act ? c.g.col[src] : 0u;
                    const uint32_t off = x - wlo;
                    const bool hit = act && ((bits[off >> 5] >> (off & 31)) & 1u);
                    const uint32_t vv[KMAX] = {r, w1, 0, 0, 0};
                    const uint32_t s0 = max(excl, tb), s1 = min(incl, tb + 64);
                    const uint64_t seg = s0 < s1 ? range_mask(s0 - tb, s1 - tb) : 0ull;
                    for (int i = 0; i < nt; ++i) {
                        const DTerm tt = gload(&P->term[tq[i]]);
                        bool ok = hit;
                        if (ok) {
                            uint32_t lo, hi;
                            bounds_of(vv, tt.gt, tt.lt, lo, hi);
                            ok = x >= lo && x < hi && (tt.label < 0 || c.g.lab[x] == (uint8_t)tt.label) &&
                                 !((tt.neq & 1) && x == r) && !((tt.neq & 2) && x == w1);
                        }
                        const uint64_t m = __ballot(ok);
                        add[i] += (uint32_t)__popcll(m & seg);
                    }
                }
                if (k < nb && q < qe) {
                    ccur[k] = qend;
                    for (int i = 0; i < nt; ++i) ccnt[(uint64_t)k * EW_TERMS + i] += add[i];
                }
            }
            __syncthreads();
            for (uint32_t i = pos + tid; i < pend; i += blockDim.x) bits[(c.g.col[i] - wlo) >> 5] = 0u;
            __syncthreads();
            pos = pend;
        }
        // tails of the owned candidates
        for (uint32_t k = tid; k < nb; k += blockDim.x) {
            if (cend[k] == 0u && ccur[k] == 0u) continue;   // label-filtered candidate
            uint32_t vv[KMAX] = {r, c.g.col[cb + k], 0, 0, 0};
            uint64_t tv[MAX_TERMS];
            int i = 0;
            for (int q = 0; q < P->nterm; ++q) {
                const DTerm t = gload(&P->term[q]);
                if (!t.cheap && !t.agg && i < nt && tq[i] == q) tv[q] = ccnt[(uint64_t)k * EW_TERMS + i++];
                else tv[q] = cheap_term<BYTES>(c, vv, t, 0);
            }
            acc += poly_eval(P, tv);
        }
    }
    if (curp >= 0) flush(a, curp, acc);
    if (BYTES) {
        unsigned long long bsum = c.bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (lane == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

// ---------------------------------------------------------------- triangle-core plans
//
// Plans whose core is a triangle v0 < v1 < v2 (ids in degree order) with v1
// and v2 taken from the root's out-neighbourhood N+(v0), counted as is or
// with degree-type tail terms, and edge-core plans that sum a tail linear in
// the number of triangles closing the edge, run here: every such plan of a
// launch in one pass over the same triangles.  A wavefront takes a root (or a slice of a
// hub root's rows), inserts N+(v0) into an open-addressing hash table in its
// LDS, and streams the rows N+(v1), v1 in N+(v0), flattened over the lanes
// with CQ_UNROLL reads in flight per lane.  An entry y found in the table
// closes the triangle (v0, v1, y): y > v1 because it comes from N+(v1), and
// y is adjacent to v0.  Each triangle is met exactly once, at its lowest
// vertex.  Lookups cost LDS reads only; the rows are the global traffic.
constexpr uint32_t CQ_HASH = 2048;   // slots per wavefront; N+(v0) fills at most half
constexpr uint32_t CQ_EMPTY = 0xffffffffu;
constexpr int CQ_UNROLL = 4;

__device__ __forceinline__ void wave_sync() {
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
}

// Fibonacci hashing onto the 2^11 slots.
__device__ __forceinline__ uint32_t cq_slot(uint32_t x) { return (x * 0x9E3779B1u) >> 21; }

// A slot holds a key in its top 32 - KS bits.  With KS = 10 the low bits
// count the triangles found on the edge (v0, key): at most CQ_SMAX - 1, so
// they never reach the key, and a key stays below CQ_EMPTY >> KS when
// n <= CQ_PACK_MAX.
template <int KS>
__device__ __forceinline__ void cq_insert(uint32_t* H, uint32_t x) {
    uint32_t h = cq_slot(x);
    while (atomicCAS(&H[h], CQ_EMPTY, x << KS) != CQ_EMPTY) h = (h + 1) & (CQ_HASH - 1);
}

// Slot of x, or -1.  The table always holds an empty slot, so a probe for
// an absent key ends.
template <int KS>
__device__ __forceinline__ int cq_find(const uint32_t* H, uint32_t x) {
    uint32_t h = cq_slot(x);
    for (;;) {
        const uint32_t k = H[h];
        if (k == CQ_EMPTY) return -1;
        if ((k >> KS) == x) return (int)h;
        h = (h + 1) & (CQ_HASH - 1);
    }
}

// Slot of a key known to be present.  All keys of the table are removed
// together, so a probe walks past slots other lanes have already emptied
// (an empty slot never holds a key).
template <int KS>
__device__ __forceinline__ uint32_t cq_slot_of(const uint32_t* H, uint32_t x) {
    uint32_t h = cq_slot(x);
    while ((H[h] >> KS) != x) h = (h + 1) & (CQ_HASH - 1);
    return h;
}

// Tail of one plan for the core match (v0, v1, v2) with degrees d0, d1, d2.
// A term over a whole adjacency list whose excluded vertices are all known
// neighbours of its owner is that owner's degree less their number (the
// same value as cheap_term computes); other cheap terms go through
// cheap_term.  The set-size term of an edge-core plan is 1: this triangle's
// share of it (the tail is linear in it).
template <bool BYTES>
__device__ u128 cq_eval(Ctx& c, gcp<DPlan> P, uint32_t v0, uint32_t v1, uint32_t v2, uint32_t d0, uint32_t d1,
                        uint32_t d2) {
    uint64_t tv[CQ_TERMS];
    const uint32_t vv[KMAX] = {v0, v1, v2, 0u, 0u};
#pragma unroll 1
    for (int q = 0; q < P->nterm; ++q) {
        const DTerm t = gload(&P->term[q]);
        const int o = __builtin_ctz((uint32_t)t.adj);
        if (!t.cheap) {
            tv[q] = 1;
        } else if ((t.gt | t.lt) == 0 && (t.neq & ~t.sure) == 0) {
            const uint32_t d = o == 0 ? d0 : (o == 1 ? d1 : d2);
            tv[q] = (uint64_t)(d - (uint32_t)__builtin_popcount((uint32_t)t.neq));
            if (BYTES) c.bytes += 8;
        } else {
            tv[q] = cheap_term<BYTES>(c, vv, t, 0);
        }
    }
    i128 s = 0;
    for (int m = 0; m < P->nmono; ++m) {
        const DMono M = gload(&P->mono[m]);
        i128 prod = (i128)M.coef;
        for (int f = 0; f < M.nf; ++f) prod *= (i128)tv[M.f[f]];
        s += prod;
    }
    return s > 0 ? (u128)s : (u128)0;
}

// What one plan adds for the triangle a < b < c of this lane, with degrees
// da, db, dc.  Per lane, no cross-lane reads.  A triangle-core plan
// takes it as its core match.  An edge-core plan sums over edges (v0, v1)
// in the orientation of its level 1 the tail of every common neighbour
// within its set-size term's bounds, so each of the triangle's three edges
// adds its tail when the opposite vertex is within those bounds.
template <bool BYTES>
__device__ __forceinline__ u128 cq_tail(Ctx& c, gcp<DPlan> P, uint32_t a, uint32_t b, uint32_t cc, uint32_t da,
                                        uint32_t db, uint32_t dc) {
    if (P->nterm == 0) return (u128)(uint32_t)P->mult;
    uint8_t hg = 0, hl = 0;
    for (int q = 0; q < P->nterm; ++q)
        if (!P->term[q].cheap) {
            hg = P->term[q].gt;
            hl = P->term[q].lt;
        }
    const bool tri = P->ncore == 3;
    const bool up = P->lev[1].gt != 0;
    u128 s = 0;
#pragma unroll 1
    for (int e = 0; e < (tri ? 1 : 3); ++e) {
        // edge (lo, hi) of the triangle and its opposite vertex x (for a
        // triangle core: the core itself)
        const uint32_t lo = e == 2 ? b : a, hi = e == 0 ? b : cc, x = e == 0 ? cc : (e == 1 ? b : a);
        const uint32_t dlo = e == 2 ? db : da, dhi = e == 0 ? db : dc, dx = e == 0 ? dc : (e == 1 ? db : da);
        const bool fwd = tri || up;
        const uint32_t v0 = fwd ? lo : hi, v1 = fwd ? hi : lo;
        const uint32_t d0 = fwd ? dlo : dhi, d1 = fwd ? dhi : dlo;
        const bool ok = (!(hg & 1) || x > v0) && (!(hg & 2) || x > v1) && (!(hl & 1) || x < v0) &&
                        (!(hl & 2) || x < v1);
        if (ok) s += cq_eval<BYTES>(c, P, v0, v1, x, d0, d1, dx);
    }
    return s;
}

// Triangles found by the stream wait in a per-wavefront LDS queue of
// (v0, v1, v2, deg v1) until 64 are there; then every lane evaluates the
// tails of one, so the tail code runs with all lanes busy.
constexpr uint32_t CQ_QCAP = 128;

template <bool BYTES>
__device__ __forceinline__ void cq_drain(Ctx& c, const KArgs& a, const uint4* Q, uint32_t k, u128* acc) {
    const uint32_t lane = (uint32_t)wave_lane();
    if (lane < k) {
        const uint4 e = Q[lane];
        const uint32_t d0 = a.g.rp[e.x + 1] - a.g.rp[e.x];
        const uint32_t d2 = a.g.rp[e.z + 1] - a.g.rp[e.z];
        if (BYTES) c.bytes += 16;
#pragma unroll 1
        for (int p = 0; p < a.nplans; ++p) {
            const u128 t = cq_tail<BYTES>(c, (gcp<DPlan>)a.plans + p, e.x, e.y, e.z, d0, e.w, d2);
#pragma unroll
            for (int k = 0; k < CQ_PLANS; ++k)
                if (k == p) acc[k] += t;
        }
    }
}

// With supports (MODE 1 or 2) the launch also counts, for every edge
// {u < w}, the triangles on it (its support, at w's place in N+(u)): the
// edge (v1, v2) of a triangle found in row v1 by one returning-free global
// atomic, the edges (v0, v1) and (v0, v2) in LDS (a counter per row of the
// chunk, and one per hash slot: in the slot's low bits for MODE 2, in a
// 16-bit array beside the table for MODE 1), added to the global array once
// per row and root.
template <bool BYTES, int MODE>
__global__ void __launch_bounds__(256) clique_kernel(KArgs a) {
    constexpr bool SUP = MODE != 0;
    constexpr bool SEP = MODE == 1;           // separate slot counters
    constexpr int KS = MODE == 2 ? 10 : 0;    // key shift in a slot
    __shared__ uint32_t s_hash[4][CQ_HASH];
    __shared__ uint4 s_queue[4][CQ_QCAP];
    __shared__ uint32_t s_scnt[SEP ? 4 : 1][SEP ? CQ_HASH / 2 : 1];   // two 16-bit counters a word
    __shared__ uint32_t s_rcnt[SUP ? 4 : 1][64];
    const int lane = wave_lane();
    const int wv = threadIdx.x >> 6;
    uint32_t* H = s_hash[wv];
    uint4* Q = s_queue[wv];
    uint32_t* SC = s_scnt[SEP ? wv : 0];
    uint32_t* RC = s_rcnt[SUP ? wv : 0];
    uint32_t qn = 0;
    for (uint32_t i = lane; i < CQ_HASH; i += 64) H[i] = CQ_EMPTY;
    if (SEP)
        for (uint32_t i = lane; i < CQ_HASH / 2; i += 64) SC[i] = 0;
    if (SUP) RC[lane] = 0;
    wave_sync();
    Ctx c;
    c.g = dgraph(a.g);
    c.P = nullptr;
    c.buf = nullptr;
    c.stride = 0;
    c.bytes = 0;
    c.bmw = nullptr;
    c.bm = nullptr;
    const int np = a.nplans;
    bool counts_only = true;   // every plan counts its triangles: a tally suffices
    for (int p = 0; p < np; ++p) counts_only = counts_only && a.plans[p].nterm == 0;
    u128 acc[CQ_PLANS];
#pragma unroll
    for (int p = 0; p < CQ_PLANS; ++p) acc[p] = 0;
    uint64_t tally = 0;
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(a.head, 1u);
        it = bcast(it);
        if (it >= a.nitems) break;
        if (a.cancel) {
            uint32_t stop = 0;
            if (lane == 0) stop = (uint32_t)__atomic_load_n(a.cancel, __ATOMIC_RELAXED);
            if (bcast(stop)) break;
        }
        const KItem item = a.items[it];
        for (uint32_t r = item.r0; r < item.r1; ++r) {
            const uint32_t b = a.g.split[r], e = a.g.rp[r + 1];
            const uint32_t s = e - b;
            if (s < 2 || s > CQ_SMAX) continue;
            const uint32_t i0 = item.s0, i1 = min(item.s1, s);
            if (i0 >= i1) continue;
            if (BYTES && lane == 0) c.bytes += 12 + 4ull * s;
            for (uint32_t i = lane; i < s; i += 64) cq_insert<KS>(H, a.g.col[b + i]);
            wave_sync();
            for (uint32_t base = i0; base < i1; base += 64) {
                const uint32_t i = base + lane;
                const bool valid = i < i1;
                const uint32_t x = valid ? a.g.col[b + i] : 0u;
                uint32_t pb = 0, len = 0, dx = 0;
                if (valid) {
                    pb = a.g.split[x];
                    const uint32_t xe = a.g.rp[x + 1];
                    len = xe - pb;
                    dx = xe - a.g.rp[x];
                    if (BYTES) c.bytes += 16 + 4ull * len;
                }
                const uint32_t incl = wave_incl_scan(len);
                const uint32_t total = __shfl(incl, 63);
                const uint32_t excl = incl - len;
                for (uint32_t t0 = 0; t0 < total; t0 += 64 * CQ_UNROLL) {
                    uint32_t y[CQ_UNROLL], src[CQ_UNROLL];
                    int o[CQ_UNROLL];
                    bool act[CQ_UNROLL];
#pragma unroll
                    for (int u = 0; u < CQ_UNROLL; ++u) {
                        const uint32_t t = t0 + (uint32_t)(u * 64) + lane;
                        act[u] = t < total;
                        o[u] = owner_of(incl, act[u] ? t : total - 1);
                        src[u] = __shfl(pb, o[u]) + (t - __shfl(excl, o[u]));
                        y[u] = act[u] ? a.g.col[src[u]] : 0u;
                    }
#pragma unroll
                    for (int u = 0; u < CQ_UNROLL; ++u) {
                        const int slot = act[u] ? cq_find<KS>(H, y[u]) : -1;
                        const bool hit = slot >= 0;
                        if (SUP && hit) {
                            atomicAdd(&a.support[src[u]], 1u);
                            atomicAdd(&RC[o[u]], 1u);
                            const uint32_t h = (uint32_t)slot;
                            if (SEP) atomicAdd(&SC[h >> 1], 1u << ((h & 1u) * 16));
                            else atomicAdd(&H[h], 1u);
                        }
                        if (counts_only) {
                            tally += hit ? 1u : 0u;
                            continue;
                        }
                        const uint64_t hm = __ballot(hit);
                        if (hm == 0) continue;
                        const uint32_t xo = __shfl(x, o[u]);
                        const uint32_t dxo = __shfl(dx, o[u]);
                        if (hit) Q[qn + lane_prefix(hm)] = make_uint4(r, xo, y[u], dxo);
                        qn += (uint32_t)__popcll(hm);
                        if (qn >= 64) {
                            wave_sync();
                            cq_drain<BYTES>(c, a, Q, 64, acc);
                            const uint32_t rest = qn - 64;
                            const uint4 t = (uint32_t)lane < rest ? Q[64 + lane] : make_uint4(0u, 0u, 0u, 0u);
                            wave_sync();
                            if ((uint32_t)lane < rest) Q[lane] = t;
                            wave_sync();
                            qn = rest;
                        }
                    }
                }
                if (SUP) {
                    // edges (v0, x) of this chunk's rows
                    wave_sync();
                    const uint32_t k = RC[lane];
                    if (k) {
                        atomicAdd(&a.support[b + i], k);
                        RC[lane] = 0;
                    }
                    wave_sync();
                }
            }
            wave_sync();
            if (SUP) {
                // edges (v0, y) for the y of N+(v0) closing triangles
                for (uint32_t i = lane; i < s; i += 64) {
                    const uint32_t h = cq_slot_of<KS>(H, a.g.col[b + i]);
                    const uint32_t k = SEP ? (SC[h >> 1] >> ((h & 1u) * 16)) & 0xffffu : H[h] & ((1u << KS) - 1);
                    if (k) atomicAdd(&a.support[b + i], k);
                }
                wave_sync();
                if (SEP) {
                    for (uint32_t i = lane; i < s; i += 64) SC[cq_slot_of<KS>(H, a.g.col[b + i]) >> 1] = 0;
                    wave_sync();
                }
            }
            for (uint32_t i = lane; i < s; i += 64) H[cq_slot_of<KS>(H, a.g.col[b + i])] = CQ_EMPTY;
            wave_sync();
        }
    }
    if (qn) {
        wave_sync();
        cq_drain<BYTES>(c, a, Q, qn, acc);
    }
#pragma unroll
    for (int p = 0; p < CQ_PLANS; ++p)
        if (p < np) flush(a, p, counts_only ? (u128)tally * (u128)(uint32_t)a.plans[p].mult : acc[p]);
    if (BYTES) {
        unsigned long long bsum = c.bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (lane == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

// Closed forms summed over the triangles, with the triangle counts of their
// three edges (DPlan::tagg TAGG_DTAIL, TAGG_FAN; the kernel total less
// twelve times the 4-cliques is the count).  Every triangle once, at its
// lowest vertex v0, as in clique_kernel: N+(v0) goes into the wave's LDS
// hash table with each key's position in the list beside it, the rows N+(x)
// of its out-neighbours x are streamed flattened over the lanes, and an
// entry y found in the table closes the triangle (v0, x, y).  The supports
// of (v0, x), (v0, y) and (x, y) sit at x's and y's places in N+(v0) and at
// y's place in N+(x).  Each lane adds its triangles' terms for every plan.
template <bool BYTES>
__global__ void __launch_bounds__(256) trisup_kernel(KArgs a) {
    __shared__ uint32_t s_hash[4][CQ_HASH];
    __shared__ uint16_t s_pos[4][CQ_HASH];
    const int lane = wave_lane();
    const int wv = threadIdx.x >> 6;
    uint32_t* H = s_hash[wv];
    uint16_t* Pos = s_pos[wv];
    for (uint32_t i = lane; i < CQ_HASH; i += 64) H[i] = CQ_EMPTY;
    wave_sync();
    const int np = a.nplans;
    int32_t kind[CQ_PLANS];
#pragma unroll
    for (int p = 0; p < CQ_PLANS; ++p) kind[p] = p < np ? ((gcp<DPlan>)a.plans + p)->tagg : 0;
    u128 acc[CQ_PLANS];
#pragma unroll
    for (int p = 0; p < CQ_PLANS; ++p) acc[p] = 0;
    uint64_t bytes = 0;
    const uint32_t* sup = a.support;
    for (;;) {
        uint32_t it = 0;
        if (lane == 0) it = atomicAdd(a.head, 1u);
        it = bcast(it);
        if (it >= a.nitems) break;
        if (a.cancel) {
            uint32_t stop = 0;
            if (lane == 0) stop = (uint32_t)__atomic_load_n(a.cancel, __ATOMIC_RELAXED);
            if (bcast(stop)) break;
        }
        const KItem item = a.items[it];
        for (uint32_t r = item.r0; r < item.r1; ++r) {
            const uint32_t b = a.g.split[r], e = a.g.rp[r + 1];
            const uint32_t s = e - b;
            if (s < 2 || s > CQ_SMAX) continue;
            const uint32_t i0 = item.s0, i1 = min(item.s1, s);
            if (i0 >= i1) continue;
            const uint32_t d0 = e - a.g.rp[r];
            if (BYTES && lane == 0) bytes += 12 + 4ull * s;
            for (uint32_t i = lane; i < s; i += 64) {
                const uint32_t x = a.g.col[b + i];
                uint32_t h = cq_slot(x);
                while (atomicCAS(&H[h], CQ_EMPTY, x) != CQ_EMPTY) h = (h + 1) & (CQ_HASH - 1);
                Pos[h] = (uint16_t)i;
            }
            wave_sync();
            for (uint32_t base = i0; base < i1; base += 64) {
                const uint32_t i = base + lane;
                const bool valid = i < i1;
                uint32_t pb = 0, len = 0, dx = 0, t0x = 0;
                if (valid) {
                    const uint32_t x = a.g.col[b + i];
                    pb = a.g.split[x];
                    const uint32_t xe = a.g.rp[x + 1];
                    len = xe - pb;
                    dx = xe - a.g.rp[x];
                    t0x = sup[b + i];
                    if (BYTES) bytes += 20 + 4ull * len;
                }
                const uint32_t incl = wave_incl_scan(len);
                const uint32_t total = __shfl(incl, 63);
                const uint32_t excl = incl - len;
                for (uint32_t t0 = 0; t0 < total; t0 += 64) {
                    const uint32_t t = t0 + lane;
                    const bool act = t < total;
                    const int o = owner_of(incl, act ? t : total - 1);
                    const uint32_t src = __shfl(pb, o) + (t - __shfl(excl, o));
                    const uint32_t odx = __shfl(dx, o), ot0x = __shfl(t0x, o);
                    if (!act) continue;
                    const uint32_t y = a.g.col[src];
                    const int slot = cq_find<0>(H, y);
                    if (slot < 0) continue;
                    // the triangle (r, x, y) with its three edge supports
                    const uint64_t t0y = sup[b + Pos[slot]], txy = sup[src];
                    const uint64_t dy = a.g.rp[y + 1] - a.g.rp[y];
                    if (BYTES) bytes += 16;
                    const uint64_t u01 = ot0x - 1, u02 = t0y - 1, u12 = txy - 1;
#pragma unroll
                    for (int p = 0; p < CQ_PLANS; ++p) {
                        if (kind[p] == TAGG_DTAIL)
                            acc[p] += (u128)((uint64_t)(d0 - 2) * u12) + (u128)((uint64_t)(odx - 2) * u02) +
                                      (u128)((dy - 2) * u01);
                        else if (kind[p] == TAGG_FAN)
                            acc[p] += (u128)(u01 * u02) + (u128)(u01 * u12) + (u128)(u02 * u12);
                    }
                }
            }
            wave_sync();
            for (uint32_t i = lane; i < s; i += 64) H[cq_slot_of<0>(H, a.g.col[b + i])] = CQ_EMPTY;
            wave_sync();
        }
    }
#pragma unroll
    for (int p = 0; p < CQ_PLANS; ++p)
        if (p < np) flush(a, p, acc[p]);
    if (BYTES) {
        unsigned long long bsum = bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (lane == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

// Per-vertex support sums: every edge {u < w} adds its support t to both
// ends (a register sum for u, one global atomic for w), so vtri[v] ends at
// twice the triangles through v.  With a.mirror each count is also written
// at u's entry in N(w), so that both ends' lists hold it.
template <bool BYTES>
__global__ void __launch_bounds__(256) vtri_kernel(KArgs a) {
    uint64_t bytes = 0;
    const uint32_t step = gridDim.x * blockDim.x;
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < a.g.n; u += step) {
        const uint32_t pb = a.g.split[u], pe = a.g.rp[u + 1];
        if (BYTES) bytes += 8 + 8ull * (pe - pb);
        uint64_t su = 0;
        for (uint32_t p = pb; p < pe; ++p) {
            const uint32_t t = a.support[p];
            if (t) {
                const uint32_t w = a.g.col[p];
                atomicAdd((unsigned long long*)&a.vtri[w], (unsigned long long)t);
                su += t;
                if (BYTES) bytes += 8;
                if (a.mirror) {
                    // u's entry in the lower part of N(w)
                    const uint32_t q = lower_bound_u32(a.g.col, a.g.rp[w], a.g.split[w], u);
                    a.support[q] = t;
                    if (BYTES) bytes += 12;
                }
            }
        }
        if (su) atomicAdd((unsigned long long*)&a.vtri[u], (unsigned long long)su);
        if (BYTES && su) bytes += 8;
    }
    if (BYTES) {
        unsigned long long bsum = bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (wave_lane() == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

// The triangle-count closed forms (DPlan::tagg) at one vertex u with T(u)
// triangles: the per-vertex part, then the part of each out-edge {u < w}
// with support t.  Sums wrap modulo 2^128 (the plan's total is a count,
// never negative, so the wrapped partial sums add up to it exactly).
__device__ __forceinline__ u128 tagg_vertex(int32_t kind, uint64_t Tu) {
    if (kind == TAGG_BOWTIE) return ((u128)Tu * (u128)(Tu ? Tu - 1 : 0)) >> 1;
    return 0;
}
__device__ __forceinline__ u128 tagg_edge(int32_t kind, uint64_t Tu, uint64_t Tw, uint32_t du, uint32_t dw,
                                          uint32_t t) {
    const u128 pairs = (u128)t * (u128)(t ? t - 1 : 0);   // t (t - 1)
    if (kind == TAGG_BOWTIE) return (u128)0 - pairs;
    if (kind == TAGG_HOUSE) return (u128)0 - 2 * pairs;
    // an edge on a triangle has both ends of degree 2 or more
    if (kind == TAGG_TAILED) return t ? (u128)t * (u128)(du + dw - 4) : (u128)0;
    if (kind == TAGG_TRIANGLE) return (u128)t;
    if (kind != TAGG_TRIPATH) return 0;   // summed elsewhere (trisup_kernel, k4ear_kernel)
    // TAGG_TRIPATH: apex u with path vertex w, then apex w with path vertex u
    const u128 fwd = (u128)(Tu - t) * (u128)(dw - 1) + (u128)(Tw - t) * (u128)(du - 1);
    return fwd - 2 * pairs;
}

// Edge-support plans, and edge-core plans with cheap terms only (then
// without a support array): one thread per vertex u walks its out-list;
// each edge {u < w} takes its support t, orients itself as the plan's
// level 1 requires, and adds the tail with the set-size term equal to t.
// Plans with a triangle-count closed form add their per-vertex and per-edge
// parts.  The supports stay as they are (every replay clears them first).
template <bool BYTES>
__global__ void __launch_bounds__(256) support_kernel(KArgs a) {
    const int np = a.nplans;
    Ctx c;
    c.g = dgraph(a.g);
    c.P = nullptr;
    c.buf = nullptr;
    c.stride = 0;
    c.bytes = 0;
    c.bmw = nullptr;
    c.bm = nullptr;
    u128 acc[CQ_PLANS];
#pragma unroll
    for (int p = 0; p < CQ_PLANS; ++p) acc[p] = 0;
    const uint32_t step = gridDim.x * blockDim.x;
    for (uint32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < a.g.n; u += step) {
        const uint32_t pb = a.g.split[u], pe = a.g.rp[u + 1];
        const uint32_t du = pe - a.g.rp[u];
        if (BYTES) c.bytes += 12 + 8ull * (pe - pb);
        const uint64_t Tu = a.vtri ? a.vtri[u] >> 1 : 0;
        if (a.vtri) {
            if (BYTES) c.bytes += 8;
#pragma unroll 1
            for (int q = 0; q < np; ++q) {
                const int32_t kind = ((gcp<DPlan>)a.plans + q)->tagg;
                if (!kind) continue;
                const u128 add = tagg_vertex(kind, Tu);
#pragma unroll
                for (int k = 0; k < CQ_PLANS; ++k)
                    if (k == q) acc[k] += add;
            }
        }
        for (uint32_t p = pb; p < pe; ++p) {
            const uint32_t w = a.g.col[p];
            // an edge on no triangle still adds the tail's terms without t
            const uint32_t t = a.support ? a.support[p] : 0u;
            const uint32_t dw = a.g.rp[w + 1] - a.g.rp[w];
            if (BYTES) c.bytes += 8;
            const uint64_t Tw = a.vtri ? a.vtri[w] >> 1 : 0;
            if (BYTES && a.vtri) c.bytes += 8;
#pragma unroll 1
            for (int q = 0; q < np; ++q) {
                gcp<DPlan> P = (gcp<DPlan>)a.plans + q;
                if (P->tagg) {
                    const u128 add = tagg_edge(P->tagg, Tu, Tw, du, dw, t);
#pragma unroll
                    for (int k = 0; k < CQ_PLANS; ++k)
                        if (k == q) acc[k] += add;
                    continue;
                }
                const bool up = P->lev[1].gt != 0;
                const uint32_t v0 = up ? u : w, v1 = up ? w : u;
                const uint32_t d0 = up ? du : dw, d1 = up ? dw : du;
                uint64_t tv[CQ_TERMS];
                const uint32_t vv[KMAX] = {v0, v1, 0u, 0u, 0u};
#pragma unroll 1
                for (int k = 0; k < P->nterm; ++k) {
                    const DTerm T = gload(&P->term[k]);
                    if (!T.cheap) tv[k] = t;
                    else if ((T.gt | T.lt) == 0 && (T.neq & ~T.sure) == 0)
                        tv[k] = (uint64_t)((__builtin_ctz((uint32_t)T.adj) == 0 ? d0 : d1) -
                                           (uint32_t)__builtin_popcount((uint32_t)T.neq));
                    else tv[k] = cheap_term<BYTES>(c, vv, T, 0);
                }
                i128 sum = 0;
                for (int m = 0; m < P->nmono; ++m) {
                    const DMono M = gload(&P->mono[m]);
                    i128 prod = (i128)M.coef;
                    for (int f = 0; f < M.nf; ++f) prod *= (i128)tv[M.f[f]];
                    sum += prod;
                }
                const u128 add = sum > 0 ? (u128)sum : (u128)0;
#pragma unroll
                for (int k = 0; k < CQ_PLANS; ++k)
                    if (k == q) acc[k] += add;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < CQ_PLANS; ++p)
        if (p < np) flush(a, p, acc[p]);
    if (BYTES) {
        unsigned long long bsum = c.bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (wave_lane() == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

// ---------------------------------------------------------------- 4-clique plans
//
// A 4-clique v0 < v1 < v2 < v3 lies in N+(v0): v1 < v2 < v3 is a triangle of
// the graph induced on the root's out-neighbourhood.  For each root this
// kernel builds that graph as bit rows in LDS (row i holds the later
// out-neighbours j > i adjacent to the i-th, found by streaming N+(x_i)
// against a hash of N+(v0) that maps an id to its position), then counts
// its triangles: every bit (i, j) adds the popcount of row i AND row j.
// Light roots (3 .. C4_LIGHT out-neighbours) take one wavefront each,
// heavier ones (up to C4_ROOT_MAX) a whole workgroup, in a 44 KB table up to
// C4_HEAVY and a 152 KB one above; larger roots run in the general kernel.
constexpr uint32_t C4_LIGHT = C4_LIGHT_MAX;
constexpr uint32_t C4_HEAVY = C4_HEAVY_MAX;
constexpr uint32_t C4_LDS_WORDS = 11264;   // 44 KB: a workgroup's table for up to 512 out-neighbours
// 152 KB: 4096 keys, 4096 positions, 1024 rows of 32 words (one workgroup a CU)
constexpr uint32_t C4_HUGE_WORDS = 4096 + 2048 + 1024 * 32;
// a wavefront's table for up to 128: 256 keys, 256 positions, 128 rows of 4 words
constexpr uint32_t C4_WAVE_WORDS = 256 + 128 + 128 * 4;

// LDS layout of one root's table: keys[H], positions (u16)[H], rows[S * W].
template <int LOGH>
struct C4Table {
    uint32_t* keys;
    uint16_t* pos;
    uint32_t* rows;
    __device__ C4Table(uint32_t* base) {
        keys = base;
        pos = (uint16_t*)(base + (1u << LOGH));
        rows = base + (1u << LOGH) + (1u << LOGH) / 2;
    }
    __device__ static uint32_t slot(uint32_t x) { return (x * 0x9E3779B1u) >> (32 - LOGH); }
    __device__ void insert(uint32_t x, uint32_t i) {
        uint32_t h = slot(x);
        while (atomicCAS(&keys[h], CQ_EMPTY, x) != CQ_EMPTY) h = (h + 1) & ((1u << LOGH) - 1);
        pos[h] = (uint16_t)i;
    }
    // position of x in N+(v0), or -1; the table always has an empty slot
    __device__ int find(uint32_t x) const {
        uint32_t h = slot(x);
        for (;;) {
            const uint32_t k = keys[h];
            if (k == x) return pos[h];
            if (k == CQ_EMPTY) return -1;
            h = (h + 1) & ((1u << LOGH) - 1);
        }
    }
};

// One root's 4-cliques by NT cooperating threads: a wavefront (NT = 64) or
// the whole workgroup (`sync` is then __syncthreads, otherwise a wavefront
// barrier).  Returns this thread's share.  With SUP the row stream also
// fills the edge supports of every triangle {r < x < y} it meets (the
// triangles at their lowest vertex, each once): (x, y) by a global atomic
// at y's place in N+(x); (r, x) and (r, y) once per root from the row's
// popcount and a per-position LDS counter `pc` (s words).
template <int LOGH, bool WG, bool BYTES, uint32_t NT, bool SUP>
__device__ uint64_t c4_root(Ctx& c, const KGraph& g, uint32_t* base, uint32_t r, uint32_t b, uint32_t s,
                            uint32_t* sup, uint32_t* pc) {
    const uint32_t tid = WG ? threadIdx.x : (uint32_t)wave_lane();
    auto sync = [] {
        if (WG) __syncthreads();
        else wave_sync();
    };
    C4Table<LOGH> T(base);
    const uint32_t W = (s + 31) >> 5;
    for (uint32_t i = tid; i < (1u << LOGH); i += NT) T.keys[i] = CQ_EMPTY;
    for (uint32_t i = tid; i < s * W; i += NT) T.rows[i] = 0;
    if (SUP)
        for (uint32_t i = tid; i < s; i += NT) pc[i] = 0;
    sync();
    for (uint32_t i = tid; i < s; i += NT) T.insert(g.col[b + i], i);
    if (BYTES && tid == 0) c.bytes += 12 + 4ull * s;
    sync();
    // rows: wavefront w of the group streams row chunks w, w + NT/64, ...
    const int lane = wave_lane();
    const uint32_t wv = WG ? (threadIdx.x >> 6) : 0;
    for (uint32_t base_i = wv * 64; base_i < s; base_i += NT) {
        const uint32_t i = base_i + lane;
        const bool valid = i < s;
        const uint32_t x = valid ? g.col[b + i] : 0u;
        uint32_t pb = 0, len = 0;
        if (valid) {
            pb = g.split[x];
            len = g.rp[x + 1] - pb;
            if (BYTES) c.bytes += 12 + 4ull * len;
        }
        const uint32_t incl = wave_incl_scan(len);
        const uint32_t total = __shfl(incl, 63);
        const uint32_t excl = incl - len;
        for (uint32_t t0 = 0; t0 < total; t0 += 64 * CQ_UNROLL) {
            uint32_t y[CQ_UNROLL], src[CQ_UNROLL];
            int o[CQ_UNROLL];
            bool act[CQ_UNROLL];
#pragma unroll
            for (int u = 0; u < CQ_UNROLL; ++u) {
                const uint32_t t = t0 + (uint32_t)(u * 64) + lane;
                act[u] = t < total;
                o[u] = owner_of(incl, act[u] ? t : total - 1);
                src[u] = __shfl(pb, o[u]) + (t - __shfl(excl, o[u]));
                y[u] = act[u] ? g.col[src[u]] : 0u;
            }
#pragma unroll
            for (int u = 0; u < CQ_UNROLL; ++u) {
                const int j = act[u] ? T.find(y[u]) : -1;
                if (j >= 0) {
                    const uint32_t row = base_i + (uint32_t)o[u];
                    atomicOr(&T.rows[row * W + ((uint32_t)j >> 5)], 1u << (j & 31));
                    if (SUP) {
                        atomicAdd(&sup[src[u]], 1u);
                        atomicAdd(&pc[j], 1u);
                    }
                }
            }
        }
    }
    sync();
    if (SUP) {
        // (r, x_i): the triangles with x_i in the middle (row i's bits) and
        // on top (the rows holding bit i)
        for (uint32_t i = tid; i < s; i += NT) {
            uint32_t k = pc[i];
            for (uint32_t w = 0; w < W; ++w) k += (uint32_t)__popc(T.rows[i * W + w]);
            if (k) atomicAdd(&sup[b + i], k);
        }
    }
    // triangles of the row graph: task (i, w) takes the bits of word w of row i
    uint64_t cnt = 0;
    for (uint32_t t = tid; t < s * W; t += NT) {
        const uint32_t i = t / W, w = t - i * W;
        const uint32_t* ri = T.rows + i * W;
        uint32_t m = ri[w];
        while (m) {
            const uint32_t j = (w << 5) + (uint32_t)__builtin_ctz(m);
            m &= m - 1;
            const uint32_t* rj = T.rows + j * W;
            for (uint32_t w2 = j >> 5; w2 < W; ++w2) cnt += (uint32_t)__popc(ri[w2] & rj[w2]);
        }
    }
    sync();
    return cnt;
}

// MODE 0: wavefront roots; 1: workgroup roots up to C4_HEAVY; 2: workgroup
// roots up to C4_ROOT_MAX.  The 152 KB table of MODE 2 leaves one workgroup
// a CU, so that mode runs C4_HUGE_NT threads a workgroup (rows and row pairs
// of one root spread over more wavefronts); MODE 1 runs C4_HEAVY_NT.
#ifndef PM_C4_HEAVY_NT
#define PM_C4_HEAVY_NT 512
#endif
#ifndef PM_C4_HUGE_NT
#define PM_C4_HUGE_NT 1024
#endif
constexpr uint32_t C4_HEAVY_NT = PM_C4_HEAVY_NT;
constexpr uint32_t C4_HUGE_NT = PM_C4_HUGE_NT;
constexpr uint32_t c4_threads(int mode) { return mode == 2 ? C4_HUGE_NT : (mode == 1 ? C4_HEAVY_NT : 256u); }
// a table's words and the most out-neighbours a root of the mode has (the
// per-position support counters follow the table)
constexpr uint32_t c4_table_words(int mode) {
    return mode == 2 ? C4_HUGE_WORDS : (mode == 1 ? C4_LDS_WORDS : C4_WAVE_WORDS);
}
constexpr uint32_t c4_max_s(int mode) { return mode == 2 ? C4_ROOT_MAX : (mode == 1 ? C4_HEAVY : C4_LIGHT); }

// SUP: also fill the edge supports (a.support) of every triangle at roots
// of 2 .. c4_max_s out-neighbours (the items then hold roots of two).
template <bool BYTES, int MODE, bool SUP>
__global__ void __launch_bounds__(c4_threads(MODE)) clique4_kernel(KArgs a) {
    constexpr bool WG = MODE != 0;
    constexpr uint32_t TW = c4_table_words(MODE) + c4_max_s(MODE);
    __shared__ uint32_t s_lds[WG ? TW : 4 * TW];
    const int lane = wave_lane();
    uint32_t* base = WG ? s_lds : s_lds + (threadIdx.x >> 6) * TW;
    uint32_t* pc = base + c4_table_words(MODE);
    __shared__ uint32_t s_it;
    Ctx c;
    c.g = dgraph(a.g);
    c.P = nullptr;
    c.buf = nullptr;
    c.stride = 0;
    c.bytes = 0;
    c.bmw = nullptr;
    c.bm = nullptr;
    const int np = a.nplans;
    uint64_t cnt = 0;
    for (;;) {
        uint32_t it = 0;
        if (WG) {
            if (threadIdx.x == 0) {
                uint32_t v = atomicAdd(a.head, 1u);
                if (v < a.nitems && a.cancel && __atomic_load_n(a.cancel, __ATOMIC_RELAXED)) v = a.nitems;
                s_it = v;
            }
            __syncthreads();
            it = s_it;
            __syncthreads();
        } else {
            if (lane == 0) {
                it = atomicAdd(a.head, 1u);
                if (it < a.nitems && a.cancel && __atomic_load_n(a.cancel, __ATOMIC_RELAXED)) it = a.nitems;
            }
            it = bcast(it);
        }
        if (it >= a.nitems) break;
        const KItem item = a.items[it];
        for (uint32_t r = item.r0; r < item.r1; ++r) {
            const uint32_t b = a.g.split[r], e = a.g.rp[r + 1];
            const uint32_t s = e - b;
            if (s < (SUP ? 2u : 3u) || s > c4_max_s(MODE)) continue;
            if (MODE == 2) cnt += c4_root<12, true, BYTES, C4_HUGE_NT, SUP>(c, a.g, base, r, b, s, a.support, pc);
            else if (WG) cnt += c4_root<11, true, BYTES, C4_HEAVY_NT, SUP>(c, a.g, base, r, b, s, a.support, pc);
            else cnt += c4_root<8, false, BYTES, 64, SUP>(c, a.g, base, r, b, s, a.support, pc);
        }
    }
#pragma unroll
    for (int p = 0; p < CQ_PLANS; ++p)
        if (p < np) flush(a, p, (u128)cnt * (u128)(uint32_t)a.plans[p].mult);
    if (BYTES) {
        unsigned long long bsum = c.bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (lane == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

// Clears `words` 32-bit words; four at a time (the region is 16-byte
// aligned), then the tail.
__global__ void zero_kernel(uint32_t* p, uint64_t words) {
    const uint64_t quads = words / 4;
    uint4* q = (uint4*)p;
    const uint64_t step = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (uint64_t i = t; i < quads; i += step) q[i] = make_uint4(0u, 0u, 0u, 0u);
    for (uint64_t i = quads * 4 + t; i < words; i += step) p[i] = 0u;
}

int launch_zero(uint32_t* p, uint64_t words, hipStream_t s) {
    int grid = (int)std::min<uint64_t>(1024, (words + 255) / 256);
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(zero_kernel, dim3(grid), dim3(256), 0, s, p, words);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_edge_window(const KArgs& a, int grid, bool count_bytes, hipStream_t s) {
    if (count_bytes)
        hipLaunchKernelGGL(edge_window_kernel<true>, dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(edge_window_kernel<false>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// ---------------------------------------------------------------- hub bitmaps

// One wavefront per hub sets the bits of its adjacency list in its zeroed
// bitmap (lists are sorted, so the lane holding the first entry of a word
// assembles the word and writes it alone).
__global__ void hub_bitmap_kernel(KGraph g, uint32_t* bm, uint32_t hub0, uint32_t words) {
    const int lane = wave_lane();
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    for (uint32_t h = hub0 + blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); h < g.n; h += nw) {
        uint32_t* row = bm + (uint64_t)(h - hub0) * words;
        const uint32_t b = g.rp[h], e = g.rp[h + 1];
        for (uint32_t p = b + lane; p < e; p += 64) {
            const uint32_t x = g.col[p], w = x >> 5;
            if (p == b || (g.col[p - 1] >> 5) != w) {
                uint32_t bits = 0;
                for (uint32_t q = p; q < e; ++q) {
                    const uint32_t y = g.col[q];
                    if ((y >> 5) != w) break;
                    bits |= 1u << (y & 31);
                }
                row[w] = bits;
            }
        }
    }
}

int launch_hub_bitmaps(const KGraph& g, uint32_t* bm, uint32_t hub0, uint32_t words, hipStream_t s) {
    if (hub0 >= g.n) return 0;
    const uint32_t hubs = g.n - hub0;
    const int grid = (int)std::min<uint32_t>(4096, (hubs + 3) / 4);
    hipLaunchKernelGGL(hub_bitmap_kernel, dim3(grid), dim3(256), 0, s, g, bm, hub0, words);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int agg_window_cu_blocks() { return AW_CU_BLOCKS; }

int launch_agg_window(const KArgs& a, int grid, bool count_bytes, hipStream_t s) {
    // path counts are bounded by the largest degree (the adjacency stride)
    const bool h16 = !a.wide && a.wscr_stride <= 0xffffu;
    if (h16) {
        if (count_bytes) hipLaunchKernelGGL((agg_window_kernel<true, true>), dim3(grid), dim3(AW_THREADS), 0, s, a);
        else hipLaunchKernelGGL((agg_window_kernel<false, true>), dim3(grid), dim3(AW_THREADS), 0, s, a);
    } else {
        if (count_bytes) hipLaunchKernelGGL((agg_window_kernel<true, false>), dim3(grid), dim3(AW_THREADS), 0, s, a);
        else hipLaunchKernelGGL((agg_window_kernel<false, false>), dim3(grid), dim3(AW_THREADS), 0, s, a);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_clique(const KArgs& a, int grid, bool count_bytes, hipStream_t s) {
    if (a.support && a.g.n <= CQ_PACK_MAX) {
        if (count_bytes) hipLaunchKernelGGL((clique_kernel<true, 2>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((clique_kernel<false, 2>), dim3(grid), dim3(256), 0, s, a);
    } else if (a.support) {
        if (count_bytes) hipLaunchKernelGGL((clique_kernel<true, 1>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((clique_kernel<false, 1>), dim3(grid), dim3(256), 0, s, a);
    } else {
        if (count_bytes) hipLaunchKernelGGL((clique_kernel<true, 0>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((clique_kernel<false, 0>), dim3(grid), dim3(256), 0, s, a);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_house(const KArgs& a, int grid, bool count_bytes, hipStream_t s) {
    if (count_bytes) hipLaunchKernelGGL(house_kernel<true>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(house_kernel<false>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_trisup(const KArgs& a, int grid, bool count_bytes, hipStream_t s) {
    if (count_bytes) hipLaunchKernelGGL(trisup_kernel<true>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(trisup_kernel<false>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_vtri(const KArgs& a, int grid, bool count_bytes, hipStream_t s) {
    if (count_bytes) hipLaunchKernelGGL(vtri_kernel<true>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(vtri_kernel<false>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_support(const KArgs& a, int grid, bool count_bytes, hipStream_t s) {
    if (count_bytes) hipLaunchKernelGGL(support_kernel<true>, dim3(grid), dim3(256), 0, s, a);
    else hipLaunchKernelGGL(support_kernel<false>, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

// The K4 with an ear on one edge (TAGG_K4EAR): each 4-clique once, at its
// lowest vertex r, as a triangle {i, j, k} of the graph induced on N+(r);
// the count is the sum over the 4-cliques of t(e) - 2 over their six edges
// (the ear's apex is any other common neighbour of the edge).  Per root the
// bit rows are built symmetric (row i holds every out-neighbour of r
// adjacent to x_i), then the rows are streamed again: each edge (i, j) of
// the induced graph, met as x_j in N+(x_i), has lt = |row i AND row j|
// triangles of the induced graph on it and adds
// lt (2 (t(x_i, x_j) - 2) + (t(r, x_i) - 2) + (t(r, x_j) - 2)), which over
// all edges is twice the count (every triangle's vertex terms come from
// two of its edges).  Needs complete supports.
template <int LOGH, bool WG, bool BYTES, uint32_t NT>
__device__ u128 c4_ear_root(Ctx& c, const KGraph& g, uint32_t* base, uint32_t b, uint32_t s,
                            const uint32_t* sup) {
    const uint32_t tid = WG ? threadIdx.x : (uint32_t)wave_lane();
    auto sync = [] {
        if (WG) __syncthreads();
        else wave_sync();
    };
    C4Table<LOGH> T(base);
    const uint32_t W = (s + 31) >> 5;
    for (uint32_t i = tid; i < (1u << LOGH); i += NT) T.keys[i] = CQ_EMPTY;
    for (uint32_t i = tid; i < s * W; i += NT) T.rows[i] = 0;
    sync();
    for (uint32_t i = tid; i < s; i += NT) T.insert(g.col[b + i], i);
    if (BYTES && tid == 0) c.bytes += 12 + 4ull * s;
    sync();
    const int lane = wave_lane();
    const uint32_t wv = WG ? (threadIdx.x >> 6) : 0;
    u128 acc = 0;
#pragma unroll 1
    for (int pass = 0; pass < 2; ++pass) {
        for (uint32_t base_i = wv * 64; base_i < s; base_i += NT) {
            const uint32_t i = base_i + lane;
            const bool valid = i < s;
            const uint32_t x = valid ? g.col[b + i] : 0u;
            uint32_t pb = 0, len = 0, tri = 0;
            if (valid) {
                pb = g.split[x];
                len = g.rp[x + 1] - pb;
                if (pass) tri = sup[b + i];
                if (BYTES) c.bytes += (pass ? 16 : 12) + 4ull * len;
            }
            const uint32_t incl = wave_incl_scan(len);
            const uint32_t total = __shfl(incl, 63);
            const uint32_t excl = incl - len;
            for (uint32_t t0 = 0; t0 < total; t0 += 64) {
                const uint32_t t = t0 + lane;
                const bool act = t < total;
                const int o = owner_of(incl, act ? t : total - 1);
                const uint32_t src = __shfl(pb, o) + (t - __shfl(excl, o));
                const uint32_t ot = __shfl(tri, o);
                if (!act) continue;
                const int j = T.find(g.col[src]);
                if (j < 0) continue;
                const uint32_t row = base_i + (uint32_t)o;
                if (pass == 0) {
                    atomicOr(&T.rows[row * W + ((uint32_t)j >> 5)], 1u << (j & 31));
                    atomicOr(&T.rows[(uint32_t)j * W + (row >> 5)], 1u << (row & 31));
                } else {
                    const uint32_t* ri = T.rows + row * W;
                    const uint32_t* rj = T.rows + (uint32_t)j * W;
                    uint32_t lt = 0;
                    for (uint32_t w = 0; w < W; ++w) lt += (uint32_t)__popc(ri[w] & rj[w]);
                    if (lt) {
                        // an edge on a triangle of the induced graph lies on
                        // two 4-cliques' worth of triangles: every t here is 2+
                        const uint64_t wsum = 2ull * (sup[src] - 2) + (ot - 2) + (sup[b + j] - 2);
                        acc += (u128)((uint64_t)lt * wsum);
                        if (BYTES) c.bytes += 8;
                    }
                }
            }
        }
        sync();
    }
    return acc;
}

template <bool BYTES, int MODE>
__global__ void __launch_bounds__(c4_threads(MODE)) k4ear_kernel(KArgs a) {
    constexpr bool WG = MODE != 0;
    constexpr uint32_t TW = c4_table_words(MODE) + c4_max_s(MODE);
    __shared__ uint32_t s_lds[WG ? TW : 4 * TW];
    const int lane = wave_lane();
    uint32_t* base = WG ? s_lds : s_lds + (threadIdx.x >> 6) * TW;
    __shared__ uint32_t s_it;
    Ctx c;
    c.g = dgraph(a.g);
    c.P = nullptr;
    c.buf = nullptr;
    c.stride = 0;
    c.bytes = 0;
    c.bmw = nullptr;
    c.bm = nullptr;
    u128 acc = 0;
    for (;;) {
        uint32_t it = 0;
        if (WG) {
            if (threadIdx.x == 0) {
                uint32_t v = atomicAdd(a.head, 1u);
                if (v < a.nitems && a.cancel && __atomic_load_n(a.cancel, __ATOMIC_RELAXED)) v = a.nitems;
                s_it = v;
            }
            __syncthreads();
            it = s_it;
            __syncthreads();
        } else {
            if (lane == 0) {
                it = atomicAdd(a.head, 1u);
                if (it < a.nitems && a.cancel && __atomic_load_n(a.cancel, __ATOMIC_RELAXED)) it = a.nitems;
            }
            it = bcast(it);
        }
        if (it >= a.nitems) break;
        const KItem item = a.items[it];
        for (uint32_t r = item.r0; r < item.r1; ++r) {
            const uint32_t b = a.g.split[r], e = a.g.rp[r + 1];
            const uint32_t s = e - b;
            if (s < 3 || s > c4_max_s(MODE)) continue;
            if (MODE == 2) acc += c4_ear_root<12, true, BYTES, C4_HUGE_NT>(c, a.g, base, b, s, a.support);
            else if (WG) acc += c4_ear_root<11, true, BYTES, C4_HEAVY_NT>(c, a.g, base, b, s, a.support);
            else acc += c4_ear_root<8, false, BYTES, 64>(c, a.g, base, b, s, a.support);
        }
    }
    flush(a, 0, acc);
    if (BYTES) {
        unsigned long long bsum = c.bytes;
        for (int off = 32; off >= 1; off >>= 1) bsum += __shfl_xor(bsum, off);
        if (lane == 0) atomicAdd((unsigned long long*)a.bytes, bsum);
    }
}

int launch_k4ear(const KArgs& a, int grid, int mode, bool count_bytes, hipStream_t s) {
    if (mode == 2) {
        if (count_bytes) hipLaunchKernelGGL((k4ear_kernel<true, 2>), dim3(grid), dim3(c4_threads(2)), 0, s, a);
        else hipLaunchKernelGGL((k4ear_kernel<false, 2>), dim3(grid), dim3(c4_threads(2)), 0, s, a);
    } else if (mode == 1) {
        if (count_bytes) hipLaunchKernelGGL((k4ear_kernel<true, 1>), dim3(grid), dim3(c4_threads(1)), 0, s, a);
        else hipLaunchKernelGGL((k4ear_kernel<false, 1>), dim3(grid), dim3(c4_threads(1)), 0, s, a);
    } else {
        if (count_bytes) hipLaunchKernelGGL((k4ear_kernel<true, 0>), dim3(grid), dim3(256), 0, s, a);
        else hipLaunchKernelGGL((k4ear_kernel<false, 0>), dim3(grid), dim3(256), 0, s, a);
    }
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

template <int MODE, bool SUP>
static void launch_c4(const KArgs& a, int grid, bool count_bytes, hipStream_t s) {
    if (count_bytes) hipLaunchKernelGGL((clique4_kernel<true, MODE, SUP>), dim3(grid), dim3(c4_threads(MODE)), 0, s, a);
    else hipLaunchKernelGGL((clique4_kernel<false, MODE, SUP>), dim3(grid), dim3(c4_threads(MODE)), 0, s, a);
}

int launch_clique4(const KArgs& a, int grid, int mode, bool count_bytes, hipStream_t s) {
    const bool sup = a.support != nullptr;
    if (mode == 2) sup ? launch_c4<2, true>(a, grid, count_bytes, s) : launch_c4<2, false>(a, grid, count_bytes, s);
    else if (mode == 1) sup ? launch_c4<1, true>(a, grid, count_bytes, s) : launch_c4<1, false>(a, grid, count_bytes, s);
    else sup ? launch_c4<0, true>(a, grid, count_bytes, s) : launch_c4<0, false>(a, grid, count_bytes, s);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

int launch_cycle5(const KArgs& a, int grid, bool count_bytes, hipStream_t s) {
    if (count_bytes)
        hipLaunchKernelGGL(cycle5_kernel<true>, dim3(grid), dim3(256), 0, s, a);
    else
        hipLaunchKernelGGL(cycle5_kernel<false>, dim3(grid), dim3(256), 0, s, a);
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
