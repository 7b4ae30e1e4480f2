// Labeled 3-edge frequent subgraph mining with minimum-node-image support.
//
// For every edge-induced labeled pattern with three edges (triangle, 3-edge
// path a-b-c-d, 3-star) the MNI support is the smallest, over the pattern's
// vertices, of the number of distinct data vertices that some match maps
// that pattern vertex to (Preliminaries, FSM; domains of symmetric pattern
// vertices coincide).  Domain membership is an existence question, so one
// lane owns one data vertex x and decides, for every pattern and every
// pattern vertex at once, whether a match can place x there:
//
//   * 3-star centre: the neighbour-label histogram of x covers the leaf
//     label multiset.
//   * 3-star leaf: some neighbour c of x (the centre) has, besides x,
//     neighbours covering the other two leaf labels.
//   * path inner vertex b = x: some neighbour c with label lc such that x has
//     a neighbour a != c with label la, c has a neighbour d != x with label
//     ld, and a != d (the one ambiguous case, both witnesses unique and of
//     the same label, is settled by an adjacency test).
//   * path end a = x: some neighbour b and c in N(b)\{x} whose neighbours
//     outside {x, b} include label ld; per vertex b the kernel first tabulates,
//     for every (lc, ld), how many such c exist and how many of them have a
//     single witness, then x subtracts itself and (only when needed) the
//     witnesses it would take away, found by a sorted-list intersection.
//   * triangle: x lies on a triangle whose other two labels are (ly, lz);
//     a pre-pass lists every triangle once from its lowest vertex in the
//     degree order (a hash of the root's out-list in LDS, its rows streamed
//     against it) and records the label pair at each corner.
//
// Each membership increments a per-(pattern, column) counter once per
// vertex, so the counters are the domain sizes.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fsm.hpp"

namespace pm {

__device__ __forceinline__ bool fsm_has(const uint32_t* __restrict__ col, uint32_t lo, uint32_t hi, uint32_t x) {
    const uint32_t end = hi;
    while (lo < hi) {
        uint32_t mid = (lo + hi) >> 1;
        if (col[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < end && col[lo] == x;
}

// ---- per-vertex label histogram and presence masks ----------------------
__global__ void fsm_hist(FsmArgs a) {
    for (uint32_t x = blockIdx.x * blockDim.x + threadIdx.x; x < a.n; x += gridDim.x * blockDim.x) {
        uint32_t h[FSM_LMAX];
        for (int l = 0; l < FSM_LMAX; ++l) h[l] = 0;
        for (uint32_t p = a.rp[x]; p < a.rp[x + 1]; ++p) h[a.lab[a.col[p]]]++;
        uint32_t pm1 = 0, pm2 = 0, pm3 = 0;
        for (int l = 0; l < a.L; ++l) {
            a.hist[(uint64_t)x * FSM_LMAX + l] = h[l];
            if (h[l] >= 1) pm1 |= 1u << l;
            if (h[l] >= 2) pm2 |= 1u << l;
            if (h[l] >= 3) pm3 |= 1u << l;
        }
        for (int w = 0; w < 4; ++w) a.tri[(uint64_t)x * 4 + w] = 0ull;
        a.pres[(uint64_t)x * 3 + 0] = pm1;
        a.pres[(uint64_t)x * 3 + 1] = pm2;
        a.pres[(uint64_t)x * 3 + 2] = pm3;
    }
}

// labels present among N(v) \ {one neighbour carrying label `drop`}
__device__ __forceinline__ uint32_t present_minus(const FsmArgs& a, uint32_t v, int drop) {
    uint32_t p1 = a.pres[(uint64_t)v * 3 + 0], p2 = a.pres[(uint64_t)v * 3 + 1];
    return (p2 >> drop) & 1 ? p1 : (p1 & ~(1u << drop));
}
__device__ __forceinline__ uint32_t twice_minus(const FsmArgs& a, uint32_t v, int drop) {
    uint32_t p2 = a.pres[(uint64_t)v * 3 + 1], p3 = a.pres[(uint64_t)v * 3 + 2];
    return (p3 >> drop) & 1 ? p2 : (p2 & ~(1u << drop));
}

// ---- triangle label pairs ---------------------------------------------------
__device__ __forceinline__ void pair_or(const FsmArgs& a, uint32_t x, int l1, int l2) {
    if (l1 > l2) { int t = l1; l1 = l2; l2 = t; }
    const int bit = l1 * FSM_LMAX + l2;
    atomicOr(&a.tri[(uint64_t)x * 4 + (bit >> 6)], 1ull << (bit & 63));
}

// ---- triangles, each listed once from its lowest vertex u (degree order).
// One wavefront per root: N+(u) goes into an open-addressing hash in LDS
// (Fibonacci hashing, linear probing) and the rows N+(v), v in N+(u), are
// streamed flattened over the lanes (a prefix sum numbers the row entries,
// each lane takes one and finds its row by a shuffle search); an entry w
// found in the table closes (u, v, w).  A root with more than FT_SMAX
// out-neighbours merges its rows instead, one row per lane.
constexpr uint32_t FT_HASH = 2048, FT_SMAX = 1024, FT_EMPTY = 0xffffffffu;

__device__ __forceinline__ uint32_t ft_slot(uint32_t x) { return (x * 0x9E3779B1u) >> 21; }

__device__ __forceinline__ void ft_sync() {
    __threadfence_block();
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ uint32_t ft_scan(uint32_t x) {
    const int lane = __lane_id();
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    return x;
}

// lane whose inclusive prefix range holds entry t (all lanes execute it)
__device__ __forceinline__ int ft_owner(uint32_t incl, uint32_t t) {
    int lo = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1) {
        const uint32_t v = __shfl(incl, lo + step - 1);
        if (v <= t) lo += step;
    }
    return lo;
}

__device__ __forceinline__ void ft_found(const FsmArgs& a, uint32_t u, uint32_t v, uint32_t w) {
    const int lu = a.lab[u], lv = a.lab[v], lw = a.lab[w];
    pair_or(a, u, lv, lw);
    pair_or(a, v, lu, lw);
    pair_or(a, w, lu, lv);
}

__global__ void __launch_bounds__(256) fsm_tri(FsmArgs a) {
    __shared__ uint32_t s_hash[4][FT_HASH];
    const int lane = __lane_id();
    uint32_t* H = s_hash[threadIdx.x >> 6];
    for (uint32_t i = lane; i < FT_HASH; i += 64) H[i] = FT_EMPTY;
    ft_sync();
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    for (uint32_t u = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; u < a.n; u += nw) {
        const uint32_t b = a.split[u], e = a.rp[u + 1], s = e - b;
        if (s < 2) continue;
        if (s > FT_SMAX) {
            for (uint32_t p = b + lane; p < e; p += 64) {
                const uint32_t v = a.col[p];
                uint32_t i = p + 1, j = a.split[v];
                const uint32_t je = a.rp[v + 1];
                while (i < e && j < je) {
                    const uint32_t x = a.col[i], y = a.col[j];
                    if (x == y) {
                        ft_found(a, u, v, x);
                        ++i;
                        ++j;
                    } else if (x < y) {
                        ++i;
                    } else {
                        ++j;
                    }
                }
            }
            continue;
        }
        for (uint32_t i = lane; i < s; i += 64) {
            const uint32_t x = a.col[b + i];
            uint32_t h = ft_slot(x);
            while (atomicCAS(&H[h], FT_EMPTY, x) != FT_EMPTY) h = (h + 1) & (FT_HASH - 1);
        }
        ft_sync();
        for (uint32_t base = 0; base < s; base += 64) {
            const uint32_t i = base + lane;
            const bool valid = i < s;
            const uint32_t v = valid ? a.col[b + i] : 0u;
            const uint32_t pb = valid ? a.split[v] : 0u;
            const uint32_t len = valid ? a.rp[v + 1] - pb : 0u;
            const uint32_t incl = ft_scan(len);
            const uint32_t total = __shfl(incl, 63);
            const uint32_t excl = incl - len;
            for (uint32_t t0 = 0; t0 < total; t0 += 64) {
                const uint32_t t = t0 + lane;
                const bool act = t < total;
                const int o = ft_owner(incl, act ? t : total - 1);
                const uint32_t src = __shfl(pb, o) + (t - __shfl(excl, o));
                const uint32_t vo = __shfl(v, o);
                if (!act) continue;
                const uint32_t w = a.col[src];
                uint32_t h = ft_slot(w);
                for (;;) {
                    const uint32_t k = H[h];
                    if (k == w) {
                        ft_found(a, u, vo, w);
                        break;
                    }
                    if (k == FT_EMPTY) break;
                    h = (h + 1) & (FT_HASH - 1);
                }
            }
        }
        ft_sync();
        // remove the keys (all together: a probe walks past emptied slots)
        for (uint32_t i = lane; i < s; i += 64) {
            const uint32_t x = a.col[b + i];
            uint32_t h = ft_slot(x);
            while (H[h] != x) h = (h + 1) & (FT_HASH - 1);
            H[h] = FT_EMPTY;
        }
        ft_sync();
    }
}

// ---- per vertex b: for every (lc, ld), how many c in N(b) (label lc) have a
// neighbour of label ld outside {b}, and how many of those have exactly one.
// Vertices up to BT_HEAVY neighbours take one thread; larger ones one
// wavefront, whose lanes share N(b) and count in LDS (then saturate).
constexpr uint32_t BT_HEAVY = 256;

__global__ void __launch_bounds__(256) fsm_btab(FsmArgs a) {
    __shared__ uint32_t s_cnt[4][FSM_LMAX * FSM_LMAX], s_frag[4][FSM_LMAX * FSM_LMAX], s_wm[4][FSM_LMAX];
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < a.n; b += gridDim.x * blockDim.x) {
        if (a.rp[b + 1] - a.rp[b] > BT_HEAVY) continue;
        uint8_t* cnt = a.bcnt + (uint64_t)b * FSM_LMAX * FSM_LMAX;
        uint8_t* frag = a.bfrag + (uint64_t)b * FSM_LMAX * FSM_LMAX;
        uint32_t* wm = a.bmask + (uint64_t)b * FSM_LMAX;
        for (int i = 0; i < FSM_LMAX * FSM_LMAX; ++i) {
            cnt[i] = 0;
            frag[i] = 0;
        }
        for (int i = 0; i < FSM_LMAX; ++i) wm[i] = 0;
        const int lb = a.lab[b];
        for (uint32_t p = a.rp[b]; p < a.rp[b + 1]; ++p) {
            const uint32_t c = a.col[p];
            const int lc = a.lab[c];
            uint32_t e = present_minus(a, c, lb);
            wm[lc] |= e;
            while (e) {
                const int ld = __builtin_ctz(e);
                e &= e - 1;
                uint32_t k = a.hist[(uint64_t)c * FSM_LMAX + ld] - (ld == lb ? 1u : 0u);
                uint8_t& cc = cnt[lc * FSM_LMAX + ld];
                if (cc < 255) ++cc;
                if (k == 1) {
                    uint8_t& ff = frag[lc * FSM_LMAX + ld];
                    if (ff < 255) ++ff;
                }
            }
        }
    }
    // heavy vertices: a wavefront each
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    uint32_t* C = s_cnt[wv];
    uint32_t* F = s_frag[wv];
    uint32_t* WM = s_wm[wv];
    for (uint32_t i = lane; i < FSM_LMAX * FSM_LMAX; i += 64) {
        C[i] = 0;
        F[i] = 0;
    }
    if (lane < FSM_LMAX) WM[lane] = 0;
    ft_sync();
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    for (uint32_t b = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; b < a.n; b += nw) {
        const uint32_t pb = a.rp[b], pe = a.rp[b + 1];
        if (pe - pb <= BT_HEAVY) continue;
        const int lb = a.lab[b];
        for (uint32_t p = pb + lane; p < pe; p += 64) {
            const uint32_t c = a.col[p];
            const int lc = a.lab[c];
            uint32_t e = present_minus(a, c, lb);
            if (e) atomicOr(&WM[lc], e);
            while (e) {
                const int ld = __builtin_ctz(e);
                e &= e - 1;
                const uint32_t k = a.hist[(uint64_t)c * FSM_LMAX + ld] - (ld == lb ? 1u : 0u);
                atomicAdd(&C[lc * FSM_LMAX + ld], 1u);
                if (k == 1) atomicAdd(&F[lc * FSM_LMAX + ld], 1u);
            }
        }
        ft_sync();
        uint8_t* cnt = a.bcnt + (uint64_t)b * FSM_LMAX * FSM_LMAX;
        uint8_t* frag = a.bfrag + (uint64_t)b * FSM_LMAX * FSM_LMAX;
        for (uint32_t i = lane; i < FSM_LMAX * FSM_LMAX; i += 64) {
            cnt[i] = (uint8_t)min(C[i], 255u);
            frag[i] = (uint8_t)min(F[i], 255u);
            C[i] = 0;
            F[i] = 0;
        }
        if (lane < FSM_LMAX) {
            a.bmask[(uint64_t)b * FSM_LMAX + lane] = WM[lane];
            WM[lane] = 0;
        }
        ft_sync();
    }
}

// path slot of the ordered label tuple, and the canonical column of position i
__device__ __forceinline__ void p4_where(const FsmArgs& a, int la, int lb, int lc, int ld, int pos, int& slot,
                                         int& colidx) {
    const int L = a.L;
    const int code = a.p4code[((la * L + lb) * L + lc) * L + ld];
    slot = code >> 2;
    const int rev = (code >> 1) & 1, pal = code & 1;
    colidx = rev ? 3 - pos : pos;
    if (pal && colidx >= 2) colidx = 3 - colidx;
}

// column of a vertex of label lx in a sorted label triple: first position
__device__ __forceinline__ int first_pos(int l0, int l1, int l2, int lx) {
    return l0 == lx ? 0 : (l1 == lx ? 1 : 2);
}

__device__ __forceinline__ void sort3(int& l0, int& l1, int& l2) {
    if (l0 > l1) { int t = l0; l0 = l1; l1 = t; }
    if (l1 > l2) { int t = l1; l1 = l2; l2 = t; }
    if (l0 > l1) { int t = l0; l0 = l1; l1 = t; }
}

// The unique neighbour of x with label l other than `skip` (none -> n).
__device__ uint32_t unique_other(const FsmArgs& a, uint32_t x, int l, uint32_t skip) {
    for (uint32_t p = a.rp[x]; p < a.rp[x + 1]; ++p) {
        uint32_t y = a.col[p];
        if (y != skip && a.lab[y] == l) return y;
    }
    return a.n;
}

__device__ __forceinline__ uint64_t wave_or64(uint64_t m) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) m |= __shfl_xor(m, off);
    return m;
}

// Membership sets of one vertex, as 256-bit sets (4 words) per label:
//   region 0  U[lc]: 3-star leaf, centre label lc, bit (l2*16 + l3) = the
//             other two leaf labels (l2 <= l3)
//   region 1  M[lc]: path inner b = x, bit (la*16 + ld) for the path a-x-c-d
//   region 2  V[lb]: path end a = x, bit (lc*16 + ld) for the path x-b-c-d
//   tri:      triangle, bit (l2*16 + l3) = the other two labels (l2 <= l3)
enum { REG_U = 0, REG_M = 1, REG_V = 2 };

__device__ __forceinline__ void where_of(const FsmArgs& a, int reg, int lab, int bit, int lx, int& slot,
                                         int& colidx) {
    const int L = a.L;
    const int hi = bit / FSM_LMAX, lo = bit % FSM_LMAX;
    if (reg == REG_U) {
        int s0 = lx, s1 = hi, s2 = lo;
        sort3(s0, s1, s2);
        slot = a.s3code[((lab * L + s0) * L + s1) * L + s2];
        colidx = 1 + first_pos(s0, s1, s2, lx);
    } else if (reg == REG_M) {
        p4_where(a, hi, lx, lab, lo, 1, slot, colidx);
    } else if (reg == REG_V) {
        p4_where(a, lx, lab, hi, lo, 0, slot, colidx);
    } else {
        int s0 = lx, s1 = hi, s2 = lo;
        sort3(s0, s1, s2);
        slot = a.tricode[(s0 * L + s1) * L + s2];
        colidx = first_pos(s0, s1, s2, lx);
    }
}

// Adds one word of every lane's membership set to the domain counters.  In a
// label-uniform wave the lanes sharing a bit add one popcount with a single
// atomic; otherwise each lane adds its own bits.  Called by all lanes.
__device__ __forceinline__ void emit_word(const FsmArgs& a, uint64_t m, bool uniform, int lx, int reg, int lab,
                                          int w) {
    if (uniform) {
        uint64_t u = wave_or64(m);
        while (u) {
            const int b = __builtin_ctzll(u);
            u &= u - 1;
            const uint64_t who = __ballot((m >> b) & 1ull);
            if (__lane_id() == 0) {
                int slot, colidx;
                where_of(a, reg, lab, (w << 6) + b, lx, slot, colidx);
                atomicAdd(&a.counts[(uint64_t)slot * 4 + colidx], (uint32_t)__popcll(who));
            }
        }
    } else {
        while (m) {
            const int b = __builtin_ctzll(m);
            m &= m - 1;
            int slot, colidx;
            where_of(a, reg, lab, (w << 6) + b, lx, slot, colidx);
            atomicAdd(&a.counts[(uint64_t)slot * 4 + colidx], 1u);
        }
    }
}

__device__ __forceinline__ void set_bit(uint64_t* r, int bit) { r[bit >> 6] |= 1ull << (bit & 63); }
__device__ __forceinline__ bool has_bit(const uint64_t* r, int bit) { return (r[bit >> 6] >> (bit & 63)) & 1ull; }

// Pass-1 contribution of neighbour c of x (label lx): the label pairs
// (l2 <= l3) that c's other neighbours cover, as four 64-bit words of the
// 3-star-leaf set U[lab(c)]; row l2 holds the labels above l2 present in
// N(c) \ {x}, and l2 itself when twice present.
__device__ __forceinline__ void leaf_pairs(uint32_t pr, uint32_t tw, uint64_t& f0, uint64_t& f1, uint64_t& f2,
                                           uint64_t& f3) {
    f0 = f1 = f2 = f3 = 0;
    uint32_t e2 = pr;
    while (e2) {
        const int l2 = __builtin_ctz(e2);
        e2 &= e2 - 1;
        const uint32_t row = (pr & ~((2u << l2) - 1u)) | (tw & (1u << l2));
        const uint64_t sh = (uint64_t)row << ((l2 & 3) * 16);
        const int wd = l2 >> 2;
        f0 |= wd == 0 ? sh : 0ull;
        f1 |= wd == 1 ? sh : 0ull;
        f2 |= wd == 2 ? sh : 0ull;
        f3 |= wd == 3 ? sh : 0ull;
    }
}

// Path-inner row set M[lc] of x: bit (la*16 + ld) when a path a-x-c-d with
// lab(a) = la, lab(c) = lc, lab(d) = ld exists.  pd / t2: labels present once
// / twice among N(c) \ {x}, OR-ed over the neighbours c of label lc.
__device__ void inner_rows(const FsmArgs& a, uint32_t x, int lx, int lc, uint32_t pd, uint32_t t2, uint64_t& m0,
                           uint64_t& m1, uint64_t& m2, uint64_t& m3) {
    const int L = a.L;
    const uint32_t xs = a.rp[x], xe = a.rp[x + 1];
    const uint32_t* hx = a.hist + (uint64_t)x * FSM_LMAX;
    // a: labels of N(x) \ {c} for some c of label lc
    const uint32_t pa = hx[lc] >= 2 ? a.pres[(uint64_t)x * 3] : (a.pres[(uint64_t)x * 3] & ~(1u << lc));
    m0 = m1 = m2 = m3 = 0;
    uint32_t ea = pa & ((1u << L) - 1u);
    while (ea) {
        const int la = __builtin_ctz(ea);
        ea &= ea - 1;
        uint32_t row = pd;   // labels ld of d
        if ((row >> la) & 1) {
            // ld == la needs a != d
            const uint32_t na = hx[la] - (lc == la ? 1u : 0u);
            if (na < 2 && !((t2 >> la) & 1)) {
                // every candidate c has one witness d; x one witness a:
                // valid iff some c (label lc) has its witness d != a
                bool ok = false;
                for (uint32_t p = xs; p < xe && !ok; ++p) {
                    const uint32_t c = a.col[p];
                    if (a.lab[c] != lc) continue;
                    if (!((present_minus(a, c, lx) >> la) & 1)) continue;
                    const uint32_t aa = unique_other(a, x, la, c);
                    if (aa >= a.n) continue;
                    if (!fsm_has(a.col, a.rp[c], a.rp[c + 1], aa)) ok = true;
                }
                if (!ok) row &= ~(1u << la);
            }
        }
        const uint64_t sh = (uint64_t)row << ((la & 3) * 16);
        const int wd = la >> 2;
        m0 |= wd == 0 ? sh : 0ull;
        m1 |= wd == 1 ? sh : 0ull;
        m2 |= wd == 2 ? sh : 0ull;
        m3 |= wd == 3 ? sh : 0ull;
    }
}

// Path end: whether x (label lx) starts a path x-b-c-d through its
// neighbour b (label lb) with lab(c) = lc, lab(d) = ld.  ex: labels present
// among N(x) \ {b}.
__device__ bool end_ok(const FsmArgs& a, uint32_t x, int lx, uint32_t b, int lb, int lc, int ld, uint32_t ex) {
    const int bit = lc * FSM_LMAX + ld;
    const uint32_t cn = a.bcnt[(uint64_t)b * FSM_LMAX * FSM_LMAX + bit];
    const uint32_t fr = a.bfrag[(uint64_t)b * FSM_LMAX * FSM_LMAX + bit];
    const uint32_t self = (lc == lx && ((ex >> ld) & 1)) ? 1u : 0u;
    if (cn < 255 && cn < self + 1) return false;
    if (cn < 255 && cn >= self + 1 + fr) return true;
    if (ld != lx) return cn >= self + 1;
    // exact: c in N(b) \ {x}, label lc, with a label-ld neighbour outside {b, x}
    for (uint32_t q = a.rp[b]; q < a.rp[b + 1]; ++q) {
        const uint32_t c = a.col[q];
        if (c == x || a.lab[c] != lc) continue;
        uint32_t k = a.hist[(uint64_t)c * FSM_LMAX + ld] - (ld == lb ? 1u : 0u);
        if (k >= 1 && fsm_has(a.col, a.rp[c], a.rp[c + 1], x)) --k;
        if (k >= 1) return true;
    }
    return false;
}

// 3-star centre: x's neighbour-label histogram covers the leaf labels
// l1 <= l2 <= l3.
__device__ __forceinline__ bool centre_ok(const uint32_t* hx, int l1, int l2, int l3) {
    const uint32_t n1 = hx[l1], n2 = hx[l2], n3 = hx[l3];
    if (l1 == l3) return n1 >= 3;
    if (l1 == l2) return n1 >= 2 && n3 >= 1;
    if (l2 == l3) return n1 >= 1 && n2 >= 2;
    return n1 >= 1 && n2 >= 1 && n3 >= 1;
}

// Vertices are taken in label order, so most wavefronts hold one label and
// the domain counters see one atomic per (pattern, column) per wavefront.
__global__ void __launch_bounds__(256) fsm_main(FsmArgs a) {
    const int L = a.L;
    const int lane = __lane_id();
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t* U = a.scratch + tid * FSM_SCRATCH_WORDS;   // FSM_LMAX * 4 words each
    uint64_t* M = U + FSM_LMAX * 4;
    uint64_t* V = M + FSM_LMAX * 4;
    for (uint64_t base = tid - lane; base < a.n; base += stride) {   // wave-uniform trip count
        const uint64_t i = base + lane;
        // vertices of degree FSM_HUB or more are left to fsm_hub
        const uint32_t xo = i < a.n ? a.order[i] : 0u;
        const bool act = i < a.n && a.rp[xo + 1] - a.rp[xo] < FSM_HUB;
        const uint32_t x = act ? xo : 0u;
        const int lx = act ? (int)a.lab[x] : -1;
        const uint32_t xs = act ? a.rp[x] : 0u, xe = act ? a.rp[x + 1] : 0u;
        // label-uniform wave: every active lane has the first lane's label
        const int lx0 = __shfl(lx, 0);
        const bool uniform = __ballot(act && lx != lx0) == 0ull;
        const uint32_t* hx = a.hist + (uint64_t)x * FSM_LMAX;
        for (int q = 0; q < FSM_LMAX * 12; ++q) U[q] = 0;
        uint64_t tp[4] = {0, 0, 0, 0};
        if (act && xs != xe) {
            // ---- 3-star leaf and path inner, one pass over N(x) -----------
            uint32_t Pd[FSM_LMAX], T2[FSM_LMAX];
            for (int q = 0; q < FSM_LMAX; ++q) Pd[q] = T2[q] = 0;
            for (uint32_t p = xs; p < xe; ++p) {
                const uint32_t c = a.col[p];
                const int lc = a.lab[c];
                const uint32_t pr = present_minus(a, c, lx), tw = twice_minus(a, c, lx);
                Pd[lc] |= pr;
                T2[lc] |= tw;
                uint64_t f0, f1, f2, f3;
                leaf_pairs(pr, tw, f0, f1, f2, f3);
                uint64_t* u = U + lc * 4;
                if (f0 & ~u[0]) u[0] |= f0;
                if (f1 & ~u[1]) u[1] |= f1;
                if (f2 & ~u[2]) u[2] |= f2;
                if (f3 & ~u[3]) u[3] |= f3;
            }
            for (int lc = 0; lc < L; ++lc) {
                if (!Pd[lc]) continue;
                uint64_t m0, m1, m2, m3;
                inner_rows(a, x, lx, lc, Pd[lc], T2[lc], m0, m1, m2, m3);
                uint64_t* mm = M + lc * 4;
                mm[0] = m0;
                mm[1] = m1;
                mm[2] = m2;
                mm[3] = m3;
            }
            // ---- path end: V[lb] = (lc, ld) reachable from x via b ---------
            for (uint32_t p = xs; p < xe; ++p) {
                const uint32_t b = a.col[p];
                const int lb = a.lab[b];
                const uint32_t* wm = a.bmask + (uint64_t)b * FSM_LMAX;
                const uint32_t ex = present_minus(a, x, lb);  // x as a c-candidate of b
                uint64_t* v = V + lb * 4;
                for (int lc = 0; lc < L; ++lc) {
                    // only the (lc, ld) not yet known reachable
                    const uint32_t known = (uint32_t)((v[lc >> 2] >> ((lc & 3) * 16)) & 0xffffu);
                    uint32_t dm = wm[lc] & ~known;
                    while (dm) {
                        const int ld = __builtin_ctz(dm);
                        dm &= dm - 1;
                        const int bit = lc * FSM_LMAX + ld;
                        const bool ok = end_ok(a, x, lx, b, lb, lc, ld, ex);
                        if (ok) set_bit(v, bit);
                    }
                }
            }
            // ---- triangle: label pairs listed by the pre-pass ---------------
            for (int w = 0; w < 4; ++w) tp[w] = a.tri[(uint64_t)x * 4 + w];
        }
        // ---- 3-star centre: the label histogram covers the leaf multiset --
        const int lxs = uniform ? lx0 : lx;
        for (int l1 = 0; l1 < L; ++l1)
            for (int l2 = l1; l2 < L; ++l2)
                for (int l3 = l2; l3 < L; ++l3) {
                    const bool ok = act && xs != xe && centre_ok(hx, l1, l2, l3);
                    if (uniform) {
                        const uint64_t who = __ballot(ok);
                        if (lane == 0 && who)
                            atomicAdd(&a.counts[(uint64_t)a.s3code[((lxs * L + l1) * L + l2) * L + l3] * 4],
                                      (uint32_t)__popcll(who));
                    } else if (ok) {
                        atomicAdd(&a.counts[(uint64_t)a.s3code[((lx * L + l1) * L + l2) * L + l3] * 4], 1u);
                    }
                }
        // ---- emit the membership sets --------------------------------------
        for (int lab = 0; lab < L; ++lab)
            for (int w = 0; w < 4; ++w) {
                emit_word(a, U[lab * 4 + w], uniform, lxs, REG_U, lab, w);
                emit_word(a, M[lab * 4 + w], uniform, lxs, REG_M, lab, w);
                emit_word(a, V[lab * 4 + w], uniform, lxs, REG_V, lab, w);
            }
        for (int w = 0; w < 4; ++w) emit_word(a, tp[w], uniform, lxs, 3, 0, w);
    }
}

// Vertices of degree FSM_HUB or more: one wavefront each.  The lanes split
// N(x) in both passes and OR their findings into the vertex's membership
// sets in LDS; the path-inner rows take one lane per label lc; the 3-star
// centre triples and the set words are spread over the lanes for emission.
// The decisions are the lane path's (leaf_pairs, inner_rows, end_ok,
// centre_ok), so both paths give the same sets.  Ids ascend with degree, so
// the hubs are the ids from a.hub0 on.
__global__ void __launch_bounds__(256) fsm_hub(FsmArgs a) {
    __shared__ unsigned long long sU[4][FSM_LMAX * 4], sM[4][FSM_LMAX * 4], sV[4][FSM_LMAX * 4];
    __shared__ uint32_t sPd[4][FSM_LMAX], sT2[4][FSM_LMAX];
    const int L = a.L;
    const int lane = __lane_id();
    const int wv = threadIdx.x >> 6;
    unsigned long long* U = sU[wv];
    unsigned long long* M = sM[wv];
    unsigned long long* V = sV[wv];
    uint32_t* Pd = sPd[wv];
    uint32_t* T2 = sT2[wv];
    const uint32_t nw = gridDim.x * (blockDim.x >> 6);
    for (uint32_t x = a.hub0 + blockIdx.x * (blockDim.x >> 6) + wv; x < a.n; x += nw) {
        const uint32_t xs = a.rp[x], xe = a.rp[x + 1];
        if (xe - xs < FSM_HUB) continue;
        const int lx = a.lab[x];
        const uint32_t* hx = a.hist + (uint64_t)x * FSM_LMAX;
        for (uint32_t i = lane; i < FSM_LMAX * 4; i += 64) U[i] = M[i] = V[i] = 0ull;
        if (lane < FSM_LMAX) Pd[lane] = T2[lane] = 0u;
        ft_sync();
        // ---- pass 1: 3-star leaf sets and the per-label presence masks ----
        for (uint32_t p = xs + lane; p < xe; p += 64) {
            const uint32_t c = a.col[p];
            const int lc = a.lab[c];
            const uint32_t pr = present_minus(a, c, lx), tw = twice_minus(a, c, lx);
            if (pr) atomicOr(&Pd[lc], pr);
            if (tw) atomicOr(&T2[lc], tw);
            uint64_t f[4];
            leaf_pairs(pr, tw, f[0], f[1], f[2], f[3]);
#pragma unroll
            for (int w = 0; w < 4; ++w)
                if (f[w] & ~U[lc * 4 + w]) atomicOr(&U[lc * 4 + w], (unsigned long long)f[w]);
        }
        ft_sync();
        // ---- path inner: one lane per label lc --------------------------
        if (lane < L && Pd[lane]) {
            uint64_t m0, m1, m2, m3;
            inner_rows(a, x, lx, lane, Pd[lane], T2[lane], m0, m1, m2, m3);
            M[lane * 4 + 0] = m0;
            M[lane * 4 + 1] = m1;
            M[lane * 4 + 2] = m2;
            M[lane * 4 + 3] = m3;
        }
        // ---- path end: lanes split the neighbours b ---------------------
        for (uint32_t p = xs + lane; p < xe; p += 64) {
            const uint32_t b = a.col[p];
            const int lb = a.lab[b];
            const uint32_t* wm = a.bmask + (uint64_t)b * FSM_LMAX;
            const uint32_t ex = present_minus(a, x, lb);
            for (int lc = 0; lc < L; ++lc) {
                // bits another lane has set need no second decision (bits
                // are only ever set, so a stale read costs work, not results)
                const uint64_t vw = __atomic_load_n(&V[lb * 4 + (lc >> 2)], __ATOMIC_RELAXED);
                const uint32_t known = (uint32_t)((vw >> ((lc & 3) * 16)) & 0xffffu);
                uint32_t dm = wm[lc] & ~known;
                while (dm) {
                    const int ld = __builtin_ctz(dm);
                    dm &= dm - 1;
                    if (end_ok(a, x, lx, b, lb, lc, ld, ex)) {
                        const int bit = lc * FSM_LMAX + ld;
                        atomicOr(&V[lb * 4 + (bit >> 6)], 1ull << (bit & 63));
                    }
                }
            }
        }
        ft_sync();
        // ---- 3-star centre: triples l1 <= l2 <= l3 over the lanes --------
        for (int t = lane; t < L * L * L; t += 64) {
            const int l1 = t / (L * L), l2 = (t / L) % L, l3 = t % L;
            if (l1 > l2 || l2 > l3) continue;
            if (centre_ok(hx, l1, l2, l3))
                atomicAdd(&a.counts[(uint64_t)a.s3code[((lx * L + l1) * L + l2) * L + l3] * 4], 1u);
        }
        // ---- emit: one set word per lane at a time ------------------------
        for (int t = lane; t < 3 * L * 4 + 4; t += 64) {
            int reg, lab, w;
            uint64_t m;
            if (t < 3 * L * 4) {
                reg = t / (L * 4);
                lab = (t / 4) % L;
                w = t % 4;
                m = reg == REG_U ? U[lab * 4 + w] : (reg == REG_M ? M[lab * 4 + w] : V[lab * 4 + w]);
            } else {
                reg = 3;
                lab = 0;
                w = t - 3 * L * 4;
                m = a.tri[(uint64_t)x * 4 + w];
            }
            while (m) {
                const int b = __builtin_ctzll(m);
                m &= m - 1;
                int slot, colidx;
                where_of(a, reg, lab, (w << 6) + b, lx, slot, colidx);
                atomicAdd(&a.counts[(uint64_t)slot * 4 + colidx], 1u);
            }
        }
        ft_sync();
    }
}

int launch_fsm(const FsmArgs& a, int grid, hipStream_t s, hipEvent_t* ev) {
    if (ev) hipEventRecord(ev[0], s);
    hipLaunchKernelGGL(fsm_hist, dim3(grid), dim3(256), 0, s, a);
    if (hipGetLastError() != hipSuccess) return -1;
    if (ev) hipEventRecord(ev[1], s);
    hipLaunchKernelGGL(fsm_tri, dim3(grid), dim3(256), 0, s, a);
    if (hipGetLastError() != hipSuccess) return -1;
    if (ev) hipEventRecord(ev[2], s);
    hipLaunchKernelGGL(fsm_btab, dim3(grid), dim3(256), 0, s, a);
    if (hipGetLastError() != hipSuccess) return -1;
    if (ev) hipEventRecord(ev[3], s);
    hipLaunchKernelGGL(fsm_main, dim3(grid), dim3(256), 0, s, a);
    if (hipGetLastError() != hipSuccess) return -1;
    if (ev) hipEventRecord(ev[4], s);
    if (a.hub0 < a.n) hipLaunchKernelGGL(fsm_hub, dim3(grid), dim3(256), 0, s, a);
    if (ev) hipEventRecord(ev[5], s);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pm
