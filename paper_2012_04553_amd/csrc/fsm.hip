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
//   * triangle: x lies on a triangle whose other two labels are (ly, lz).
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

// ---- per vertex b: for every (lc, ld), how many c in N(b) (label lc) have a
// neighbour of label ld outside {b}, and how many of those have exactly one.
__global__ void fsm_btab(FsmArgs a) {
    for (uint32_t b = blockIdx.x * blockDim.x + threadIdx.x; b < a.n; b += gridDim.x * blockDim.x) {
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
}

__device__ __forceinline__ void bump(const FsmArgs& a, int slot, int colidx) {
    atomicAdd(&a.counts[(uint64_t)slot * 4 + colidx], 1u);
}

// path slot of the ordered label tuple, and the canonical column of position i
__device__ __forceinline__ void p4_member(const FsmArgs& a, int la, int lb, int lc, int ld, int pos) {
    const int L = a.L;
    int code = a.p4code[((la * L + lb) * L + lc) * L + ld];
    int slot = code >> 2;
    int rev = (code >> 1) & 1, pal = code & 1;
    int colidx = rev ? 3 - pos : pos;
    if (pal && colidx >= 2) colidx = 3 - colidx;
    bump(a, slot, colidx);
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

__global__ void __launch_bounds__(256) fsm_main(FsmArgs a) {
    const int L = a.L;
    const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t* scratch = a.scratch + tid * FSM_SCRATCH_WORDS;
    for (uint32_t x = (uint32_t)tid; x < a.n; x += gridDim.x * blockDim.x) {
        const int lx = a.lab[x];
        const uint32_t xs = a.rp[x], xe = a.rp[x + 1];
        if (xs == xe) continue;
        const uint32_t* hx = a.hist + (uint64_t)x * FSM_LMAX;
        // ---- 3-star centre ------------------------------------------------
        for (int l1 = 0; l1 < L; ++l1)
            for (int l2 = l1; l2 < L; ++l2)
                for (int l3 = l2; l3 < L; ++l3) {
                    uint32_t n1 = hx[l1], n2 = hx[l2], n3 = hx[l3];
                    bool ok;
                    if (l1 == l3) ok = n1 >= 3;
                    else if (l1 == l2) ok = n1 >= 2 && n3 >= 1;
                    else if (l2 == l3) ok = n1 >= 1 && n2 >= 2;
                    else ok = n1 >= 1 && n2 >= 1 && n3 >= 1;
                    if (ok) bump(a, a.s3code[((lx * L + l1) * L + l2) * L + l3], 0);
                }
        // ---- 3-star leaf: U[lc] = pairs {l2 <= l3} coverable besides x ------
        // pair index over (l2 <= l3): bit l2*L + l3 in a 256-bit set
        uint64_t* U = scratch;  // FSM_LMAX * 4 words
        for (int i = 0; i < FSM_LMAX * 4; ++i) U[i] = 0;
        // ---- path inner: Pd[lc] = labels of d reachable; T2[lc]: twice ----
        uint32_t Pd[FSM_LMAX], T2[FSM_LMAX];
        for (int i = 0; i < FSM_LMAX; ++i) Pd[i] = T2[i] = 0;
        for (uint32_t p = xs; p < xe; ++p) {
            const uint32_t c = a.col[p];
            const int lc = a.lab[c];
            const uint32_t pr = present_minus(a, c, lx), tw = twice_minus(a, c, lx);
            Pd[lc] |= pr;
            T2[lc] |= tw;
            // pairs coverable by c's other neighbours
            uint64_t* u = U + lc * 4;
            uint32_t e2 = pr;
            while (e2) {
                int l2 = __builtin_ctz(e2);
                e2 &= e2 - 1;
                uint32_t hi = pr & ~((2u << l2) - 1u);  // l3 > l2
                if ((tw >> l2) & 1) hi |= 1u << l2;     // l3 == l2
                while (hi) {
                    int l3 = __builtin_ctz(hi);
                    hi &= hi - 1;
                    int bit = l2 * FSM_LMAX + l3;
                    u[bit >> 6] |= 1ull << (bit & 63);
                }
            }
        }
        for (int lc = 0; lc < L; ++lc) {
            const uint64_t* u = U + lc * 4;
            for (int w = 0; w < 4; ++w) {
                uint64_t m = u[w];
                while (m) {
                    int bit = (w << 6) + __builtin_ctzll(m);
                    m &= m - 1;
                    int l2 = bit / FSM_LMAX, l3 = bit % FSM_LMAX;
                    int s0 = lx, s1 = l2, s2 = l3;
                    sort3(s0, s1, s2);
                    bump(a, a.s3code[((lc * L + s0) * L + s1) * L + s2], 1 + first_pos(s0, s1, s2, lx));
                }
            }
        }
        for (int lc = 0; lc < L; ++lc) {
            if (!Pd[lc]) continue;
            // a: labels of N(x) \ {c} for some c of label lc
            const uint32_t pa = hx[lc] >= 2 ? a.pres[(uint64_t)x * 3] : (a.pres[(uint64_t)x * 3] & ~(1u << lc));
            for (int la = 0; la < L; ++la) {
                if (!((pa >> la) & 1)) continue;
                uint32_t dset = Pd[lc];
                while (dset) {
                    const int ld = __builtin_ctz(dset);
                    dset &= dset - 1;
                    bool ok = true;
                    if (la == ld) {
                        const uint32_t na = hx[la] - (lc == la ? 1u : 0u);
                        if (na < 2 && !((T2[lc] >> la) & 1)) {
                            // every candidate c has one witness d; x one witness a:
                            // valid iff some c (label lc) has its witness d != a
                            ok = false;
                            for (uint32_t p = xs; p < xe && !ok; ++p) {
                                const uint32_t c = a.col[p];
                                if (a.lab[c] != lc) continue;
                                if (!((present_minus(a, c, lx) >> la) & 1)) continue;
                                const uint32_t aa = unique_other(a, x, la, c);
                                if (aa >= a.n) continue;
                                if (!fsm_has(a.col, a.rp[c], a.rp[c + 1], aa)) ok = true;
                            }
                        }
                    }
                    if (ok) p4_member(a, la, lx, lc, ld, 1);
                }
            }
        }
        // ---- path end: V[lb] = (lc, ld) reachable from x via b -------------
        uint64_t* V = scratch + FSM_LMAX * 4;  // FSM_LMAX * 4 words
        for (int i = 0; i < FSM_LMAX * 4; ++i) V[i] = 0;
        for (uint32_t p = xs; p < xe; ++p) {
            const uint32_t b = a.col[p];
            const int lb = a.lab[b];
            const uint32_t* wm = a.bmask + (uint64_t)b * FSM_LMAX;
            const uint8_t* cnt = a.bcnt + (uint64_t)b * FSM_LMAX * FSM_LMAX;
            const uint8_t* frag = a.bfrag + (uint64_t)b * FSM_LMAX * FSM_LMAX;
            const uint32_t ex = present_minus(a, x, lb);  // x as a c-candidate of b
            uint64_t* v = V + lb * 4;
            for (int lc = 0; lc < L; ++lc) {
                uint32_t dm = wm[lc];
                while (dm) {
                    const int ld = __builtin_ctz(dm);
                    dm &= dm - 1;
                    const int bit = lc * FSM_LMAX + ld;
                    if ((v[bit >> 6] >> (bit & 63)) & 1ull) continue;
                    const uint32_t cn = cnt[lc * FSM_LMAX + ld];
                    const uint32_t fr = frag[lc * FSM_LMAX + ld];
                    const uint32_t self = (lc == lx && ((ex >> ld) & 1)) ? 1u : 0u;
                    bool ok;
                    if (cn < 255 && cn < self + 1) ok = false;
                    else if (cn < 255 && cn >= self + 1 + fr) ok = true;
                    else if (ld != lx) ok = cn >= self + 1;
                    else {
                        // exact: c in N(b) \ {x}, label lc, with a label-ld neighbour
                        // outside {b, x}
                        ok = false;
                        for (uint32_t q = a.rp[b]; q < a.rp[b + 1] && !ok; ++q) {
                            const uint32_t c = a.col[q];
                            if (c == x || a.lab[c] != lc) continue;
                            uint32_t k = a.hist[(uint64_t)c * FSM_LMAX + ld] - (ld == lb ? 1u : 0u);
                            if (k >= 1 && fsm_has(a.col, a.rp[c], a.rp[c + 1], x)) --k;
                            if (k >= 1) ok = true;
                        }
                    }
                    if (ok) v[bit >> 6] |= 1ull << (bit & 63);
                }
            }
        }
        for (int lb = 0; lb < L; ++lb) {
            const uint64_t* v = V + lb * 4;
            for (int w = 0; w < 4; ++w) {
                uint64_t m = v[w];
                while (m) {
                    const int bit = (w << 6) + __builtin_ctzll(m);
                    m &= m - 1;
                    p4_member(a, lx, lb, bit / FSM_LMAX, bit % FSM_LMAX, 0);
                }
            }
        }
        // ---- triangle: label pairs of the other two vertices ---------------
        uint64_t tp[4] = {0, 0, 0, 0};
        for (uint32_t p = xs; p < xe; ++p) {
            const uint32_t y = a.col[p];
            const uint32_t ys = a.rp[y], ye = a.rp[y + 1];
            // z in N(x) with z > y, z in N(y): scan the shorter tail
            const uint32_t xt = p + 1;
            uint32_t yt = ys;
            {
                uint32_t lo = ys, hi = ye;
                while (lo < hi) {
                    uint32_t mid = (lo + hi) >> 1;
                    if (a.col[mid] <= y) lo = mid + 1;
                    else hi = mid;
                }
                yt = lo;
            }
            const int ly = a.lab[y];
            if (xe - xt <= ye - yt) {
                for (uint32_t q = xt; q < xe; ++q) {
                    const uint32_t z = a.col[q];
                    if (fsm_has(a.col, yt, ye, z)) {
                        int l2 = ly, l3 = a.lab[z];
                        if (l2 > l3) { int t = l2; l2 = l3; l3 = t; }
                        const int bit = l2 * FSM_LMAX + l3;
                        tp[bit >> 6] |= 1ull << (bit & 63);
                    }
                }
            } else {
                for (uint32_t q = yt; q < ye; ++q) {
                    const uint32_t z = a.col[q];
                    if (fsm_has(a.col, xt, xe, z)) {
                        int l2 = ly, l3 = a.lab[z];
                        if (l2 > l3) { int t = l2; l2 = l3; l3 = t; }
                        const int bit = l2 * FSM_LMAX + l3;
                        tp[bit >> 6] |= 1ull << (bit & 63);
                    }
                }
            }
        }
        for (int w = 0; w < 4; ++w) {
            uint64_t m = tp[w];
            while (m) {
                const int bit = (w << 6) + __builtin_ctzll(m);
                m &= m - 1;
                int s0 = lx, s1 = bit / FSM_LMAX, s2 = bit % FSM_LMAX;
                sort3(s0, s1, s2);
                bump(a, a.tricode[(s0 * L + s1) * L + s2], first_pos(s0, s1, s2, lx));
            }
        }
    }
}

int launch_fsm(const FsmArgs& a, int grid, hipStream_t s) {
    hipLaunchKernelGGL(fsm_hist, dim3(grid), dim3(256), 0, s, a);
    if (hipGetLastError() != hipSuccess) return -1;
    hipLaunchKernelGGL(fsm_btab, dim3(grid), dim3(256), 0, s, a);
    if (hipGetLastError() != hipSuccess) return -1;
    hipLaunchKernelGGL(fsm_main, dim3(grid), dim3(256), 0, s, a);
    return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace pm
