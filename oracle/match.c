/*
 * Oracle matchers -- TEST INFRASTRUCTURE ONLY.
 *
 * Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may
 * load this library.  It shares no code with the HIP path.
 *
 * Plain, slow, obviously-correct CPU counting from the paper's definitions:
 *
 *  - or_count_maps: tier A.  Counts matches of a pattern (Preliminaries,
 *    "Pattern Semantics": an injective map preserving every edge and every
 *    anti-edge, and labels when present).  Pattern vertices are mapped in a
 *    given connected order; candidates for a vertex are the neighbours of
 *    its first already-mapped pattern neighbour; then EVERY pattern edge and
 *    anti-edge to earlier vertices is checked by binary search, and
 *    injectivity by a scan.  No symmetry breaking, no set algebra.
 *
 *  - or_census: tier A'.  Enumerates every connected induced k-vertex
 *    subgraph exactly once (ESU enumeration) and histograms its induced edge
 *    mask (vertices taken in ascending id order).  Gives vertex-induced
 *    counts by a route independent of or_count_maps.
 *
 *  - or_tier_c4: closed forms for edge-induced 3- and 4-vertex counts on
 *    large graphs (per-edge common-neighbour counts by sorted merge,
 *    co-degree counting for 4-cycles, clique enumeration for K4).
 *
 *  - or_mni_maps: minimum-node-image domains (Preliminaries, "Frequent
 *    Subgraph Mining": one column per pattern vertex holding m(v) of every
 *    match) by enumerating every match.
 *  - or_mni_column: the size of one such column on large graphs, by a
 *    search from every candidate vertex that stops at its first match.
 *  - or_list_maps: every match written out (listing on tiny graphs).
 *  - or_mni_labelings: the columns of every labeling of one unlabeled
 *    pattern at once: each match of the unlabeled pattern is a match of
 *    exactly one labeled pattern, the one whose vertex i carries the label
 *    of its image.
 *
 * Graph: simple undirected CSR, ascending adjacency, uint32 ids.
 * Pattern edge (i<j) is bit j*(j-1)/2+i of a mask.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

static int pbit(int i, int j) {
    if (i > j) { int t = i; i = j; j = t; }
    return j * (j - 1) / 2 + i;
}

static int adjacent(const uint32_t* rp, const uint32_t* col, uint32_t u, uint32_t v) {
    uint32_t lo = rp[u], hi = rp[u + 1];
    while (lo < hi) {
        uint32_t mid = lo + (hi - lo) / 2;
        if (col[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo < rp[u + 1] && col[lo] == v;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ */
/* Tier A: injective-map backtracking                                  */
/* ------------------------------------------------------------------ */

typedef struct {
    const uint32_t* rp;
    const uint32_t* col;
    const uint8_t* lab;     /* nullable */
    int k;
    int order[8];           /* order[j] = pattern vertex mapped at step j */
    int anchor[8];          /* step index of first earlier neighbour      */
    int plab[8];            /* label per pattern vertex, -1 = any          */
    uint32_t emask, amask;
    uint8_t* dom;           /* optional: k*n domain flags (MNI)            */
    uint32_t n;
} mapctx;

static int step_ok(const mapctx* c, const uint32_t* img, int j, uint32_t x) {
    int pj = c->order[j];
    if (c->lab && c->plab[pj] >= 0 && (int)c->lab[x] != c->plab[pj]) return 0;
    if (!c->lab && c->plab[pj] >= 0) return 0;
    for (int i = 0; i < j; ++i) if (img[i] == x) return 0;
    for (int i = 0; i < j; ++i) {
        int pi = c->order[i];
        int b = pbit(pi, pj);
        if ((c->emask >> b) & 1) {
            if (!adjacent(c->rp, c->col, img[i], x)) return 0;
        } else if ((c->amask >> b) & 1) {
            if (adjacent(c->rp, c->col, img[i], x)) return 0;
        }
    }
    return 1;
}

static u128 extend(const mapctx* c, uint32_t* img, int j) {
    if (j == c->k) {
        if (c->dom) {
            for (int i = 0; i < c->k; ++i)
                c->dom[(size_t)c->order[i] * c->n + img[i]] = 1;
        }
        return 1;
    }
    uint32_t a = img[c->anchor[j]];
    u128 total = 0;
    for (uint32_t e = c->rp[a]; e < c->rp[a + 1]; ++e) {
        uint32_t x = c->col[e];
        if (!step_ok(c, img, j, x)) continue;
        img[j] = x;
        total += extend(c, img, j + 1);
    }
    return total;
}

static int setup_ctx(mapctx* c, uint32_t n, const uint32_t* rp, const uint32_t* col,
                     const uint8_t* lab, int k, const int* order, uint32_t emask,
                     uint32_t amask, const int* plab) {
    if (k < 1 || k > 8) return -1;
    c->rp = rp; c->col = col; c->lab = lab; c->k = k; c->emask = emask;
    c->amask = amask; c->dom = NULL; c->n = n;
    for (int j = 0; j < k; ++j) {
        c->order[j] = order[j];
        c->plab[j] = plab ? plab[j] : -1;
    }
    for (int j = 1; j < k; ++j) {
        c->anchor[j] = -1;
        for (int i = 0; i < j; ++i)
            if ((emask >> pbit(order[i], order[j])) & 1) { c->anchor[j] = i; break; }
        if (c->anchor[j] < 0) return -2; /* order not connected */
    }
    return 0;
}

/* Number of matches (injective maps) whose first mapped vertex lies in
 * [root_lo, root_hi).  Result returned as 128-bit (lo, hi). */
int or_count_maps(uint32_t n, const uint32_t* rp, const uint32_t* col,
                  const uint8_t* lab, int k, const int* order, uint32_t emask,
                  uint32_t amask, const int* plab, uint32_t root_lo,
                  uint32_t root_hi, uint64_t* out_lo, uint64_t* out_hi) {
    mapctx c;
    int rc = setup_ctx(&c, n, rp, col, lab, k, order, emask, amask, plab);
    if (rc) return rc;
    if (root_hi > n) root_hi = n;
    int nt = or_num_threads();
    u128* part = (u128*)calloc((size_t)nt, sizeof(u128));
#pragma omp parallel
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        uint32_t img[8];
        u128 acc = 0;
#pragma omp for schedule(dynamic, 16)
        for (int64_t r = root_lo; r < (int64_t)root_hi; ++r) {
            if (!step_ok(&c, img, 0, (uint32_t)r)) continue;
            img[0] = (uint32_t)r;
            acc += extend(&c, img, 1);
        }
        part[t] = acc;
    }
    u128 tot = 0;
    for (int t = 0; t < nt; ++t) tot += part[t];
    free(part);
    *out_lo = (uint64_t)tot;
    *out_hi = (uint64_t)(tot >> 64);
    return 0;
}

/* MNI domains by full match enumeration: dom[v*n + x] = 1 when some match
 * maps pattern vertex v to data vertex x.  Single-threaded. */
int or_mni_maps(uint32_t n, const uint32_t* rp, const uint32_t* col,
                const uint8_t* lab, int k, const int* order, uint32_t emask,
                uint32_t amask, const int* plab, uint8_t* dom,
                uint64_t* out_lo, uint64_t* out_hi) {
    mapctx c;
    int rc = setup_ctx(&c, n, rp, col, lab, k, order, emask, amask, plab);
    if (rc) return rc;
    c.dom = dom;
    memset(dom, 0, (size_t)k * n);
    uint32_t img[8];
    u128 tot = 0;
    for (uint32_t r = 0; r < n; ++r) {
        if (!step_ok(&c, img, 0, r)) continue;
        img[0] = r;
        tot += extend(&c, img, 1);
    }
    *out_lo = (uint64_t)tot;
    *out_hi = (uint64_t)(tot >> 64);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Tier A': census of connected induced k-subgraphs (ESU)               */
/* ------------------------------------------------------------------ */

typedef struct {
    const uint32_t* rp;
    const uint32_t* col;
    int k;
    uint64_t* hist;          /* per-thread histogram, 1 << C(k,2) entries */
    uint32_t* sub;           /* current vertex set (size k)               */
    uint32_t* ext;           /* extension stacks, one segment per depth   */
    size_t ext_cap;          /* capacity of one segment                   */
} esu;

static int in_list(const uint32_t* a, int len, uint32_t x) {
    for (int i = 0; i < len; ++i) if (a[i] == x) return 1;
    return 0;
}

static void esu_emit(esu* e) {
    uint32_t s[8];
    int k = e->k;
    memcpy(s, e->sub, sizeof(uint32_t) * k);
    for (int i = 1; i < k; ++i) {       /* insertion sort, k <= 8 */
        uint32_t x = s[i]; int j = i - 1;
        while (j >= 0 && s[j] > x) { s[j + 1] = s[j]; --j; }
        s[j + 1] = x;
    }
    uint32_t mask = 0;
    for (int j = 1; j < k; ++j)
        for (int i = 0; i < j; ++i)
            if (adjacent(e->rp, e->col, s[i], s[j])) mask |= 1u << pbit(i, j);
    e->hist[mask] += 1;
}

/* neighbour of the current set (some member adjacent to x)? */
static int touches_sub(const esu* e, int len, uint32_t x) {
    for (int i = 0; i < len; ++i)
        if (e->sub[i] == x || adjacent(e->rp, e->col, e->sub[i], x)) return 1;
    return 0;
}

static void esu_extend(esu* e, int len, uint32_t* ext, size_t next, uint32_t v) {
    if (len == e->k) { esu_emit(e); return; }
    uint32_t* nxt = ext + e->ext_cap;
    while (next > 0) {
        uint32_t w = ext[--next];
        /* new extension set: remaining ext plus exclusive neighbours of w */
        size_t nn = next;
        memcpy(nxt, ext, next * sizeof(uint32_t));
        for (uint32_t p = e->rp[w]; p < e->rp[w + 1]; ++p) {
            uint32_t u = e->col[p];
            if (u <= v) continue;
            if (touches_sub(e, len, u)) continue;      /* not exclusive  */
            if (in_list(nxt, (int)nn, u)) continue;
            nxt[nn++] = u;
        }
        e->sub[len] = w;
        esu_extend(e, len + 1, nxt, nn, v);
    }
}

/* hist has 1 << (k*(k-1)/2) entries, indexed by the induced mask of the
 * subgraph with its vertices in ascending id order. */
int or_census(uint32_t n, const uint32_t* rp, const uint32_t* col, int k,
              uint64_t* hist) {
    if (k < 2 || k > 6) return -1;
    size_t nh = (size_t)1 << (k * (k - 1) / 2);
    uint32_t maxd = 0;
    for (uint32_t v = 0; v < n; ++v)
        if (rp[v + 1] - rp[v] > maxd) maxd = rp[v + 1] - rp[v];
    size_t cap = (size_t)k * (maxd + 1) + 8;
    int nt = or_num_threads();
    uint64_t* parts = (uint64_t*)calloc((size_t)nt * nh, sizeof(uint64_t));
#pragma omp parallel
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        esu e;
        e.rp = rp; e.col = col; e.k = k; e.hist = parts + (size_t)t * nh;
        uint32_t sub[8];
        e.sub = sub;
        e.ext_cap = cap;
        e.ext = (uint32_t*)malloc(sizeof(uint32_t) * cap * (k + 1));
#pragma omp for schedule(dynamic, 8)
        for (int64_t vv = 0; vv < (int64_t)n; ++vv) {
            uint32_t v = (uint32_t)vv;
            size_t ne = 0;
            for (uint32_t p = rp[v]; p < rp[v + 1]; ++p)
                if (col[p] > v) e.ext[ne++] = col[p];
            sub[0] = v;
            esu_extend(&e, 1, e.ext, ne, v);
        }
        free(e.ext);
    }
    memset(hist, 0, nh * sizeof(uint64_t));
    for (int t = 0; t < nt; ++t)
        for (size_t i = 0; i < nh; ++i) hist[i] += parts[(size_t)t * nh + i];
    free(parts);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Tier C: closed forms for edge-induced counts, k <= 4                 */
/* ------------------------------------------------------------------ */

static uint32_t merge_common(const uint32_t* a, uint32_t la, const uint32_t* b, uint32_t lb) {
    uint32_t i = 0, j = 0, c = 0;
    while (i < la && j < lb) {
        if (a[i] < b[j]) ++i;
        else if (a[i] > b[j]) ++j;
        else { ++c; ++i; ++j; }
    }
    return c;
}

/* out[0..8] as 128-bit pairs (lo, hi), in this order:
 *   0 edges m, 1 wedges sum C(d,2), 2 triangles T, 3 3-stars sum C(d,3),
 *   4 P4^E, 5 tailed-triangle^E, 6 C4^E, 7 diamond^E, 8 K4.
 * Formulas: T = sum over edges of common neighbours / 3;
 *   P4^E = sum_edges (d_u-1)(d_v-1) - 3T;
 *   TT^E = sum_v t_v (d_v - 2) with t_v = triangles at v;
 *   C4^E = 1/2 sum_{u<w} C(codeg(u,w), 2);
 *   D^E  = sum_edges C(t_uv, 2);
 *   K4 by enumerating u->v->w->x over the degree-oriented DAG. */
int or_tier_c4(uint32_t n, const uint32_t* rp, const uint32_t* col, uint64_t* out) {
    int nt = or_num_threads();
    const int NQ = 9;
    u128* part = (u128*)calloc((size_t)nt * NQ, sizeof(u128));
    uint64_t* tv = (uint64_t*)calloc(n, sizeof(uint64_t)); /* 2 * triangles at v */
    /* pass 1: per-edge common neighbours -> T, P4 part, D, t_v */
#pragma omp parallel
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        u128* q = part + (size_t)t * NQ;
#pragma omp for schedule(dynamic, 64)
        for (int64_t uu = 0; uu < (int64_t)n; ++uu) {
            uint32_t u = (uint32_t)uu;
            uint64_t du = rp[u + 1] - rp[u];
            q[1] += (u128)(du * (du - (du > 0)) / 2);
            if (du >= 3) q[3] += (u128)du * (du - 1) * (du - 2) / 6;
            for (uint32_t p = rp[u]; p < rp[u + 1]; ++p) {
                uint32_t v = col[p];
                if (v <= u) continue;
                uint64_t tuv = merge_common(col + rp[u], rp[u + 1] - rp[u],
                                            col + rp[v], rp[v + 1] - rp[v]);
                uint64_t dv = rp[v + 1] - rp[v];
#pragma omp atomic
                tv[u] += tuv;
#pragma omp atomic
                tv[v] += tuv;
                q[0] += 1;
                q[2] += tuv;                                   /* 3T */
                q[4] += (u128)(du - 1) * (dv - 1);
                q[7] += (u128)tuv * (tuv - (tuv > 0)) / 2;
            }
        }
    }
    /* degree-oriented out-lists for K4: u -> v when (deg u, u) < (deg v, v) */
    uint32_t* orp = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
    uint32_t* ocol = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)rp[n] / 2 + 1));
    orp[0] = 0;
    for (uint32_t u = 0; u < n; ++u) {
        uint32_t du = rp[u + 1] - rp[u], c = orp[u];
        for (uint32_t p = rp[u]; p < rp[u + 1]; ++p) {
            uint32_t v = col[p], dv = rp[v + 1] - rp[v];
            if (du < dv || (du == dv && u < v)) ocol[c++] = v;
        }
        orp[u + 1] = c;
    }
    /* pass 2: tailed triangles, C4 via co-degree, K4 */
#pragma omp parallel
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        u128* q = part + (size_t)t * NQ;
        uint32_t* cnt = (uint32_t*)calloc(n, sizeof(uint32_t));
        uint32_t* touched = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
        uint32_t* s1 = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t uu = 0; uu < (int64_t)n; ++uu) {
            uint32_t u = (uint32_t)uu;
            uint64_t du = rp[u + 1] - rp[u];
            if (du >= 2) q[5] += (u128)(tv[u] / 2) * (du - 2);
            /* co-degree with every w > u */
            uint32_t nt2 = 0;
            for (uint32_t p = rp[u]; p < rp[u + 1]; ++p) {
                uint32_t v = col[p];
                for (uint32_t r = rp[v]; r < rp[v + 1]; ++r) {
                    uint32_t w = col[r];
                    if (w <= u) continue;
                    if (cnt[w]++ == 0) touched[nt2++] = w;
                }
            }
            for (uint32_t i = 0; i < nt2; ++i) {
                uint64_t c = cnt[touched[i]];
                q[6] += (u128)(c * (c - 1) / 2);
                cnt[touched[i]] = 0;
            }
            /* K4 over the oriented DAG: u -> v -> w -> x */
            for (uint32_t p = orp[u]; p < orp[u + 1]; ++p) {
                uint32_t v = ocol[p];
                uint32_t ls = 0;
                uint32_t i = orp[u], j = orp[v];
                while (i < orp[u + 1] && j < orp[v + 1]) {
                    if (ocol[i] < ocol[j]) ++i;
                    else if (ocol[i] > ocol[j]) ++j;
                    else { s1[ls++] = ocol[i]; ++i; ++j; }
                }
                for (uint32_t a = 0; a < ls; ++a) {
                    uint32_t w = s1[a];
                    q[8] += merge_common(s1, ls, ocol + orp[w], orp[w + 1] - orp[w]);
                }
            }
        }
        free(cnt);
        free(touched);
        free(s1);
    }
    free(orp);
    free(ocol);
    u128 tot[9];
    memset(tot, 0, sizeof(tot));
    for (int t = 0; t < nt; ++t)
        for (int i = 0; i < NQ; ++i) tot[i] += part[(size_t)t * NQ + i];
    free(part);
    free(tv);
    tot[2] /= 3;                       /* T */
    tot[4] -= 3 * tot[2];              /* P4^E */
    tot[6] /= 2;                       /* each 4-cycle has two diagonals */
    for (int i = 0; i < NQ; ++i) {
        out[2 * i] = (uint64_t)tot[i];
        out[2 * i + 1] = (uint64_t)(tot[i] >> 64);
    }
    return 0;
}

/* The same closed forms restricted to a sample of roots: only roots u with
 * u % stride == offset contribute, each with exactly the terms the full
 * computation credits to u (its degree terms, its edges to higher ids, its
 * co-degrees with higher ids, its 4-cliques as the DAG source), plus the
 * tailed-triangle term of u, which needs the triangles at u over all of u's
 * edges.  out[0..8] (128-bit pairs) hold the raw sums before the divisions
 * of or_tier_c4: summed over every offset they equal its raw sums, so
 * 3T, P4 + 3T and 2 C4 sit in slots 2, 4 and 6. */
int or_tier_c4_sample(uint32_t n, const uint32_t* rp, const uint32_t* col, uint32_t stride,
                      uint32_t offset, uint64_t* out) {
    if (stride == 0) return -1;
    int nt = or_num_threads();
    const int NQ = 9;
    u128* part = (u128*)calloc((size_t)nt * NQ, sizeof(u128));
    uint32_t* orp = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
    uint32_t* ocol = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)rp[n] / 2 + 1));
    orp[0] = 0;
    for (uint32_t u = 0; u < n; ++u) {
        uint32_t du = rp[u + 1] - rp[u], c = orp[u];
        for (uint32_t p = rp[u]; p < rp[u + 1]; ++p) {
            uint32_t v = col[p], dv = rp[v + 1] - rp[v];
            if (du < dv || (du == dv && u < v)) ocol[c++] = v;
        }
        orp[u + 1] = c;
    }
#pragma omp parallel
    {
        int t = 0;
#ifdef _OPENMP
        t = omp_get_thread_num();
#endif
        u128* q = part + (size_t)t * NQ;
        uint32_t* cnt = (uint32_t*)calloc(n, sizeof(uint32_t));
        uint32_t* touched = (uint32_t*)malloc(sizeof(uint32_t) * (size_t)n);
        uint32_t* s1 = (uint32_t*)malloc(sizeof(uint32_t) * ((size_t)n + 1));
#pragma omp for schedule(dynamic, 16)
        for (int64_t uu = offset; uu < (int64_t)n; uu += stride) {
            uint32_t u = (uint32_t)uu;
            uint64_t du = rp[u + 1] - rp[u];
            q[1] += (u128)(du * (du - (du > 0)) / 2);
            if (du >= 3) q[3] += (u128)du * (du - 1) * (du - 2) / 6;
            uint64_t tvu = 0;   /* 2 * triangles at u */
            for (uint32_t p = rp[u]; p < rp[u + 1]; ++p) {
                uint32_t v = col[p];
                uint64_t tuv = merge_common(col + rp[u], rp[u + 1] - rp[u], col + rp[v], rp[v + 1] - rp[v]);
                tvu += tuv;
                if (v <= u) continue;
                uint64_t dv = rp[v + 1] - rp[v];
                q[0] += 1;
                q[2] += tuv;
                q[4] += (u128)(du - 1) * (dv - 1);
                q[7] += (u128)tuv * (tuv - (tuv > 0)) / 2;
            }
            if (du >= 2) q[5] += (u128)(tvu / 2) * (du - 2);
            uint32_t nt2 = 0;
            for (uint32_t p = rp[u]; p < rp[u + 1]; ++p) {
                uint32_t v = col[p];
                for (uint32_t r = rp[v]; r < rp[v + 1]; ++r) {
                    uint32_t w = col[r];
                    if (w <= u) continue;
                    if (cnt[w]++ == 0) touched[nt2++] = w;
                }
            }
            for (uint32_t i = 0; i < nt2; ++i) {
                uint64_t c = cnt[touched[i]];
                q[6] += (u128)(c * (c - 1) / 2);
                cnt[touched[i]] = 0;
            }
            for (uint32_t p = orp[u]; p < orp[u + 1]; ++p) {
                uint32_t v = ocol[p];
                uint32_t ls = 0;
                uint32_t i = orp[u], j = orp[v];
                while (i < orp[u + 1] && j < orp[v + 1]) {
                    if (ocol[i] < ocol[j]) ++i;
                    else if (ocol[i] > ocol[j]) ++j;
                    else { s1[ls++] = ocol[i]; ++i; ++j; }
                }
                for (uint32_t a = 0; a < ls; ++a) {
                    uint32_t w = s1[a];
                    q[8] += merge_common(s1, ls, ocol + orp[w], orp[w + 1] - orp[w]);
                }
            }
        }
        free(cnt);
        free(touched);
        free(s1);
    }
    free(orp);
    free(ocol);
    u128 tot[9];
    memset(tot, 0, sizeof(tot));
    for (int t = 0; t < nt; ++t)
        for (int i = 0; i < NQ; ++i) tot[i] += part[(size_t)t * NQ + i];
    free(part);
    for (int i = 0; i < NQ; ++i) {
        out[2 * i] = (uint64_t)tot[i];
        out[2 * i + 1] = (uint64_t)(tot[i] >> 64);
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* MNI column size by rooted existence                                  */
/* ------------------------------------------------------------------ */

static int exists_from(const mapctx* c, uint32_t* img, int j) {
    if (j == c->k) return 1;
    uint32_t a = img[c->anchor[j]];
    for (uint32_t e = c->rp[a]; e < c->rp[a + 1]; ++e) {
        uint32_t x = c->col[e];
        if (!step_ok(c, img, j, x)) continue;
        img[j] = x;
        if (exists_from(c, img, j + 1)) return 1;
    }
    return 0;
}

/* |D(v)| for the pattern vertex order[0]: the number of data vertices x for
 * which some match maps order[0] to x (a depth-first search from x that
 * stops at the first match).  `order` must start at the column vertex and
 * be connected. */
int or_mni_column(uint32_t n, const uint32_t* rp, const uint32_t* col, const uint8_t* lab,
                  int k, const int* order, uint32_t emask, uint32_t amask, const int* plab,
                  uint64_t* out) {
    mapctx c;
    int rc = setup_ctx(&c, n, rp, col, lab, k, order, emask, amask, plab);
    if (rc) return rc;
    uint64_t total = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : total)
    for (int64_t r = 0; r < (int64_t)n; ++r) {
        uint32_t img[8];
        if (!step_ok(&c, img, 0, (uint32_t)r)) continue;
        img[0] = (uint32_t)r;
        if (exists_from(&c, img, 1)) total += 1;
    }
    *out = total;
    return 0;
}

/* ------------------------------------------------------------------ */
/* MNI columns of every labeling of one pattern                         */
/* ------------------------------------------------------------------ */

/* A match m of the unlabeled pattern is a match of the labeled pattern
 * (same vertices and edges) with vertex i labeled lab[m(i)], and every
 * match of a labeled pattern arises so.  Enumerate the unlabeled matches
 * once and file each under the key sum_v lab[m(v)] * L^v of its
 * labeling (v = pattern vertex).  sel[key] >= 0 picks the labelings to
 * record; their domains are bitmaps dom[(sel*k + v) * words + x/64].
 * out[sel*k + v] = |D(v)| of that labeling. */
typedef struct {
    mapctx c;
    int L;
    const int32_t* sel;
    uint64_t* dom;
    size_t words;
} lblctx;

static void extend_labelings(const lblctx* t, uint32_t* img, int j) {
    const mapctx* c = &t->c;
    if (j == c->k) {
        uint32_t vimg[8];
        for (int i = 0; i < c->k; ++i) vimg[c->order[i]] = img[i];
        int64_t key = 0, mul = 1;
        for (int v = 0; v < c->k; ++v) {
            key += (int64_t)c->lab[vimg[v]] * mul;
            mul *= t->L;
        }
        int32_t s = t->sel[key];
        if (s < 0) return;
        for (int v = 0; v < c->k; ++v) {
            uint64_t* w = &t->dom[((size_t)s * c->k + v) * t->words + (vimg[v] >> 6)];
            uint64_t bit = 1ull << (vimg[v] & 63);
            if (!(*w & bit)) {
#pragma omp atomic
                *w |= bit;
            }
        }
        return;
    }
    uint32_t a = img[c->anchor[j]];
    for (uint32_t e = c->rp[a]; e < c->rp[a + 1]; ++e) {
        uint32_t x = c->col[e];
        if (!step_ok(c, img, j, x)) continue;
        img[j] = x;
        extend_labelings(t, img, j + 1);
    }
}

int or_mni_labelings(uint32_t n, const uint32_t* rp, const uint32_t* col, const uint8_t* lab,
                     int k, const int* order, uint32_t emask, uint32_t amask, int L,
                     const int32_t* sel, int nsel, uint64_t* out) {
    lblctx t;
    int rc = setup_ctx(&t.c, n, rp, col, lab, k, order, emask, amask, NULL);
    if (rc) return rc;
    if (!lab || L < 1) return -3;
    for (uint32_t x = 0; x < n; ++x)
        if (lab[x] >= L) return -4;
    t.L = L;
    t.sel = sel;
    t.words = ((size_t)n + 63) / 64;
    t.dom = (uint64_t*)calloc((size_t)nsel * k * t.words, sizeof(uint64_t));
    if (!t.dom) return -5;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t r = 0; r < (int64_t)n; ++r) {
        uint32_t img[8];
        if (!step_ok(&t.c, img, 0, (uint32_t)r)) continue;
        img[0] = (uint32_t)r;
        extend_labelings(&t, img, 1);
    }
    for (size_t q = 0; q < (size_t)nsel * k; ++q) {
        uint64_t cnt = 0;
        for (size_t w = 0; w < t.words; ++w) cnt += (uint64_t)__builtin_popcountll(t.dom[q * t.words + w]);
        out[q] = cnt;
    }
    free(t.dom);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Listing: every match written out                                     */
/* ------------------------------------------------------------------ */

typedef struct {
    mapctx c;
    uint32_t* out;          /* cap matches of k ids, pattern-vertex order */
    uint64_t cap, count;
} listctx;

static void extend_list(listctx* t, uint32_t* img, int j) {
    const mapctx* c = &t->c;
    if (j == c->k) {
        if (t->count < t->cap)
            for (int i = 0; i < c->k; ++i) t->out[t->count * (uint64_t)c->k + c->order[i]] = img[i];
        t->count++;
        return;
    }
    uint32_t a = img[c->anchor[j]];
    for (uint32_t e = c->rp[a]; e < c->rp[a + 1]; ++e) {
        uint32_t x = c->col[e];
        if (!step_ok(c, img, j, x)) continue;
        img[j] = x;
        extend_list(t, img, j + 1);
    }
}

/* Every match (injective map preserving edges, anti-edges and labels) of
 * the pattern; the first min(count, cap) are written to out.  Single
 * threaded, for small graphs. */
int or_list_maps(uint32_t n, const uint32_t* rp, const uint32_t* col, const uint8_t* lab, int k,
                 const int* order, uint32_t emask, uint32_t amask, const int* plab, uint64_t cap,
                 uint32_t* out, uint64_t* count) {
    listctx t;
    int rc = setup_ctx(&t.c, n, rp, col, lab, k, order, emask, amask, plab);
    if (rc) return rc;
    t.out = out;
    t.cap = cap;
    t.count = 0;
    uint32_t img[8];
    for (uint32_t r = 0; r < n; ++r) {
        if (!step_ok(&t.c, img, 0, r)) continue;
        img[0] = r;
        extend_list(&t, img, 1);
    }
    *count = t.count;
    return 0;
}
