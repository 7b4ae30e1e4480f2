// Internal declarations of the pattern-morphing engine (host side).
#pragma once
#include <array>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/pm.h"

namespace pm {

constexpr int KMAX = 5;         // largest supported pattern
constexpr int MAX_LEAF = 4;     // leaves counted by inclusion-exclusion
constexpr int MAX_TERMS = 48;   // distinct set-size terms of one plan
constexpr int MAX_MONO = 96;    // monomials of one plan's tail polynomial
constexpr int MAX_FAC = 4;      // factors per monomial
constexpr int LOCAL_MAX = 1024; // largest out-neighbourhood of the bitmap clique mode

using Perm = std::array<uint8_t, 8>;

// A pattern: k vertices, edge bitmask (pair i<j at bit j*(j-1)/2+i),
// vertex- or edge-induced, optional labels (-1 = any).
struct Pat {
    int k = 0;
    uint32_t em = 0;
    bool vi = false;
    std::array<int8_t, 8> lab{{-1, -1, -1, -1, -1, -1, -1, -1}};
    bool operator==(const Pat& o) const {
        return k == o.k && em == o.em && vi == o.vi && lab == o.lab;
    }
};

inline int pair_bit(int i, int j) {
    if (i > j) std::swap(i, j);
    return j * (j - 1) / 2 + i;
}
inline bool has_edge(uint32_t m, int i, int j) { return (m >> pair_bit(i, j)) & 1u; }
inline uint32_t full_mask(int k) { return (k * (k - 1) / 2 >= 32) ? ~0u : ((1u << (k * (k - 1) / 2)) - 1u); }
inline int popc(uint32_t x) { return __builtin_popcount(x); }

// ---- algebra.cpp ----
uint32_t permute_mask(int k, uint32_t m, const Perm& p);
bool is_connected(int k, uint32_t m);
std::vector<Perm> all_perms(int k);
Pat canonical(const Pat& p);                       // smallest (mask, labels) relabelling
std::vector<Perm> automorphisms(const Pat& p);      // label-preserving, edge (and anti-edge) preserving
// number of permutations f with f(E(p)) subset E(q) and labels of p carried to q
int64_t injections(const Pat& p, const Pat& q);
// Naive-PMR alternative set for COUNT: union of the same-size edge-induced
// superpatterns of every vertex-induced query (vertex-induced queries only;
// edge-induced queries are matched as given).  matrix is npat x nalt.
struct MorphPlan {
    std::vector<Pat> alt;
    std::vector<int64_t> matrix;   // row-major npat x alt.size()
};
int morph_plan_count(const std::vector<Pat>& q, int morph, MorphPlan* out, std::string* err,
                     const std::function<double(const Pat&)>& cost = nullptr);
// Cost-based alternative set with vertex- and edge-induced alternatives
// mixed (cost of a pattern as matched: p.vi says how)
int morph_plan_mixed(const std::vector<Pat>& qs, const std::function<double(const Pat&)>& cost, MorphPlan* out,
                     std::string* err);
// combine alternative counts: out[i] = sum_j matrix[i][j]*alt[j]; checked int64
int unmorph(const MorphPlan& mp, size_t npat, const std::vector<int64_t>& alt_counts,
            std::vector<int64_t>* out, std::string* err);

// ---- planner.cpp ----
// Device plan: levels of the core enumeration and the tail polynomial.
struct DLevel {          // candidate x for core level j must satisfy:
    uint8_t adj;         //   x in N(v_i) for i in adj
    uint8_t anti;        //   x not in N(v_i) for i in anti
    uint8_t gt;          //   x > v_i for i in gt
    uint8_t lt;          //   x < v_i for i in lt
    uint8_t neq;         //   x != v_i for i in neq
    int8_t label;        //   label(x) == label (when >= 0)
    uint8_t base;        //   0xff, or an earlier level whose candidate set contains this one
    uint8_t agg;         //   1: reached through bridge vertices (two-hop aggregation)
};
struct DTerm {           // |{x : constraints}| evaluated per full core match
    uint8_t adj, anti, gt, lt, neq;
    int8_t label;
    uint8_t cheap;       // one adjacency list, no anti, no label: range count
    uint8_t agg;         // equals the aggregation multiplicity of the last level
    uint8_t sure;        // cheap terms: neq levels known adjacent to the list owner
    uint8_t pad[3];
};
struct DMono {
    int64_t coef;
    uint8_t nf;
    uint8_t f[MAX_FAC];
    uint8_t pad[3];
};
struct DPlan {
    int32_t ncore;       // core levels (>= 1)
    int32_t nterm;       // 0: no leaves, the last core level is counted
    int32_t nmono;
    int32_t mult;        // multiplier when nterm == 0 (|coset reps|)
    int32_t lane_par;    // 1: tail terms all cheap -> evaluated lane-parallel
    int32_t agg_last;    // 1: last core level is a two-hop aggregation level
    uint8_t bridge_gt;   // aggregation: bridge b > v_i for i in mask
    uint8_t bridge_lt;   //              bridge b < v_i
    int8_t bridge_label;
    uint8_t bridge_src;  //              b in N(v_src)
    int32_t local;       // 1: clique with a total order, counted on a bitmap
                         //    of the root's out-neighbourhood
    int32_t bm0;         // 1: membership tests against N(v0) use a per-wave
                         //    bitmap of the root's adjacency list
    int32_t cyc5;        // 1: the edge-induced 5-cycle's pair sum, run by
                         //    cycle5_kernel (no levels or terms of its own)
    int32_t tagg;        // a closed form over per-edge triangle counts t(e)
                         // and per-vertex triangle counts T(v), evaluated
                         // per edge by support_kernel (no levels or terms):
                         // TAGG_BOWTIE or TAGG_TRIPATH
    DLevel lev[KMAX];
    DTerm term[MAX_TERMS];
    DMono mono[MAX_MONO];
};

// The edge-induced 4-cycle's two-hop plan: targets v1 < v0 aggregated over
// bridges below v0, the tail T0^2 - T0 of the bridge count (each 4-cycle at
// its highest vertex, halved by the divisor).  A root with fewer than two
// lower neighbours adds nothing to it.
inline bool c4_agg_plan(const DPlan& d) {
    if (!d.agg_last || d.ncore != 2 || d.nterm != 1 || d.nmono != 2 || d.local || d.bridge_src != 0 ||
        d.bridge_gt != 0 || d.bridge_lt != 1 || d.bridge_label >= 0 || d.lev[0].label >= 0)
        return false;
    const DLevel& L = d.lev[1];
    const DTerm& T = d.term[0];
    if (L.adj || L.anti || L.gt || L.lt != 1 || L.neq || L.label >= 0 || !L.agg) return false;
    if (T.adj != 3 || T.anti || T.gt || T.lt != 1 || T.neq || T.label >= 0 || T.cheap || !T.agg) return false;
    bool lin = false, sq = false;
    for (int m = 0; m < 2; ++m) {
        const DMono& M = d.mono[m];
        lin = lin || (M.coef == -1 && M.nf == 1 && M.f[0] == 0);
        sq = sq || (M.coef == 1 && M.nf == 2 && M.f[0] == 0 && M.f[1] == 0);
    }
    return lin && sq;
}

// Edge-core plans whose set-size terms all intersect N(v0) and N(v1): the
// heavy roots of such plans can run in edge_window_kernel.
constexpr uint32_t EW_TERMS = 4;

// Graph membership bitmaps: vertices of at least HUB_BM_DEG neighbours, the
// highest degrees first, HUB_BM_BYTES at most in all.
constexpr uint32_t HUB_BM_DEG = 64;

// Plan choice: an enumerated core level beyond three ranks this many times
// dearer than its estimate (cliques on the root's local bitmap excepted).
#ifndef PM_DEEP_PENALTY
#define PM_DEEP_PENALTY 16.0
#endif
constexpr double DEEP_PENALTY = PM_DEEP_PENALTY;
constexpr uint64_t HUB_BM_BYTES = 512ull << 20;
inline bool edge_window_ok(const DPlan& d) {
    if (d.ncore != 2 || d.agg_last || d.local || d.nterm == 0) return false;
    const DLevel& L = d.lev[1];
    if (L.adj != 1 || L.anti != 0 || L.base != 0xff) return false;
    uint32_t heavy_terms = 0;
    for (int q = 0; q < d.nterm; ++q) {
        const DTerm& t = d.term[q];
        if (t.cheap || t.agg) continue;
        if (t.adj != 3 || t.anti != 0 || ((t.gt | t.lt | t.neq) & ~3u)) return false;
        ++heavy_terms;
    }
    return heavy_terms >= 1 && heavy_terms <= EW_TERMS;
}

// Triangle-core plans, run by clique_kernel over roots with at most
// CQ_SMAX out-neighbours, up to CQ_PLANS plans a launch (ids in degree
// order, no labels, no anti-edges).  The kernel meets every triangle once,
// at its lowest vertex.  clique_kind returns
//  1 for a core v0 < v1 < v2 with v1 in N+(v0) and v2 in N+(v0) and N+(v1),
//    counted or with cheap tail terms only, and for an edge core v0 < v1
//    with one set-size term |N(v0) cap N(v1)| above v1 (the triangles this
//    edge closes with its lowest vertex v0): the plan's root is the
//    triangle's lowest vertex, so roots beyond CQ_SMAX can run elsewhere;
//  2 for an edge core (either orientation) with one set-size term
//    |N(v0) cap N(v1)| under any bounds: the sum runs over the triangle's
//    three edges, so every triangle has to be met in this kernel;
//  0 otherwise.
// The tail of an edge-core plan must hold its set-size term in every
// monomial exactly once (linear in it); other terms must be cheap.
constexpr uint32_t CQ_SMAX = 1024;
constexpr int CQ_PLANS = 4;
constexpr uint32_t CQ_TERMS = 8;
// Graphs up to this many vertices keep the per-slot triangle counters of
// the support pass inside the hash slots (a smaller LDS footprint).
constexpr uint32_t CQ_PACK_MAX = 0x3FFFFE;
inline int clique_kind(const DPlan& d) {
    if (d.ncore < 2 || d.ncore > 3 || d.agg_last || d.nterm > (int)CQ_TERMS) return 0;
    if (d.local && !(d.ncore == 3 && d.nterm == 0)) return 0;
    if (d.lev[0].label >= 0) return 0;
    const DLevel& l1 = d.lev[1];
    if (l1.adj != 1 || l1.anti || l1.label >= 0 || l1.agg) return 0;
    const bool up = l1.gt == 1 && l1.lt == 0, down = l1.lt == 1 && l1.gt == 0;
    if (!up && !(down && d.ncore == 2)) return 0;
    auto third = [](uint8_t adj, uint8_t anti, int8_t label, uint8_t gt, uint8_t lt, uint8_t neq) {
        return adj == 3 && !anti && label < 0 && !((gt | lt | neq) & ~3u);
    };
    int heavy = -1;
    for (int q = 0; q < d.nterm; ++q) {
        const DTerm& t = d.term[q];
        if (t.agg) return 0;
        if (t.cheap) continue;
        if (d.ncore == 3 || heavy >= 0 || !third(t.adj, t.anti, t.label, t.gt, t.lt, t.neq)) return 0;
        heavy = q;
    }
    if (d.ncore == 3) {
        const DLevel& l2 = d.lev[2];
        return third(l2.adj, l2.anti, l2.label, l2.gt, l2.lt, l2.neq) && (l2.gt & 2) && !l2.lt ? 1 : 0;
    }
    if (heavy < 0) return 0;
    for (int m = 0; m < d.nmono; ++m) {
        int k = 0;
        for (int f = 0; f < d.mono[m].nf; ++f) k += d.mono[m].f[f] == heavy;
        if (k != 1) return 0;
    }
    const DTerm& h = d.term[heavy];
    return up && (h.gt & 2) && !h.lt ? 1 : 2;
}
inline bool clique_ok(const DPlan& d) { return clique_kind(d) != 0; }

// Edge-support plans: an edge core (v1 in N(v0), one orientation, no
// labels) whose one set-size term is the whole common neighbourhood
// |N(v0) cap N(v1)|, with any tail polynomial in it and cheap terms (the
// diamond: the sum over edges of t^2 - t).  clique_kernel adds every
// triangle to the support counter of each of its three edges (a u32 per
// out-list position: the edge {u < w} at w's place in N+(u)), and
// support_kernel evaluates the tail per edge from its support.  This needs
// every triangle, so no root beyond CQ_SMAX.
inline bool support_ok(const DPlan& d) {
    if (d.ncore != 2 || d.agg_last || d.local || d.lev[0].label >= 0) return false;
    const DLevel& l1 = d.lev[1];
    if (l1.adj != 1 || l1.anti || l1.label >= 0 || l1.agg) return false;
    if (!((l1.gt == 1 && l1.lt == 0) || (l1.lt == 1 && l1.gt == 0))) return false;
    int heavy = -1;
    for (int q = 0; q < d.nterm; ++q) {
        const DTerm& t = d.term[q];
        if (t.agg) return false;
        if (t.cheap) continue;
        if (heavy >= 0 || t.adj != 3 || t.anti || t.label >= 0 || t.gt || t.lt || (t.neq & ~3u)) return false;
        heavy = q;
    }
    return heavy >= 0;
}

// Edge-core plans whose terms are all cheap (the 4-path: the sum over edges
// of (d(v0) - 1)(d(v1) - 1)): support_kernel evaluates them per edge, with
// no supports needed.
inline bool edge_cheap_ok(const DPlan& d) {
    if (d.ncore != 2 || d.agg_last || d.local || d.nterm == 0 || d.lev[0].label >= 0) return false;
    const DLevel& l1 = d.lev[1];
    if (l1.adj != 1 || l1.anti || l1.label >= 0 || l1.agg) return false;
    if (!((l1.gt == 1 && l1.lt == 0) || (l1.lt == 1 && l1.gt == 0))) return false;
    for (int q = 0; q < d.nterm; ++q)
        if (!d.term[q].cheap || d.term[q].agg) return false;
    return true;
}

// Counted 4-cliques v0 < v1 < v2 < v3 enumerated from N+(v0) (no labels):
// clique4_kernel counts them from bit rows of the graph induced on N+(v0),
// roots with up to C4_ROOT_MAX out-neighbours.
constexpr uint32_t C4_ROOT_MAX = 1024;
constexpr uint32_t C4_LIGHT_MAX = 128;   // roots a wavefront takes; larger ones a workgroup
constexpr uint32_t C4_HEAVY_MAX = 512;   // workgroup roots in 44 KB; larger ones in 152 KB
inline bool clique4_ok(const DPlan& d) {
    if (d.ncore != 4 || d.nterm != 0 || d.agg_last || d.lev[0].label >= 0) return false;
    for (int j = 1; j < 4; ++j) {
        const DLevel& L = d.lev[j];
        const uint8_t prev = (uint8_t)((1u << j) - 1);
        if (L.adj != prev || L.anti || L.label >= 0 || L.lt || L.agg) return false;
        if (!(L.gt & (1u << (j - 1))) || (L.gt & ~prev)) return false;
    }
    return true;
}

struct PlanInfo {
    DPlan d;
    Pat pat;
    int64_t divisor = 1;       // count = (sum over core reps of tail) / divisor
    std::array<int8_t, KMAX> order{};   // pattern vertex at each core level
    int formulation = 0;       // 0 coset, 1 pattern-chain
    double est_cost = 0;       // kernel work of this plan alone
    double total_cost = 0;     // including the sub-pattern counts it needs
    // Quotient form: the kernel sums only the product of the single-leaf set
    // sizes; the merged-leaf terms of the inclusion-exclusion are counts of
    // smaller patterns:  count = (hmult * kernel_sum - sum w_q count(q)) / autp.
    bool rewrite = false;
    int64_t hmult = 1, autp = 1;
    std::vector<std::pair<Pat, int64_t>> subs;
    // 5-cycle: count = pair sum of cycle5_kernel - the total of the
    // companion triangle plan (the one entry of subs, a marker pattern)
    bool cyc5 = false;
    std::string describe() const;
};

struct GraphStats {             // degree statistics used by the cost model
    double n = 0, m = 0;
    double avg_deg = 0;         // 2m/n
    double nbr_deg = 0;         // sum d^2 / 2m: degree of a random edge end
    double avg_out = 0;         // mean out-degree (degree-ordered orientation)
    double nbr_out = 0;         // sum (d+)^2 / m
    double max_deg = 0, max_out = 0;
    // joint per-vertex sums for exact two-level costs (p = out-degree d+,
    // q = in-degree d- in the degree-ordered orientation, d = degree)
    double s_pp = 0, s_pq = 0, s_pd = 0, s_qq = 0, s_qd = 0, s_dd = 0;
};

// tri: the graph's triangle counts per edge are available to the launch
// (closed forms of tagg_kind may be chosen)
int compile_plan(const Pat& p, const GraphStats& gs, PlanInfo* out, std::string* err, bool tri = false);
// The companion of the 5-cycle plan: a marker pattern (labels -2, never a
// query) whose plan sums, over the triangles {u < v < w}, the neighbours of
// u, v and w below u.
Pat cycle5_aux_pattern();
inline bool is_cycle5(const Pat& p) {
    if (p.k != 5 || p.vi || popc(p.em) != 5) return false;
    for (int v = 0; v < 5; ++v) {
        if (p.lab[v] != -1) return false;
        int d = 0;
        for (int w = 0; w < 5; ++w)
            if (w != v && has_edge(p.em, v, w)) ++d;
        if (d != 2) return false;
    }
    return is_connected(5, p.em);
}
// Edge-induced, unlabeled 5-vertex patterns counted in closed form from
// triangle counts (no enumeration):
//  TAGG_BOWTIE  two triangles sharing one vertex: every pair of triangles at
//    a vertex v that share only v, sum_v C(T(v), 2) - sum_e t(e)(t(e) - 1)
//    (two triangles at v that share a second vertex u share the edge vu);
//  TAGG_TRIPATH a triangle with a two-edge path hanging off one corner: for
//    every edge {u, w}, both orientations (apex, path vertex), the triangles
//    at the apex that avoid the path vertex times the path vertex's other
//    neighbours, (T(u) - t)(d(w) - 1) + (T(w) - t)(d(u) - 1), less the
//    choices whose path end lies on the triangle, 2 t (t - 1) over the edges.
//  TAGG_HOUSE   a 4-cycle with a triangle on one of its edges (a 5-cycle
//    with one chord): per edge e, its triangles times the 4-cycles through
//    it, less the choices whose apex lies on the 4-cycle, which is the sum
//    over all 4-cycles of their edges' triangle counts (house_kernel) less
//    2 t (t - 1) over the edges.
//  TAGG_TAILED  (four vertices) a triangle with a pendant edge: the
//    triangles at v times its other neighbours, sum_v T(v)(d(v) - 2), which
//    is half the sum over the edges of t (d(u) + d(w) - 4).
//  TAGG_DTAIL   a diamond with a pendant edge at one of its two tips: over
//    the triangles, sum_c (d(c) - 2)(t(opposite edge) - 1) for each corner c
//    (the diamond's tip c with the other triangle on the opposite edge, and
//    c's other neighbour), less 12 per 4-clique (the other tip is adjacent
//    to c);
//  TAGG_FAN     a vertex adjacent to all of a 3-edge path (three triangles in
//    a fan): over the triangles, the products (t(e) - 1)(t(f) - 1) of each
//    two of its edges (the triangles on e and f beyond this one), less 12
//    per 4-clique (both are the same vertex).
// The last two are summed per triangle by trisup_kernel; the 4-cliques
// enter as a quotient sub-pattern.
constexpr int32_t TAGG_BOWTIE = 1;
constexpr int32_t TAGG_TRIPATH = 2;
constexpr int32_t TAGG_HOUSE = 3;
constexpr int32_t TAGG_TAILED = 4;
constexpr int32_t TAGG_DTAIL = 5;
constexpr int32_t TAGG_FAN = 6;
// (three vertices) the triangle: a third of the sum of t over the edges, so
// that the 4-path's quotient needs no triangle pass of its own and the
// 4-clique launches can fill the supports
constexpr int32_t TAGG_TRIANGLE = 7;
//  TAGG_K4EAR   a 4-clique with a triangle on one of its edges (the ear's
//    apex another common neighbour of the edge): the sum over the 4-cliques
//    of t(e) - 2 over their six edges, per root on the graph induced on its
//    out-neighbourhood (k4ear_kernel).
constexpr int32_t TAGG_K4EAR = 8;
inline bool tagg_tri(int32_t kind) { return kind == TAGG_DTAIL || kind == TAGG_FAN; }
// closed forms that read the per-vertex triangle counts
inline bool tagg_vtri(int32_t kind) { return kind == TAGG_BOWTIE || kind == TAGG_TRIPATH; }
inline int tagg_kind(const Pat& p) {
    if (p.k < 3 || p.k > 5 || p.vi || !is_connected(p.k, p.em)) return 0;
    int deg[5] = {0, 0, 0, 0, 0};
    for (int v = 0; v < p.k; ++v) {
        if (p.lab[v] != -1) return 0;
        for (int w = 0; w < p.k; ++w)
            if (w != v && has_edge(p.em, v, w)) ++deg[v];
    }
    int hist[5] = {0, 0, 0, 0, 0};
    for (int v = 0; v < p.k; ++v) ++hist[deg[v]];
    bool tri = false;
    for (int a = 0; a < p.k; ++a)
        for (int b = a + 1; b < p.k; ++b)
            for (int c = b + 1; c < p.k; ++c)
                tri = tri || (has_edge(p.em, a, b) && has_edge(p.em, a, c) && has_edge(p.em, b, c));
    if (p.k == 3) return tri ? TAGG_TRIANGLE : 0;
    // four edges with a triangle: the fourth hangs off one corner
    if (p.k == 4) return popc(p.em) == 4 && tri ? TAGG_TAILED : 0;
    // six edges, one vertex of degree 4 and four of degree 2: the leaves pair
    // up into two triangles with the centre
    if (popc(p.em) == 6 && hist[4] == 1 && hist[2] == 4) return TAGG_BOWTIE;
    // five edges with degrees 3, 2, 2, 2, 1 and a triangle: the corner of
    // degree 3 carries the path (without a triangle it is a 4-cycle with a
    // pendant vertex)
    if (popc(p.em) == 5 && hist[3] == 1 && hist[2] == 3 && hist[1] == 1 && tri) return TAGG_TRIPATH;
    // six edges with degrees 3, 3, 2, 2, 2 and the two corners of degree 3
    // adjacent (apart, they are K_{2,3})
    if (popc(p.em) == 6 && hist[3] == 2 && hist[2] == 3) {
        int u = -1, w = -1;
        for (int v = 0; v < 5; ++v)
            if (deg[v] == 3) (u < 0 ? u : w) = v;
        if (has_edge(p.em, u, w)) return TAGG_HOUSE;
    }
    // the only five-vertex graphs with these edge counts and degrees
    if (popc(p.em) == 6 && hist[3] == 3 && hist[2] == 1 && hist[1] == 1) return TAGG_DTAIL;
    if (popc(p.em) == 7 && hist[4] == 1 && hist[3] == 2 && hist[2] == 2) return TAGG_FAN;
    if (popc(p.em) == 8 && hist[4] == 2 && hist[3] == 2 && hist[2] == 1) return TAGG_K4EAR;
    return 0;
}
// all candidate plans (for tests / autotuning)
int candidate_plans(const Pat& p, const GraphStats& gs, std::vector<PlanInfo>* out, std::string* err);

}  // namespace pm
