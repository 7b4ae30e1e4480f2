// Plan compiler: pattern -> device program for the matching kernel.
//
// A match is an injective map preserving edges and anti-edges
// (Preliminaries, "Pattern Semantics").  The number of distinct matched
// subgraphs is #matches / |Aut(p)|.  A plan splits the pattern vertices into
//   * a connected core, enumerated level by level: the candidates of a level
//     are the intersection of the neighbour lists of its earlier pattern
//     neighbours minus those of its anti-edge partners (set intersection
//     and difference), cut by symmetry-breaking bounds;
//   * leaves: vertices with no constraint between each other (no edge and
//     no anti-edge), never enumerated.  For one core match their injective
//     extensions are counted by inclusion-exclusion over set partitions of
//     the leaves:  sum_pi mu(pi) prod_{B in pi} |S_B|,  S_B = the set a vertex
//     satisfying every leaf of B's constraints may take, mu(pi) =
//     prod_B (-1)^{|B|-1} (|B|-1)!.
// Symmetry breaking (partial orders from a stabiliser chain of a group of
// pattern automorphisms, fixing core vertices in matching order) comes in
// two formulations:
//   coset:   the chain runs on Aut(core), the automorphisms of the core
//            subpattern; each core subgraph is enumerated once and the tail
//            is summed over coset representatives T of H = {automorphisms of
//            p mapping the core onto itself} restricted to the core; then
//            count = sum / (|Aut(p)| / |H|).
//   pattern: the chain runs on Aut(p) itself (leaves may receive bounds
//            relative to core vertices, never relative to each other); the
//            group left after the chain divides the sum.
// Both are exact; the cost model picks the cheaper on the graph at hand.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <map>
#include <set>

#include "internal.hpp"

namespace pm {

namespace {

using Group = std::vector<Perm>;

Perm identity() {
    Perm p{};
    for (int i = 0; i < 8; ++i) p[i] = (uint8_t)i;
    return p;
}

Perm compose(const Perm& a, const Perm& b) {  // (a o b)(x) = a(b(x))
    Perm r{};
    for (int i = 0; i < 8; ++i) r[i] = a[b[i]];
    return r;
}

Perm inverse(const Perm& a) {
    Perm r{};
    for (int i = 0; i < 8; ++i) r[a[i]] = (uint8_t)i;
    return r;
}

// Automorphisms of the core subpattern: permutations of the core vertices
// (leaves fixed) preserving edges, anti-edges and labels among core vertices.
Group core_automorphisms(const Pat& p, uint32_t core) {
    Group out;
    for (const Perm& f : all_perms(p.k)) {
        bool ok = true;
        for (int v = 0; v < p.k && ok; ++v) {
            bool in = (core >> v) & 1;
            if (!in && f[v] != v) ok = false;
            if (in && !((core >> f[v]) & 1)) ok = false;
            if (p.lab[v] != p.lab[f[v]]) ok = false;
        }
        if (!ok) continue;
        for (int a = 0; a < p.k && ok; ++a)
            for (int b = a + 1; b < p.k && ok; ++b) {
                if (!((core >> a) & 1) || !((core >> b) & 1)) continue;
                if (has_edge(p.em, a, b) != has_edge(p.em, f[a], f[b])) ok = false;
            }
        if (ok) out.push_back(f);
    }
    return out;
}

struct Rel {  // rel[u][v] = +1 if u > v required, -1 if u < v required
    int8_t r[8][8];
    Rel() { memset(r, 0, sizeof(r)); }
    void add_less(int u, int v) {  // u < v
        r[u][v] = -1;
        r[v][u] = +1;
    }
    void close(int k) {
        for (int w = 0; w < k; ++w)
            for (int u = 0; u < k; ++u)
                for (int v = 0; v < k; ++v)
                    if (r[u][w] == -1 && r[w][v] == -1) add_less(u, v);
    }
};

// Stabiliser chain over the core vertices in matching order: when the
// vertex x to fix has a non-trivial orbit, require x to be the minimum
// (dir = -1) or maximum (dir = +1) of its orbit.  Returns the residual group.
Group chain(Group G, const std::vector<int>& order, int dir, Rel* rel) {
    for (int x : order) {
        std::set<int> orbit;
        for (const Perm& g : G) orbit.insert(g[x]);
        if (orbit.size() > 1) {
            for (int y : orbit) {
                if (y == x) continue;
                if (dir < 0) rel->add_less(x, y);
                else rel->add_less(y, x);
            }
        }
        Group H;
        for (const Perm& g : G)
            if (g[x] == x) H.push_back(g);
        G.swap(H);
    }
    return G;
}

struct LeafCons {
    uint8_t adj = 0, anti = 0, gt = 0, lt = 0;
    int8_t label = -1;
    bool conflict = false;
};

bool term_equal(const DTerm& a, const DTerm& b) {
    return a.adj == b.adj && a.anti == b.anti && a.gt == b.gt && a.lt == b.lt &&
           a.neq == b.neq && a.label == b.label;
}

// set partitions of {0..n-1}
void partitions(int n, std::vector<std::vector<uint32_t>>* out) {
    std::vector<int> assign(n, 0);
    std::function<void(int, int)> rec = [&](int i, int nb) {
        if (i == n) {
            std::vector<uint32_t> blocks(nb, 0);
            for (int t = 0; t < n; ++t) blocks[assign[t]] |= 1u << t;
            out->push_back(blocks);
            return;
        }
        for (int b = 0; b <= nb; ++b) {
            assign[i] = b;
            rec(i + 1, std::max(nb, b + 1));
        }
    };
    if (n == 0) {
        out->push_back({});
        return;
    }
    rec(0, 0);
}

int64_t factorial(int n) {
    int64_t r = 1;
    for (int i = 2; i <= n; ++i) r *= i;
    return r;
}

struct Builder {
    const Pat& p;
    const GraphStats& gs;
    Builder(const Pat& pp, const GraphStats& g) : p(pp), gs(g) {}

    // Build a plan.  core/leaves are vertex masks; order lists the core
    // vertices by level; agg_last: the last core level is reached through
    // bridge leaves.  Returns false when the combination is not valid.
    bool build(uint32_t core, uint32_t leaves, const std::vector<int>& order, int form,
               int dir, bool agg_last, const Group& autp, PlanInfo* out, bool product_only = false) {
        if (product_only && (form != 0 || p.vi || agg_last || popc(leaves) < 2)) return false;
        const int k = p.k;
        const int c = (int)order.size();
        int lev_of[8];
        for (int i = 0; i < 8; ++i) lev_of[i] = -1;
        for (int j = 0; j < c; ++j) lev_of[order[j]] = j;
        uint32_t anti_pairs = p.vi ? (full_mask(k) & ~p.em) : 0u;

        // ---- symmetry breaking ------------------------------------------
        Rel rel;
        std::vector<Perm> T;       // coset representatives (as maps of pattern vertices)
        int64_t divisor = 1, hc_size = 1;
        if (form == 0) {
            Group G = core_automorphisms(p, core);
            Group Hc;  // restrictions to the core of automorphisms preserving it
            for (const Perm& g : autp) {
                bool keeps = true;
                for (int v = 0; v < k; ++v)
                    if (((core >> v) & 1) && !((core >> g[v]) & 1)) keeps = false;
                if (!keeps) continue;
                Perm r = identity();
                for (int v = 0; v < k; ++v)
                    if ((core >> v) & 1) r[v] = g[v];
                if (std::find(Hc.begin(), Hc.end(), r) == Hc.end()) Hc.push_back(r);
            }
            chain(G, order, dir, &rel);
            // left cosets sigma Hc of Hc in G
            std::vector<Perm> covered;
            for (const Perm& s : G) {
                if (std::find(covered.begin(), covered.end(), s) != covered.end()) continue;
                T.push_back(s);
                for (const Perm& h : Hc) covered.push_back(compose(s, h));
            }
            if ((int64_t)autp.size() % (int64_t)Hc.size()) return false;
            divisor = (int64_t)autp.size() / (int64_t)Hc.size();
            hc_size = (int64_t)Hc.size();
        } else {
            Group R = chain(autp, order, dir, &rel);
            // constraints between two leaves are not allowed
            for (int a = 0; a < k; ++a)
                for (int b = 0; b < k; ++b)
                    if (((leaves >> a) & 1) && ((leaves >> b) & 1) && rel.r[a][b]) return false;
            T.push_back(identity());
            divisor = (int64_t)R.size();
        }
        rel.close(k);
        for (int a = 0; a < k; ++a)
            for (int b = 0; b < k; ++b)
                if (((leaves >> a) & 1) && ((leaves >> b) & 1) && rel.r[a][b]) return false;

        DPlan d;
        memset(&d, 0, sizeof(d));
        d.ncore = c;
        d.mult = 1;
        d.bridge_src = 0xff;
        // ---- core levels --------------------------------------------------
        for (int j = 0; j < c; ++j) {
            int u = order[j];
            DLevel L;
            memset(&L, 0, sizeof(L));
            L.base = 0xff;
            L.label = p.lab[u];
            for (int i = 0; i < j; ++i) {
                int w = order[i];
                uint8_t bit = (uint8_t)(1u << i);
                if (has_edge(p.em, u, w)) L.adj |= bit;
                else if ((anti_pairs >> pair_bit(u, w)) & 1) L.anti |= bit;
                if (rel.r[u][w] > 0) L.gt |= bit;
                if (rel.r[u][w] < 0) L.lt |= bit;
            }
            for (int i = 0; i < j; ++i) {
                uint8_t bit = (uint8_t)(1u << i);
                if (!(L.adj & bit) && !(L.gt & bit) && !(L.lt & bit)) L.neq |= bit;
            }
            bool is_agg = agg_last && j == c - 1;
            if (j > 0 && !is_agg && !L.adj) return false;
            if (is_agg && L.adj) return false;
            L.agg = is_agg ? 1 : 0;
            if (j > 1 && !is_agg) {
                for (int b = j - 1; b >= 1; --b) {
                    const DLevel& B = d.lev[b];
                    if (B.agg) continue;
                    uint8_t lowb = (uint8_t)((1u << b) - 1u);
                    if ((B.adj & ~L.adj & lowb) || (B.anti & ~L.anti & lowb)) continue;
                    if ((B.gt & ~L.gt & lowb) || (B.lt & ~L.lt & lowb)) continue;
                    if (B.label >= 0 && B.label != L.label) continue;
                    L.base = (uint8_t)b;
                    break;
                }
            }
            d.lev[j] = L;
        }
        // ---- leaves and tail terms -----------------------------------------
        std::vector<int> leaf;
        for (int v = 0; v < k; ++v)
            if ((leaves >> v) & 1) leaf.push_back(v);
        if ((int)leaf.size() > MAX_LEAF) return false;
        std::vector<DTerm> terms;
        std::map<std::vector<int>, int64_t> monos;  // sorted term ids -> coef
        std::vector<std::vector<uint32_t>> all_parts, parts;
        partitions((int)leaf.size(), &all_parts);
        for (const auto& bl : all_parts)
            if (!product_only || bl.size() == leaf.size()) parts.push_back(bl);
        uint8_t all_core = (uint8_t)((1u << c) - 1u);
        for (const Perm& s : T) {
            std::vector<LeafCons> lc(leaf.size());
            for (size_t t = 0; t < leaf.size(); ++t) {
                int l = leaf[t];
                LeafCons& C = lc[t];
                C.label = p.lab[l];
                for (int cv = 0; cv < k; ++cv) {
                    if (!((core >> cv) & 1)) continue;
                    int lev = lev_of[s[cv]];
                    uint8_t bit = (uint8_t)(1u << lev);
                    if (has_edge(p.em, l, cv)) C.adj |= bit;
                    else if ((anti_pairs >> pair_bit(l, cv)) & 1) C.anti |= bit;
                    if (form == 1) {
                        if (rel.r[l][cv] > 0) C.gt |= bit;
                        if (rel.r[l][cv] < 0) C.lt |= bit;
                    }
                }
                if (!C.adj) return false;
            }
            for (const auto& blocks : parts) {
                int64_t mu = 1;
                std::vector<int> ids;
                bool zero = false;
                for (uint32_t B : blocks) {
                    int sz = popc(B);
                    mu *= ((sz - 1) % 2 ? -1 : 1) * factorial(sz - 1);
                    DTerm tm;
                    memset(&tm, 0, sizeof(tm));
                    tm.label = -1;
                    for (size_t t = 0; t < leaf.size(); ++t) {
                        if (!((B >> t) & 1)) continue;
                        tm.adj |= lc[t].adj;
                        tm.anti |= lc[t].anti;
                        tm.gt |= lc[t].gt;
                        tm.lt |= lc[t].lt;
                        if (lc[t].label >= 0) {
                            if (tm.label >= 0 && tm.label != lc[t].label) zero = true;
                            tm.label = lc[t].label;
                        }
                    }
                    if (tm.adj & tm.anti) zero = true;
                    tm.neq = (uint8_t)(all_core & ~(tm.adj | tm.gt | tm.lt));
                    tm.cheap = (popc(tm.adj) == 1 && !tm.anti && tm.label < 0) ? 1 : 0;
                    if (tm.cheap) {
                        int a = __builtin_ctz((uint32_t)tm.adj);
                        for (int i = 0; i < c; ++i)
                            if (((tm.neq >> i) & 1) && has_edge(p.em, order[a], order[i]))
                                tm.sure |= (uint8_t)(1u << i);
                    }
                    int id = -1;
                    for (size_t q = 0; q < terms.size(); ++q)
                        if (term_equal(terms[q], tm)) id = (int)q;
                    if (id < 0) {
                        id = (int)terms.size();
                        terms.push_back(tm);
                    }
                    ids.push_back(id);
                }
                if (zero) continue;
                std::sort(ids.begin(), ids.end());
                monos[ids] += mu;
            }
        }
        if (leaf.empty()) {
            d.nterm = 0;
            d.nmono = 0;
            d.mult = (int32_t)T.size();
        } else {
            // drop terms no monomial uses
            std::vector<int> used(terms.size(), 0);
            for (auto& m : monos)
                if (m.second)
                    for (int id : m.first) used[id] = 1;
            std::vector<int> remap(terms.size(), -1);
            std::vector<DTerm> kept;
            for (size_t q = 0; q < terms.size(); ++q)
                if (used[q]) {
                    remap[q] = (int)kept.size();
                    kept.push_back(terms[q]);
                }
            if (kept.size() > (size_t)MAX_TERMS) return false;
            int nm = 0;
            for (auto& m : monos) {
                if (!m.second) continue;
                if (nm >= MAX_MONO || (int)m.first.size() > MAX_FAC) return false;
                DMono& M = d.mono[nm++];
                M.coef = m.second;
                M.nf = (uint8_t)m.first.size();
                for (size_t f = 0; f < m.first.size(); ++f) M.f[f] = (uint8_t)remap[m.first[f]];
            }
            d.nmono = nm;
            d.nterm = (int32_t)kept.size();
            for (size_t q = 0; q < kept.size(); ++q) d.term[q] = kept[q];
            if (d.nterm == 0) {
                // every monomial vanished (e.g. conflicting labels): count is 0
                d.nmono = 0;
                d.mult = 0;
            }
        }
        // ---- two-hop aggregation: the bridge set must be a whole term ------
        if (agg_last) {
            int j = c - 1;
            // bridge: a leaf adjacent exactly to {src, order[j]} among core vertices
            bool found = false;
            for (size_t t = 0; t < leaf.size() && !found; ++t) {
                int l = leaf[t];
                uint8_t adjl = 0;
                for (int cv = 0; cv < k; ++cv)
                    if (((core >> cv) & 1) && has_edge(p.em, l, cv)) adjl |= (uint8_t)(1u << lev_of[cv]);
                if (popc(adjl) != 2 || !((adjl >> j) & 1)) continue;
                int src = __builtin_ctz(adjl & ~(1u << j));
                uint8_t bgt = 0, blt = 0;
                if (form == 1) {
                    for (int cv = 0; cv < k; ++cv) {
                        if (!((core >> cv) & 1)) continue;
                        if (rel.r[l][cv] > 0) bgt |= (uint8_t)(1u << lev_of[cv]);
                        if (rel.r[l][cv] < 0) blt |= (uint8_t)(1u << lev_of[cv]);
                    }
                }
                if ((bgt | blt) >> j) continue;  // bridge bound on the target itself
                d.bridge_src = (uint8_t)src;
                d.bridge_gt = bgt;
                d.bridge_lt = blt;
                d.bridge_label = p.lab[l];
                found = true;
            }
            if (!found || T.size() != 1) return false;
            // mark the term equal to the bridge set; others must be cheap
            DTerm br;
            memset(&br, 0, sizeof(br));
            br.adj = (uint8_t)((1u << d.bridge_src) | (1u << j));
            br.gt = d.bridge_gt;
            br.lt = d.bridge_lt;
            br.label = d.bridge_label;
            br.neq = (uint8_t)(all_core & ~(br.adj | br.gt | br.lt));
            for (int q = 0; q < d.nterm; ++q) {
                if (term_equal(d.term[q], br)) d.term[q].agg = 1;
                else if (!d.term[q].cheap) return false;
            }
        }
        // ---- quotient patterns of the merged-leaf terms ----------------------
        std::map<std::pair<uint32_t, std::array<int8_t, 8>>, int64_t> subw;
        if (product_only) {
            for (const auto& blocks : all_parts) {
                if (blocks.size() == leaf.size()) continue;
                Pat q;
                q.vi = false;
                int idx[8];
                int nq = 0;
                for (int v = 0; v < k; ++v)
                    if ((core >> v) & 1) {
                        idx[v] = nq;
                        q.lab[nq] = p.lab[v];
                        ++nq;
                    }
                bool conflict = false;
                std::vector<int> bidx;
                for (uint32_t B : blocks) {
                    int8_t lb = -1;
                    for (size_t t = 0; t < leaf.size(); ++t) {
                        if (!((B >> t) & 1)) continue;
                        int8_t l = p.lab[leaf[t]];
                        if (l >= 0) {
                            if (lb >= 0 && lb != l) conflict = true;
                            lb = l;
                        }
                    }
                    q.lab[nq] = lb;
                    bidx.push_back(nq++);
                }
                if (conflict) continue;
                q.k = nq;
                for (int a = 0; a < k; ++a)
                    for (int b2 = a + 1; b2 < k; ++b2)
                        if (((core >> a) & 1) && ((core >> b2) & 1) && has_edge(p.em, a, b2))
                            q.em |= 1u << pair_bit(idx[a], idx[b2]);
                for (size_t bi = 0; bi < blocks.size(); ++bi)
                    for (size_t t = 0; t < leaf.size(); ++t) {
                        if (!((blocks[bi] >> t) & 1)) continue;
                        for (int cv = 0; cv < k; ++cv)
                            if (((core >> cv) & 1) && has_edge(p.em, leaf[t], cv))
                                q.em |= 1u << pair_bit(bidx[bi], idx[cv]);
                    }
                int64_t aq = (int64_t)automorphisms(q).size();
                Pat cq = canonical(q);
                cq.vi = false;
                subw[{cq.em | ((uint32_t)cq.k << 24), cq.lab}] += aq;
            }
        }
        d.lane_par = 1;
        for (int q = 0; q < d.nterm; ++q)
            if (!d.term[q].cheap && !d.term[q].agg) d.lane_par = 0;
        d.agg_last = agg_last ? 1 : 0;
        // clique with a total ascending order: every level lies in the
        // out-neighbourhood of the root and above all earlier levels
        d.local = 0;
        if (p.em == full_mask(k) && c == k && k >= 3 && d.nterm == 0 && !agg_last && d.mult == 1 &&
            gs.max_out <= LOCAL_MAX) {
            bool ok = true;
            for (int j = 1; j < c; ++j) {
                uint8_t below = (uint8_t)((1u << j) - 1u);
                if (d.lev[j].adj != below || d.lev[j].gt != below || d.lev[j].anti || d.lev[j].label >= 0)
                    ok = false;
            }
            d.local = ok ? 1 : 0;
        }

        out->d = d;
        out->pat = p;
        out->divisor = divisor;
        for (int j = 0; j < KMAX; ++j) out->order[j] = j < c ? (int8_t)order[j] : -1;
        out->formulation = form;
        out->est_cost = estimate(out->d);
        out->total_cost = out->est_cost;
        out->rewrite = product_only;
        out->subs.clear();
        if (product_only) {
            out->hmult = hc_size;
            out->autp = (int64_t)autp.size();
            for (auto& e : subw) {
                Pat q;
                q.k = (int)(e.first.first >> 24);
                q.em = e.first.first & 0xffffffu;
                q.vi = false;
                q.lab = e.first.second;
                out->subs.push_back({q, e.second});
            }
        }
        return true;
    }

    // A plan, and its root-bitmap variant when some probe may test N(v0).
    void add(const PlanInfo& pi, std::vector<PlanInfo>* out) const {
        out->push_back(pi);
        const DPlan& d = pi.d;
        if (d.local || d.agg_last || d.ncore < 2) return;
        bool probes0 = false;
        for (int j = 2; j < d.ncore; ++j) {
            const DLevel& L = d.lev[j];
            uint8_t m = L.adj | L.anti;
            if (L.base != 0xff) m = (uint8_t)((L.adj & ~d.lev[L.base].adj) | (L.anti & ~d.lev[L.base].anti));
            if (m & 1) probes0 = true;
        }
        for (int q = 0; q < d.nterm; ++q) {
            const DTerm& t = d.term[q];
            if (!t.cheap && !t.agg && ((t.adj | t.anti) & 1)) probes0 = true;
        }
        if (!probes0) return;
        PlanInfo pb = pi;
        pb.d.bm0 = 1;
        pb.est_cost = estimate(pb.d);
        pb.total_cost = pb.est_cost;
        out->push_back(pb);
    }

    // ---- cost model -------------------------------------------------------
    // Expected work from degree statistics.  The first two levels use exact
    // joint sums over the degree sequence (power-law graphs make degrees of
    // adjacent levels strongly correlated); deeper levels use neighbour
    // averages.  A list bounded below by its owner is an out-list of the
    // degree-ordered orientation (short), bounded above an in-list.
    // type: +1 out-list, -1 in-list, 0 whole list.
    static int list_type(const DLevel& L, int owner) {
        if ((L.gt >> owner) & 1) return 1;
        if ((L.lt >> owner) & 1) return -1;
        return 0;
    }
    double root_sum(int type) const {  // sum over roots of one list of the root
        return type == 0 ? 2.0 * gs.m : gs.m;
    }
    // sum over (v0, v1) pairs of the length of a list of v0 (owner 0) or v1
    double pair_sum(int rel, int owner, int type) const {
        // rel: +1 v1 in N+(v0), -1 v1 in N-(v0), 0 either
        auto S = [&](char a, char b) {  // sum_v a(v) b(v)
            auto key = std::string() + a + b;
            if (key == "pp") return gs.s_pp;
            if (key == "pq" || key == "qp") return gs.s_pq;
            if (key == "pd" || key == "dp") return gs.s_pd;
            if (key == "qq") return gs.s_qq;
            if (key == "qd" || key == "dq") return gs.s_qd;
            return gs.s_dd;
        };
        char t = type > 0 ? 'p' : (type < 0 ? 'q' : 'd');
        if (rel == 0) return pair_sum(1, owner, type) + pair_sum(-1, owner, type);
        if (owner == 0) return S(rel > 0 ? 'p' : 'q', t);
        return S(rel > 0 ? 'q' : 'p', t);
    }
    double estimate(const DPlan& d) const {
        if (d.local) {
            // row build: merge of each out-list with the root's out-list;
            // counting: word operations per local edge and deeper level
            double rows = gs.s_pq + gs.s_pp;
            return gs.n + rows * 0.5 + gs.s_pp * 0.1 * (d.ncore - 2);
        }
        const double n = std::max(gs.n, 1.0);
        const double m = std::max(gs.m, 1.0);
        double deg_nb = std::max(gs.nbr_deg, 1.0), out_nb = std::max(gs.nbr_out, 0.5);
        double keep = std::min(1.0, std::max(0.02, deg_nb / n * 8.0));
        auto nb_len = [&](int type) {
            if (type > 0) return out_nb;
            if (type < 0) return std::max(deg_nb - out_nb, 1.0);
            return deg_nb;
        };
        double prefixes = n;   // partial matches entering the next level
        double cost = n;
        int rel1 = 0;          // how v1 relates to v0
        const int last = d.ncore - 1;
        for (int j = 1; j < d.ncore; ++j) {
            const DLevel& L = d.lev[j];
            double total, work;
            if (L.agg) {
                int s = d.bridge_src;
                int bt = ((d.bridge_gt >> s) & 1) ? 1 : (((d.bridge_lt >> s) & 1) ? -1 : 0);
                double bridges = (j == 1) ? root_sum(bt) : prefixes * nb_len(bt);
                // second hop: the bridge's list, bounded like the target
                int tt = 0;
                for (int i = 0; i < j; ++i)
                    if ((L.lt >> i) & 1) tt = -1;
                double hop = (bt < 0 && tt < 0) ? gs.s_pd / m : (tt < 0 ? deg_nb * 0.5 : deg_nb);
                work = bridges * hop * 1.5;
                total = std::min(bridges * hop, prefixes * n);
                cost += work;
                prefixes = std::max(total, 1e-9);
                continue;
            }
            double best = 1e300;
            int bi = 0;
            for (int i = 0; i < j; ++i) {
                if (!((L.adj >> i) & 1)) continue;
                int type = list_type(L, i);
                double sum;
                if (j == 1) sum = root_sum(type);
                else if (j == 2 && i <= 1) sum = pair_sum(rel1, i, type);
                else sum = prefixes * nb_len(type);
                if (sum < best) {
                    best = sum;
                    bi = i;
                }
            }
            if (j == 1) {
                for (int i = 0; i < 1; ++i) rel1 = list_type(L, 0);
            }
            int extra = popc(L.adj) - 1 + popc(L.anti);
            total = best * std::pow(keep, popc(L.adj) - 1);
            work = best * (1.0 + extra * 2.0);
            // a probe of N(v0) on the root bitmap costs one load, not a search
            if (d.bm0 && j >= 2 && ((L.anti & 1) || ((L.adj & 1) && bi != 0))) work -= best * BM_SAVING;
            bool counted = (j == last && d.nterm == 0);
            cost += work;
            if (!counted) prefixes = std::max(total, 1e-9);
        }
        // tail terms per full core match
        double tail_work = 0;
        for (int q = 0; q < d.nterm; ++q) {
            const DTerm& t = d.term[q];
            if (t.agg) {
                tail_work += prefixes * 0.5;
                continue;
            }
            if (t.cheap) {
                tail_work += prefixes * (1.0 + 2.0 * popc(t.neq & ~t.sure));
                continue;
            }
            double best = 1e300;
            int bi = 0;
            for (int i = 0; i < d.ncore; ++i) {
                if (!((t.adj >> i) & 1)) continue;
                int type = ((t.gt >> i) & 1) ? 1 : (((t.lt >> i) & 1) ? -1 : 0);
                double sum;
                if (d.ncore == 1) sum = root_sum(type);
                else if (d.ncore == 2 && !d.agg_last) sum = pair_sum(rel1, i, type);
                else sum = prefixes * nb_len(type);
                if (sum < best) {
                    best = sum;
                    bi = i;
                }
            }
            tail_work += best * (1.0 + (popc(t.adj) - 1 + popc(t.anti)) * 2.0) + prefixes * 4.0;
            if (d.bm0 && ((t.anti & 1) || ((t.adj & 1) && bi != 0))) tail_work -= best * BM_SAVING;
        }
        cost += tail_work;
        // building and clearing the root bitmap: two passes over N(v0)
        if (d.bm0) cost += 2.0 * root_sum(0);
        return cost;
    }
    static constexpr double BM_SAVING = 1.5;
};

void orders_of(const Pat& p, uint32_t core, bool agg_last, std::vector<std::vector<int>>* out) {
    std::vector<int> verts;
    for (int v = 0; v < p.k; ++v)
        if ((core >> v) & 1) verts.push_back(v);
    std::sort(verts.begin(), verts.end());
    do {
        bool ok = true;
        int c = (int)verts.size();
        for (int j = 1; j < c && ok; ++j) {
            bool adj = false;
            for (int i = 0; i < j; ++i)
                if (has_edge(p.em, verts[i], verts[j])) adj = true;
            if (agg_last && j == c - 1) ok = !adj;
            else ok = adj;
        }
        if (ok) out->push_back(verts);
    } while (std::next_permutation(verts.begin(), verts.end()));
}

}  // namespace

std::string PlanInfo::describe() const {
    char buf[512];
    std::string s;
    snprintf(buf, sizeof(buf), "k=%d em=0x%x %s form=%s div=%lld cost=%.3g total=%.3g order=", pat.k,
             pat.em, pat.vi ? "VI" : "EI", formulation ? "pattern" : "coset",
             (long long)divisor, est_cost, total_cost);
    s += buf;
    for (int j = 0; j < d.ncore; ++j) s += std::to_string(order[j]) + (j + 1 < d.ncore ? "," : "");
    for (int j = 0; j < d.ncore; ++j) {
        const DLevel& L = d.lev[j];
        snprintf(buf, sizeof(buf), " | L%d adj=%x anti=%x gt=%x lt=%x neq=%x lab=%d base=%d%s", j,
                 L.adj, L.anti, L.gt, L.lt, L.neq, L.label, L.base == 0xff ? -1 : L.base,
                 L.agg ? " AGG" : "");
        s += buf;
    }
    for (int q = 0; q < d.nterm; ++q) {
        const DTerm& t = d.term[q];
        snprintf(buf, sizeof(buf), " | T%d adj=%x anti=%x gt=%x lt=%x neq=%x lab=%d%s%s", q, t.adj,
                 t.anti, t.gt, t.lt, t.neq, t.label, t.cheap ? " cheap" : "", t.agg ? " agg" : "");
        s += buf;
    }
    s += " | poly:";
    for (int m = 0; m < d.nmono; ++m) {
        snprintf(buf, sizeof(buf), " %+lld", (long long)d.mono[m].coef);
        s += buf;
        for (int f = 0; f < d.mono[m].nf; ++f) s += "*T" + std::to_string(d.mono[m].f[f]);
    }
    if (d.nterm == 0) s += " mult=" + std::to_string(d.mult);
    if (rewrite) {
        snprintf(buf, sizeof(buf), " | quotient: (%lld*sum", (long long)hmult);
        s += buf;
        for (auto& q : subs) {
            snprintf(buf, sizeof(buf), " - %lld*N(k=%d em=0x%x)", (long long)q.second, q.first.k, q.first.em);
            s += buf;
        }
        snprintf(buf, sizeof(buf), ")/%lld", (long long)autp);
        s += buf;
    }
    if (cyc5) s += " | cycle5 pair sum minus the companion triangle plan";
    if (d.tagg == TAGG_BOWTIE) s += " | triangle counts: bowtie";
    if (d.tagg == TAGG_TRIPATH) s += " | triangle counts: triangle with a two-edge path";
    if (d.tagg == TAGG_HOUSE) s += " | triangle counts: house (4-cycle support sums)";
    if (d.tagg == TAGG_TAILED) s += " | triangle counts: tailed triangle";
    if (d.tagg == TAGG_TRIANGLE) s += " | triangle counts: triangle";
    if (d.tagg == TAGG_K4EAR) s += " | triangle counts: 4-clique with an ear (per 4-clique)";
    if (d.tagg == TAGG_DTAIL) s += " | triangle counts: diamond with a pendant at a tip (per triangle)";
    if (d.tagg == TAGG_FAN) s += " | triangle counts: fan of three triangles (per triangle)";
    if (d.lane_par) s += " lane_par";
    if (d.local) s += " local_bitmap";
    if (d.bm0) s += " root_bitmap";
    if (clique_ok(d)) s += " triangle_core";
    if (clique4_ok(d)) s += " clique4";
    if (!clique_ok(d) && support_ok(d)) s += " edge_support";
    return s;
}

int candidate_plans(const Pat& p, const GraphStats& gs, std::vector<PlanInfo>* out, std::string* err) {
    out->clear();
    if (p.k < 2 || p.k > KMAX) {
        *err = "pattern size outside 2..5";
        return PM_E_UNSUPPORTED;
    }
    if (!is_connected(p.k, p.em) || (p.em & ~full_mask(p.k))) {
        *err = "pattern must be connected with edges among its k vertices";
        return PM_E_UNSUPPORTED;
    }
    Group autp = automorphisms(p);
    Builder B(p, gs);
    const int k = p.k;
    uint32_t all = (1u << k) - 1u;
    for (uint32_t leaves = 0; leaves < (1u << k); ++leaves) {
        uint32_t core = all & ~leaves;
        if (!core) continue;
        int nl = popc(leaves);
        if (nl > MAX_LEAF) continue;
        // leaves: no constraint between any two of them
        bool indep = true;
        for (int a = 0; a < k; ++a)
            for (int b = a + 1; b < k; ++b)
                if (((leaves >> a) & 1) && ((leaves >> b) & 1)) {
                    if (has_edge(p.em, a, b) || p.vi) indep = false;
                }
        if (!indep) continue;
        for (int agg = 0; agg < 2; ++agg) {
            if (agg && (p.vi || popc(core) < 2)) continue;
            std::vector<std::vector<int>> orders;
            orders_of(p, core, agg != 0, &orders);
            for (const auto& ord : orders)
                for (int form = 0; form < 2; ++form)
                    for (int dir = -1; dir <= 1; dir += 2) {
                        PlanInfo pi;
                        if (B.build(core, leaves, ord, form, dir, agg != 0, autp, &pi)) B.add(pi, out);
                        if (!agg && form == 0 && !p.vi && popc(leaves) >= 2) {
                            PlanInfo pq;
                            if (B.build(core, leaves, ord, form, dir, false, autp, &pq, true)) B.add(pq, out);
                        }
                    }
        }
    }
    if (out->empty()) {
        *err = "no valid plan";
        return PM_E_UNSUPPORTED;
    }
    return PM_OK;
}

Pat cycle5_aux_pattern() {
    Pat a;
    a.k = 3;
    a.em = 0x7;
    a.vi = false;
    for (int i = 0; i < 3; ++i) a.lab[i] = -2;
    return a;
}

// Edge-induced, unlabeled 5-cycle: every cycle once, at its lowest vertex a
// (degree-order ids), as the sum over the edges {x < y} opposite a of
// (A(x) - [y in N+(a)]) (A(y) - [x in N+(a)]), where A(t) counts the
// out-neighbours of a adjacent to t > a (cycle5_kernel), minus the choices
// with both bridges equal: one out-neighbour b of a closing a triangle
// {b, x, y} above a.  Summed over a, those are, for every triangle
// {u < v < w}, the neighbours of u, v and w below u: the companion plan, a
// triangle core v0 < v1 < v2 with the cheap terms |N(v_i) n [0, v0)|.
static void cycle5_plans(const GraphStats& gs, PlanInfo* pc, PlanInfo* aux) {
    DPlan d;
    memset(&d, 0, sizeof(d));
    d.ncore = 1;
    d.mult = 1;
    d.cyc5 = 1;
    d.bridge_src = 0xff;
    d.lev[0].base = 0xff;
    d.lev[0].label = -1;
    pc->d = d;
    pc->divisor = 1;
    pc->cyc5 = true;
    pc->formulation = 0;
    for (int j = 0; j < KMAX; ++j) pc->order[j] = j < 1 ? 0 : -1;
    // cost: the fill streams N(b) above a for every out-neighbour b of a
    // (about sum_b d(b) d-(b)), the scan reads N+(x) for every target
    pc->est_cost = gs.s_pd + gs.s_qd * std::max(gs.avg_out, 1.0);
    pc->total_cost = pc->est_cost;
    pc->subs.clear();
    pc->subs.push_back({cycle5_aux_pattern(), 1});

    DPlan t;
    memset(&t, 0, sizeof(t));
    t.ncore = 3;
    t.mult = 1;
    t.bridge_src = 0xff;
    for (int j = 0; j < 3; ++j) {
        t.lev[j].base = 0xff;
        t.lev[j].label = -1;
    }
    t.lev[1].adj = 1;
    t.lev[1].gt = 1;
    t.lev[2].adj = 3;
    t.lev[2].gt = 3;
    t.lev[2].base = 1;
    t.nterm = 3;
    for (int q = 0; q < 3; ++q) {
        DTerm& m = t.term[q];
        m.adj = (uint8_t)(1u << q);
        m.lt = 1;
        m.label = -1;
        m.cheap = 1;
        m.neq = (uint8_t)(7u & ~(m.adj | m.lt));
        for (int i = 0; i < 3; ++i)
            if ((m.neq >> i) & 1) m.sure |= (uint8_t)(1u << i);
    }
    t.nmono = 3;
    for (int q = 0; q < 3; ++q) {
        t.mono[q].coef = 1;
        t.mono[q].nf = 1;
        t.mono[q].f[0] = (uint8_t)q;
    }
    t.lane_par = 1;
    aux->d = t;
    aux->pat = cycle5_aux_pattern();
    aux->divisor = 1;
    aux->formulation = 0;
    for (int j = 0; j < KMAX; ++j) aux->order[j] = j < 3 ? (int8_t)j : -1;
    aux->est_cost = gs.s_pp + gs.m;
    aux->total_cost = aux->est_cost;
}

// Patterns with a closed form over triangle counts (tagg_kind): no levels
// or terms; the cost is the triangle pass that fills the per-edge counts
// (about the out-wedges, s_pp) and a few passes over the edges, and for the
// house two streams of every bridge's list below its higher end (about
// sum_a d(a) d+(a), s_pd).
static void tagg_plan(const Pat& p, int kind, const GraphStats& gs, PlanInfo* out) {
    DPlan d;
    memset(&d, 0, sizeof(d));
    d.ncore = 1;
    d.mult = 1;
    d.tagg = kind;
    d.bridge_src = 0xff;
    d.lev[0].base = 0xff;
    d.lev[0].label = -1;
    out->d = d;
    out->pat = p;
    out->divisor = kind == TAGG_TAILED || kind == TAGG_K4EAR ? 2 : (kind == TAGG_TRIANGLE ? 3 : 1);
    out->formulation = 0;
    for (int j = 0; j < KMAX; ++j) out->order[j] = j < 1 ? 0 : -1;
    out->est_cost = gs.s_pp + 4 * gs.m + gs.n + (kind == TAGG_HOUSE ? 2 * gs.s_pd : 0.0) +
                    (tagg_tri(kind) ? gs.s_pq : 0.0) + (kind == TAGG_K4EAR ? 2 * gs.s_pq : 0.0);
    out->total_cost = out->est_cost;
    out->subs.clear();
    if (tagg_tri(kind)) {
        // the per-triangle sum counts each 4-clique twelve times too many
        Pat k4;
        k4.k = 4;
        k4.em = full_mask(4);
        k4.vi = false;
        out->rewrite = true;
        out->hmult = 1;
        out->autp = 1;
        out->subs.push_back({k4, 12});
    }
}

int compile_plan(const Pat& p, const GraphStats& gs, PlanInfo* out, std::string* err, bool tri) {
    if (tri) {
        const int kind = tagg_kind(p);
        if (kind) {
            tagg_plan(p, kind, gs, out);
            return PM_OK;
        }
    }
    if (p.k == 3 && p.lab[0] == -2) {
        PlanInfo pc;
        cycle5_plans(gs, &pc, out);
        return PM_OK;
    }
    if (is_cycle5(p)) {
        PlanInfo aux;
        cycle5_plans(gs, out, &aux);
        out->pat = p;
        return PM_OK;
    }
    std::vector<PlanInfo> all;
    int rc = candidate_plans(p, gs, &all, err);
    if (rc) return rc;
    // cost of every sub-pattern a quotient plan needs (its own best plan)
    std::map<std::pair<uint32_t, std::array<int8_t, 8>>, double> sub_cost;
    for (PlanInfo& pi : all) {
        double extra = 0;
        for (auto& sq : pi.subs) {
            auto key = std::make_pair(sq.first.em | ((uint32_t)sq.first.k << 24), sq.first.lab);
            auto it = sub_cost.find(key);
            if (it == sub_cost.end()) {
                PlanInfo sp;
                std::string e2;
                double c = 1e300;
                if (compile_plan(sq.first, gs, &sp, &e2, tri) == PM_OK) c = sp.total_cost;
                it = sub_cost.emplace(key, c).first;
            }
            extra += it->second;
        }
        pi.total_cost = pi.est_cost + extra;
    }
    // The estimate multiplies per-level survival fractions as if adjacency
    // constraints were independent, which undercounts the partial matches of
    // deep dense cores on clustered graphs: on R-MAT 15 it preferred a plan
    // enumerating all five levels of the K4-with-ear (0xff) over one
    // enumerating three, and took 30 s instead of a fraction of one; on
    // R-MAT 18 four-level plans of the wheel (0x1fb) and of K_{2,3} plus an
    // edge (0xfe), estimated below the three-level ones by a factor of up to
    // four, took 94 s and more than 180 s against a few seconds.  Each
    // enumerated core level beyond three therefore ranks DEEP_PENALTY times
    // dearer when choosing (est_cost itself stays as estimated); cliques
    // counted on the root's local bitmap are exempt.
    auto ranked = [](const PlanInfo& pi) {
        if (pi.d.local) return pi.total_cost;   // deep levels on the root's local bitmap
        return pi.total_cost * std::pow(DEEP_PENALTY, (double)std::max(0, pi.d.ncore - 3));
    };
    size_t best = 0;
    for (size_t i = 1; i < all.size(); ++i)
        if (ranked(all[i]) < ranked(all[best])) best = i;
    *out = all[best];
    return PM_OK;
}

}  // namespace pm
