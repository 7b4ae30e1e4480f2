// Pattern algebra for morphing (host side).
//
// Section 3.2.1 (definitions): subgraph isomorphisms between two patterns
// on the same vertices are permutations; phi(p,q) is their set.  The morph
// coefficient of q in the expansion of p^E is |phi(p^E,q^E)| / |Aut(p)|:
// the number of distinct copies of p inside one copy of q.  Theorem 3.1
// (counting form): N_E(p) = sum over same-size superpatterns q (p itself
// included) of coef(p,q) * N_V(q).  Corollary 3.1: the vertex-induced
// count follows by back-substitution, ending at the clique.  Section 4.2
// "Naive PMR": vertex-induced queries are answered from edge-induced counts
// of their superpatterns (and the clique).
#include <algorithm>
#include <functional>
#include <map>

#include "internal.hpp"

namespace pm {

uint32_t permute_mask(int k, uint32_t m, const Perm& p) {
    uint32_t out = 0;
    for (int j = 1; j < k; ++j)
        for (int i = 0; i < j; ++i)
            if (has_edge(m, i, j)) out |= 1u << pair_bit(p[i], p[j]);
    return out;
}

bool is_connected(int k, uint32_t m) {
    if (k <= 1) return true;
    uint32_t seen = 1, frontier = 1;
    while (frontier) {
        uint32_t next = 0;
        for (int x = 0; x < k; ++x) {
            if (!((frontier >> x) & 1)) continue;
            for (int y = 0; y < k; ++y)
                if (y != x && !((seen >> y) & 1) && has_edge(m, x, y)) next |= 1u << y;
        }
        seen |= next;
        frontier = next;
    }
    return seen == (1u << k) - 1;
}

std::vector<Perm> all_perms(int k) {
    std::vector<Perm> out;
    Perm p{};
    for (int i = 0; i < 8; ++i) p[i] = (uint8_t)i;
    do {
        out.push_back(p);
    } while (std::next_permutation(p.begin(), p.begin() + k));
    return out;
}

static bool labels_carried(const Pat& p, const Pat& q, const Perm& f) {
    for (int i = 0; i < p.k; ++i)
        if (p.lab[i] != q.lab[f[i]]) return false;
    return true;
}

Pat canonical(const Pat& p) {
    Pat best;
    bool have = false;
    for (const Perm& f : all_perms(p.k)) {
        Pat c;
        c.k = p.k;
        c.vi = p.vi;
        c.em = permute_mask(p.k, p.em, f);
        for (int i = 0; i < p.k; ++i) c.lab[f[i]] = p.lab[i];
        if (!have || c.em < best.em || (c.em == best.em && c.lab < best.lab)) {
            best = c;
            have = true;
        }
    }
    // a clique is both vertex- and edge-induced; keep one form
    if (best.em == full_mask(best.k)) best.vi = false;
    return best;
}

std::vector<Perm> automorphisms(const Pat& p) {
    std::vector<Perm> out;
    for (const Perm& f : all_perms(p.k))
        if (permute_mask(p.k, p.em, f) == p.em && labels_carried(p, p, f)) out.push_back(f);
    return out;
}

int64_t injections(const Pat& p, const Pat& q) {
    int64_t c = 0;
    for (const Perm& f : all_perms(p.k)) {
        if (!labels_carried(p, q, f)) continue;
        if (permute_mask(p.k, p.em, f) & ~q.em) continue;
        ++c;
    }
    return c;
}

static bool pat_less(const Pat& a, const Pat& b) {
    if (a.k != b.k) return a.k < b.k;
    if (a.em != b.em) return a.em < b.em;
    if (a.vi != b.vi) return a.vi < b.vi;
    return a.lab < b.lab;
}

// coefficient c(p,q) = injections / |Aut(p)| on edge-induced forms
static int64_t coef(const Pat& p, const Pat& q) {
    int64_t inj = injections(p, q);
    int64_t aut = (int64_t)automorphisms(p).size();
    return inj / aut;
}

// Same-size superpatterns of p: p with extra edges among its own vertices,
// canonicalised (labels travel with the vertices).
static std::vector<Pat> superpatterns(const Pat& p) {
    std::vector<Pat> out;
    uint32_t free_pairs = full_mask(p.k) & ~p.em;
    std::vector<int> bits;
    for (int b = 0; b < 32; ++b)
        if ((free_pairs >> b) & 1) bits.push_back(b);
    for (uint32_t s = 0; s < (1u << bits.size()); ++s) {
        Pat q = p;
        q.vi = false;
        for (size_t t = 0; t < bits.size(); ++t)
            if ((s >> t) & 1) q.em |= 1u << bits[t];
        Pat c = canonical(q);
        c.vi = false;
        bool dup = false;
        for (const Pat& o : out)
            if (o == c) dup = true;
        if (!dup) out.push_back(c);
    }
    return out;
}

// Cost-based alternative sets (Section 4.1's optimizer, Table 4's mixed
// sets).  Over the up-closed set U of the queries' same-size superpatterns,
// each pattern u is matched vertex-induced (V), edge-induced (E) or not at
// all.  N_V(u) is known when u is matched V, or matched E and every strict
// superpattern's N_V is known (Corollary 3.1 from the top).  A
// vertex-induced query needs its N_V known; an edge-induced query is matched
// E or needs N_V known for itself and every strict superpattern (Theorem
// 3.1).  The cheapest assignment is searched exhaustively when U has at
// most MIX_EXHAUSTIVE patterns; otherwise the cheaper of "every query as
// given" and "every pattern of U by its cheaper form" is taken (for motif
// counting, where every pattern is a query, the latter is optimal).
static constexpr size_t MIX_EXHAUSTIVE = 9;

int morph_plan_mixed(const std::vector<Pat>& qs, const std::function<double(const Pat&)>& cost, MorphPlan* out,
                     std::string* err) {
    out->alt.clear();
    out->matrix.clear();
    // U: edge-induced canonical forms, most edges first
    std::vector<Pat> U;
    std::vector<Pat> qc(qs.size());
    auto index_of = [&](const Pat& e) -> int {
        for (size_t i = 0; i < U.size(); ++i)
            if (U[i] == e) return (int)i;
        return -1;
    };
    for (size_t i = 0; i < qs.size(); ++i) {
        qc[i] = canonical(qs[i]);
        for (const Pat& q : superpatterns(qc[i]))
            if (index_of(q) < 0) U.push_back(q);
    }
    std::sort(U.begin(), U.end(), [](const Pat& a, const Pat& b) {
        int ea = popc(a.em), eb = popc(b.em);
        if (ea != eb) return ea > eb;
        return pat_less(a, b);
    });
    const size_t nu = U.size();
    // sup[u][w]: c(u, w) for every superpattern w of u (w != u), 0 otherwise
    std::vector<std::vector<int64_t>> c(nu, std::vector<int64_t>(nu, 0));
    for (size_t u = 0; u < nu; ++u)
        for (const Pat& w : superpatterns(U[u])) {
            int j = index_of(w);
            if (j >= 0 && (size_t)j != u) c[u][j] = coef(U[u], w);
        }
    std::vector<double> cV(nu), cE(nu);
    std::vector<bool> clique(nu);
    for (size_t u = 0; u < nu; ++u) {
        clique[u] = U[u].em == full_mask(U[u].k);
        Pat v = U[u];
        v.vi = !clique[u];
        cV[u] = cost(v);
        cE[u] = clique[u] ? cV[u] : cost(U[u]);
    }
    struct Q {
        int u;
        bool vi;
    };
    std::vector<Q> qv(qs.size());
    for (size_t i = 0; i < qs.size(); ++i) {
        Pat e = qc[i];
        e.vi = false;
        qv[i] = {index_of(e), qc[i].vi && qc[i].em != full_mask(qc[i].k)};
    }
    // d[u]: 0 none, 1 V, 2 E (cliques: 0 or 2)
    auto known = [&](const std::vector<int>& d, std::vector<bool>* K) {
        K->assign(nu, false);
        for (size_t u = 0; u < nu; ++u) {   // most edges first: supersets decided
            if (d[u] == 1) {
                (*K)[u] = true;
            } else if (d[u] == 2) {
                bool all = true;
                for (size_t w = 0; w < nu && all; ++w)
                    if (c[u][w] && !(*K)[w]) all = false;
                (*K)[u] = all;
            }
        }
    };
    auto feasible = [&](const std::vector<int>& d, const std::vector<bool>& K) {
        for (const Q& q : qv) {
            if (q.vi) {
                if (!K[q.u]) return false;
            } else if (d[q.u] != 2) {
                if (!K[q.u]) return false;
                for (size_t w = 0; w < nu; ++w)
                    if (c[q.u][w] && !K[w]) return false;
            }
        }
        return true;
    };
    auto total = [&](const std::vector<int>& d) {
        double t = 0;
        for (size_t u = 0; u < nu; ++u) t += d[u] == 1 ? cV[u] : (d[u] == 2 ? cE[u] : 0.0);
        return t;
    };
    std::vector<int> best;
    double best_cost = 0;
    std::vector<bool> K;
    if (nu <= MIX_EXHAUSTIVE) {
        std::vector<int> d(nu, 0);
        uint64_t combos = 1;
        for (size_t u = 0; u < nu; ++u) combos *= 3;
        for (uint64_t x = 0; x < combos; ++x) {
            uint64_t y = x;
            bool skip = false;
            for (size_t u = 0; u < nu; ++u) {
                d[u] = (int)(y % 3);
                y /= 3;
                if (clique[u] && d[u] == 1) skip = true;
            }
            if (skip) continue;
            known(d, &K);
            if (!feasible(d, K)) continue;
            const double t = total(d);
            if (best.empty() || t < best_cost) {
                best = d;
                best_cost = t;
            }
        }
    } else {
        std::vector<int> a(nu, 0), b(nu, 0);
        for (const Q& q : qv) a[q.u] = (q.vi ? 1 : 2);
        for (size_t u = 0; u < nu; ++u) b[u] = clique[u] ? 2 : (cV[u] < cE[u] ? 1 : 2);
        known(a, &K);
        const bool fa = feasible(a, K);
        best = b;
        best_cost = total(b);
        if (fa && total(a) <= best_cost) best = a;
    }
    if (best.empty()) {
        *err = "internal: no feasible alternative set";
        return PM_E_INVAL;
    }
    known(best, &K);
    // alternatives and integer rows (symbolic Corollary 3.1 from the top)
    std::vector<int> alt_of(nu, -1);
    for (size_t u = 0; u < nu; ++u)
        if (best[u]) {
            Pat a = U[u];
            a.vi = best[u] == 1;
            alt_of[u] = (int)out->alt.size();
            out->alt.push_back(a);
        }
    const size_t na = out->alt.size();
    std::vector<std::vector<__int128>> NV(nu, std::vector<__int128>(na, 0));
    for (size_t u = 0; u < nu; ++u) {
        if (!K[u]) continue;
        NV[u][alt_of[u]] = 1;
        if (best[u] == 2)
            for (size_t w = 0; w < nu; ++w)
                if (c[u][w])
                    for (size_t j = 0; j < na; ++j) NV[u][j] -= (__int128)c[u][w] * NV[w][j];
    }
    out->matrix.assign(qs.size() * na, 0);
    for (size_t i = 0; i < qs.size(); ++i) {
        const Q& q = qv[i];
        std::vector<__int128> row(na, 0);
        if (q.vi) {
            row = NV[q.u];
        } else if (best[q.u] == 2) {
            row[alt_of[q.u]] = 1;
        } else {
            row = NV[q.u];
            for (size_t w = 0; w < nu; ++w)
                if (c[q.u][w])
                    for (size_t j = 0; j < na; ++j) row[j] += (__int128)c[q.u][w] * NV[w][j];
        }
        for (size_t j = 0; j < na; ++j) {
            if (row[j] > INT64_MAX || row[j] < INT64_MIN) {
                *err = "morph coefficient outside int64";
                return PM_E_OVERFLOW;
            }
            out->matrix[i * na + j] = (int64_t)row[j];
        }
    }
    return PM_OK;
}

int morph_plan_count(const std::vector<Pat>& qs, int morph, MorphPlan* out, std::string* err,
                     const std::function<double(const Pat&)>& cost) {
    if (morph == PM_MORPH_COST && cost) return morph_plan_mixed(qs, cost, out, err);
    out->alt.clear();
    out->matrix.clear();
    std::vector<std::vector<std::pair<Pat, int64_t>>> rows(qs.size());
    for (size_t i = 0; i < qs.size(); ++i) {
        Pat p = canonical(qs[i]);
        bool clique = p.em == full_mask(p.k);
        if (morph == PM_MORPH_NONE || !p.vi || clique) {
            rows[i].push_back({p, 1});
            continue;
        }
        // lattice over the edge-induced superpatterns, most edges first
        std::vector<Pat> L = superpatterns(p);
        std::sort(L.begin(), L.end(), [](const Pat& a, const Pat& b) {
            int ea = popc(a.em), eb = popc(b.em);
            if (ea != eb) return ea > eb;
            return pat_less(a, b);
        });
        // Corollary 3.1 back-substitution, expressed in edge-induced counts:
        // N_V(r) = N_E(r) - sum_{s strictly above r} coef(r,s) N_V(s).
        // Each N_V(r) is kept as integer coefficients over the N_E of L.
        size_t nl = L.size();
        std::vector<std::vector<__int128>> nv(nl, std::vector<__int128>(nl, 0));
        for (size_t r = 0; r < nl; ++r) {
            nv[r][r] = 1;
            for (size_t s = 0; s < r; ++s) {
                if (popc(L[s].em) <= popc(L[r].em)) continue;
                int64_t c = coef(L[r], L[s]);
                if (!c) continue;
                for (size_t t = 0; t < nl; ++t) nv[r][t] -= (__int128)c * nv[s][t];
            }
        }
        // row of p itself (p's canonical edge-induced form is in L)
        Pat pe = p;
        pe.vi = false;
        size_t ip = nl;
        for (size_t r = 0; r < nl; ++r)
            if (L[r] == pe) ip = r;
        if (ip == nl) {
            *err = "internal: query missing from its own lattice";
            return PM_E_INVAL;
        }
        for (size_t t = 0; t < nl; ++t) {
            if (nv[ip][t] == 0) continue;
            if (nv[ip][t] > INT64_MAX || nv[ip][t] < INT64_MIN) {
                *err = "morph coefficient outside int64";
                return PM_E_OVERFLOW;
            }
            rows[i].push_back({L[t], (int64_t)nv[ip][t]});
        }
    }
    // union of alternative patterns
    for (auto& r : rows)
        for (auto& e : r) {
            bool dup = false;
            for (const Pat& a : out->alt)
                if (a == e.first) dup = true;
            if (!dup) out->alt.push_back(e.first);
        }
    size_t na = out->alt.size();
    out->matrix.assign(qs.size() * na, 0);
    for (size_t i = 0; i < qs.size(); ++i)
        for (auto& e : rows[i])
            for (size_t j = 0; j < na; ++j)
                if (out->alt[j] == e.first) out->matrix[i * na + j] += e.second;
    return PM_OK;
}

int unmorph(const MorphPlan& mp, size_t npat, const std::vector<int64_t>& alt_counts,
            std::vector<int64_t>* out, std::string* err) {
    size_t na = mp.alt.size();
    out->assign(npat, 0);
    for (size_t i = 0; i < npat; ++i) {
        __int128 acc = 0;
        for (size_t j = 0; j < na; ++j) {
            acc += (__int128)mp.matrix[i * na + j] * (__int128)alt_counts[j];
            if (acc > ((__int128)1 << 100) || acc < -((__int128)1 << 100)) {
                *err = "unmorph intermediate overflow";
                return PM_E_OVERFLOW;
            }
        }
        if (acc > INT64_MAX || acc < INT64_MIN) {
            *err = "unmorphed count outside int64";
            return PM_E_OVERFLOW;
        }
        (*out)[i] = (int64_t)acc;
    }
    return PM_OK;
}

}  // namespace pm
