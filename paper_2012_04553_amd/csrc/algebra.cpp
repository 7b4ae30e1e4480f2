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

int morph_plan_count(const std::vector<Pat>& qs, int morph, MorphPlan* out, std::string* err,
                     const std::function<double(const Pat&)>& cost) {
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
        if (morph == PM_MORPH_COST) {
            // Section 4.1 cost-based choice: morph only when matching the
            // edge-induced superpatterns is estimated cheaper than matching
            // the vertex-induced pattern itself
            double plain = cost ? cost(p) : 0.0, morphed = 0.0;
            for (const Pat& q : L) morphed += cost ? cost(q) : 0.0;
            if (cost && plain <= morphed) {
                rows[i].push_back({p, 1});
                continue;
            }
        }
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
