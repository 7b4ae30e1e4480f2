// Minimum-node-image support through pm_submit (host side): planning of the
// domain searches, direct and morphed, and their execution.
//
// MNI support (Preliminaries, FSM): the domain of pattern vertex v is the set
// of data vertices that some match maps v to; the support is the smallest
// domain.  Automorphic pattern vertices have equal domains, so one column
// per automorphism orbit is searched.
//
// Morphed route (Section 3.2.3, Theorem 3.2): every match of an
// edge-induced pattern p is a vertex-induced match of exactly one pattern
// p + S on the same vertices, S being the set of p's non-adjacent pairs
// whose images are adjacent; conversely every vertex-induced match of p + S
// is a match of p.  So the aggregation join is a union: the domain of v in
// p is the union over S of the domain of v in (p + S)^V.  Each p + S is
// searched in its canonical form, so the union reads, for each S, the
// column of the canonical vertex v maps to (the column permutation).  Union
// has no inverse, so only edge-induced patterns are morphed; vertex-induced
// ones are always searched directly.
//
// With existence searches the morphed route runs a superset of the direct
// route's work (one search per superpattern column instead of one per
// column), so PM_MORPH_COST takes the direct route for MNI.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <map>
#include <set>
#include <tuple>

#include "mni.hpp"
#include "runtime.hpp"

namespace pm {

namespace {

// Canonical form of p and the map of p's vertices onto it.
Pat canon_map(const Pat& p, Perm* f_out) {
    const Pat c = canonical(p);
    for (const Perm& f : all_perms(p.k)) {
        if (permute_mask(p.k, p.em, f) != c.em) continue;
        bool ok = true;
        for (int i = 0; i < p.k && ok; ++i) ok = c.lab[f[i]] == p.lab[i];
        if (ok) {
            *f_out = f;
            return c;
        }
    }
    *f_out = Perm{};
    return c;   // unreachable: canonical() is one of these images
}

int orbit_rep(const Pat& c, int v) {
    int best = v;
    for (const Perm& g : automorphisms(c)) best = std::min<int>(best, g[v]);
    return best;
}

// Existence search from pattern vertex u: step 0 = u, then repeatedly the
// unvisited vertex with the most edges to the visited ones (labeled first
// on ties), so constraints apply as early as possible.
MTask search_task(const Pat& c, int u, uint8_t* steps = nullptr) {
    MTask T;
    memset(&T, 0, sizeof(T));
    int order[KMAX];
    int step_of[8];
    for (int i = 0; i < 8; ++i) step_of[i] = -1;
    order[0] = u;
    step_of[u] = 0;
    for (int j = 1; j < c.k; ++j) {
        int best = -1, bscore = -1;
        for (int w = 0; w < c.k; ++w) {
            if (step_of[w] >= 0) continue;
            int links = 0;
            for (int i = 0; i < j; ++i) links += has_edge(c.em, w, order[i]);
            if (!links) continue;
            const int score = links * 2 + (c.lab[w] >= 0 ? 1 : 0);
            if (score > bscore) {
                bscore = score;
                best = w;
            }
        }
        order[j] = best;
        step_of[best] = j;
    }
    T.k = (uint8_t)c.k;
    for (int j = 0; j < c.k; ++j) {
        const int w = order[j];
        T.label[j] = c.lab[w];
        for (int i = 0; i < j; ++i) {
            if (has_edge(c.em, w, order[i])) T.adj[j] |= (uint8_t)(1u << i);
            else if (c.vi) T.anti[j] |= (uint8_t)(1u << i);
        }
    }
    for (int j = c.k; j < KMAX; ++j) T.label[j] = -1;
    if (steps)
        for (int j = 0; j < KMAX; ++j) steps[j] = j < c.k ? (uint8_t)order[j] : 0;
    return T;
}

using TaskKey = std::tuple<int, uint32_t, bool, std::array<int8_t, 8>, int>;

}  // namespace

int mni_plan(const std::vector<Pat>& qs, int morph, MniPlan* out, std::string* err) {
    *out = MniPlan();
    std::map<TaskKey, uint32_t> task_of;
    std::map<std::pair<uint32_t, std::array<int8_t, 8>>, uint32_t> alt_of;
    for (size_t i = 0; i < qs.size(); ++i) {
        const Pat& p = qs[i];
        if (p.k < 2 || p.k > KMAX || !is_connected(p.k, p.em) || (p.em & ~full_mask(p.k))) {
            *err = "MNI patterns must be connected with 2..5 vertices";
            return PM_E_UNSUPPORTED;
        }
        // the patterns whose columns make up p's domains: p itself, or every
        // p + S read vertex-induced
        std::vector<Pat> route;
        const bool morphed = morph == PM_MORPH_NAIVE && !p.vi && p.em != full_mask(p.k);
        if (!morphed) {
            route.push_back(p);
        } else {
            std::vector<int> nonedge;
            for (int b = 0; b < p.k * (p.k - 1) / 2; ++b)
                if (!((p.em >> b) & 1)) nonedge.push_back(b);
            for (uint32_t S = 0; S < (1u << nonedge.size()); ++S) {
                Pat q = p;
                q.vi = true;
                for (size_t t = 0; t < nonedge.size(); ++t)
                    if ((S >> t) & 1) q.em |= 1u << nonedge[t];
                route.push_back(q);
            }
        }
        std::vector<std::vector<uint32_t>> cols(p.k);
        std::vector<uint32_t> alts;
        for (const Pat& q : route) {
            Perm f;
            const Pat c = canon_map(q, &f);
            auto ak = std::make_pair(c.em | ((uint32_t)c.k << 24) | ((uint32_t)c.vi << 31), c.lab);
            auto ait = alt_of.find(ak);
            if (ait == alt_of.end()) {
                ait = alt_of.emplace(ak, (uint32_t)out->alt.size()).first;
                out->alt.push_back(c);
            }
            alts.push_back(ait->second);
            for (int v = 0; v < p.k; ++v) {
                const int u = orbit_rep(c, f[v]);
                TaskKey key{c.k, c.em, c.vi, c.lab, u};
                auto it = task_of.find(key);
                if (it == task_of.end()) {
                    it = task_of.emplace(key, (uint32_t)out->tasks.size()).first;
                    out->tasks.push_back(search_task(c, u));
                }
                if (std::find(cols[v].begin(), cols[v].end(), it->second) == cols[v].end())
                    cols[v].push_back(it->second);
            }
        }
        std::vector<uint32_t> qo;
        for (int v = 0; v < p.k; ++v) {
            MOut o;
            o.first = (uint32_t)out->list.size();
            o.count = (uint32_t)cols[v].size();
            out->list.insert(out->list.end(), cols[v].begin(), cols[v].end());
            qo.push_back((uint32_t)out->outs.size());
            out->outs.push_back(o);
        }
        out->qouts.push_back(qo);
        std::sort(alts.begin(), alts.end());
        alts.erase(std::unique(alts.begin(), alts.end()), alts.end());
        out->qalts.push_back(alts);
    }
    return PM_OK;
}

// Device layout of one MNI run: tasks | prefix | outs | list | counts +
// head | label order (the graph's, when labeled) | bitmaps.
struct MniLayout {
    uint64_t tasks = 0, prefix = 0, outs = 0, list = 0, counts = 0, head = 0, dom = 0, total = 0;
    uint64_t words = 0;
};

static uint64_t r256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

static MniLayout mni_layout(const GraphRes& G, const MniPlan& P) {
    MniLayout L;
    L.words = ((uint64_t)G.n + 31) / 32;
    uint64_t o = 0;
    L.tasks = o;
    o = r256(o + sizeof(MTask) * P.tasks.size());
    L.prefix = o;
    o = r256(o + 8 * (P.tasks.size() + 1));
    L.outs = o;
    o = r256(o + sizeof(MOut) * P.outs.size());
    L.list = o;
    o = r256(o + 4 * P.list.size());
    L.counts = o;
    o += 8 * P.outs.size();
    L.head = o;
    o = r256(o + 16);
    L.dom = o;
    o = r256(o + 4 * L.words * P.tasks.size());
    L.total = o;
    return L;
}

uint64_t Ctx_::mni_footprint(const GraphRes& G, const MniPlan& P) const {
    return mni_layout(G, P).total + (G.labeled && G.off_lorder == UINT64_MAX ? r256(4ull * G.n) : 0);
}

// The label-sorted vertex order on the device (kept with the graph).
int Ctx_::ensure_label_order(GraphRes& G) {
    if (!G.labeled || G.off_lorder != UINT64_MAX) return PM_OK;
    const uint64_t off = arena.alloc(4ull * G.n);
    if (off == UINT64_MAX) return fail(PM_E_NOMEM, "arena too small for the label order");
    HIPCHK(hipMemcpyAsync(dptr(off), G.label_order.data(), 4ull * G.n, hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
    G.off_lorder = off;
    return PM_OK;
}

// Upload the plan to `base` (arena offset of mni_layout(G, P).total bytes)
// and enqueue zero-fill, searches, unions and the copy of the column sizes
// to `host` (nout words) on stream s.
int Ctx_::enqueue_mni(GraphRes& G, const MniPlan& P, uint64_t base, unsigned long long* host, const int* cancel,
                      hipStream_t s) {
    const MniLayout L = mni_layout(G, P);
    std::vector<MTask> tasks = P.tasks;
    std::vector<uint64_t> prefix(tasks.size() + 1, 0);
    for (size_t t = 0; t < tasks.size(); ++t) {
        MTask& T = tasks[t];
        if (T.label[0] >= 0 && G.labeled) {
            const uint32_t l = (uint32_t)T.label[0];
            T.pos_b = l < G.label_begin.size() - 1 ? G.label_begin[l] : G.n;
            T.pos_e = l < G.label_begin.size() - 1 ? G.label_begin[l + 1] : G.n;
        } else {
            T.pos_b = 0;
            T.pos_e = G.n;
        }
        prefix[t + 1] = prefix[t] + (T.pos_e - T.pos_b + MNI_CHUNK - 1) / MNI_CHUNK;
    }
    char* b = (char*)dptr(base);
    HIPCHK(hipMemcpyAsync(b + L.tasks, tasks.data(), sizeof(MTask) * tasks.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(b + L.prefix, prefix.data(), 8 * prefix.size(), hipMemcpyHostToDevice, s));
    HIPCHK(hipMemcpyAsync(b + L.outs, P.outs.data(), sizeof(MOut) * P.outs.size(), hipMemcpyHostToDevice, s));
    if (!P.list.empty())
        HIPCHK(hipMemcpyAsync(b + L.list, P.list.data(), 4 * P.list.size(), hipMemcpyHostToDevice, s));
    if (launch_zero((uint32_t*)(b + L.counts), (L.total - L.counts) / 4, s))
        return fail(PM_E_DEVICE, "zero-fill launch failed");
    MArgs a{};
    a.g.rp = (const uint32_t*)dptr(G.off_rp);
    a.g.col = (const uint32_t*)dptr(G.off_col);
    a.g.split = (const uint32_t*)dptr(G.off_split);
    a.g.lab = G.labeled ? (const uint8_t*)dptr(G.off_lab) : nullptr;
    a.g.n = G.n;
    a.order = G.labeled ? (const uint32_t*)dptr(G.off_lorder) : nullptr;
    a.tasks = (const MTask*)(b + L.tasks);
    a.prefix = (const uint64_t*)(b + L.prefix);
    a.ntasks = (uint32_t)tasks.size();
    a.dom = (uint32_t*)(b + L.dom);
    a.words = L.words;
    a.head = (uint32_t*)(b + L.head);
    a.cancel = cancel;
    if (prefix.back() && launch_mni(a, num_cus * 8, s)) return fail(PM_E_DEVICE, "MNI search launch failed");
    if (launch_mni_union(a.dom, L.words, (const uint32_t*)(b + L.list), (const MOut*)(b + L.outs),
                         (uint32_t)P.outs.size(), (unsigned long long*)(b + L.counts),
                         (int)std::min<size_t>(P.outs.size(), (size_t)num_cus * 8), s))
        return fail(PM_E_DEVICE, "MNI union launch failed");
    HIPCHK(hipMemcpyAsync(host, b + L.counts, 8 * P.outs.size(), hipMemcpyDeviceToHost, s));
    return PM_OK;
}

// Run a plan to completion on the context's stream; sup[i] = support of
// query pattern i.
int Ctx_::run_mni_sync(GraphRes& G, const MniPlan& P, std::vector<int64_t>* sup) {
    int rc = ensure_label_order(G);
    if (rc) return rc;
    const uint64_t bytes = mni_layout(G, P).total;
    const uint64_t off = arena.alloc(bytes);
    if (off == UINT64_MAX) return fail(PM_E_NOMEM, "arena too small for the MNI domains");
    std::vector<unsigned long long> host(P.outs.size(), 0);
    unsigned long long* pinned = nullptr;
    if (hipHostMalloc((void**)&pinned, 8 * std::max<size_t>(1, P.outs.size()), 0) != hipSuccess) {
        arena.release(off);
        return fail(PM_E_DEVICE, "pinned allocation failed");
    }
    rc = enqueue_mni(G, P, off, pinned, nullptr, stream);
    if (rc == PM_OK) {
        hipError_t e = hipStreamSynchronize(stream);
        if (e != hipSuccess) rc = fail(PM_E_DEVICE, std::string("MNI kernels failed: ") + hipGetErrorString(e));
    }
    if (rc == PM_OK) memcpy(host.data(), pinned, 8 * P.outs.size());
    hipHostFree(pinned);
    arena.release(off);
    if (rc) return rc;
    sup->assign(P.qouts.size(), 0);
    for (size_t i = 0; i < P.qouts.size(); ++i) {
        int64_t m = INT64_MAX;
        for (uint32_t o : P.qouts[i]) m = std::min<int64_t>(m, (int64_t)host[o]);
        (*sup)[i] = P.qouts[i].empty() ? 0 : m;
    }
    return PM_OK;
}

int Ctx_::submit_mni(GraphRes& G, uint32_t gid, const std::vector<Pat>& ps, int morph, uint64_t* ticket) {
    auto t0 = std::chrono::steady_clock::now();
    auto Q = std::make_unique<Query>();
    Q->gid = gid;
    Q->npat = (uint32_t)ps.size();
    Q->mni = true;
    std::string err;
    int rc = mni_plan(ps, morph == PM_MORPH_NAIVE ? PM_MORPH_NAIVE : PM_MORPH_NONE, &Q->mni_plan, &err);
    if (rc) return fail(rc, err);
    rc = ensure_label_order(G);
    if (rc) return rc;
    HIPCHK(hipSetDevice(device));
    const uint64_t bytes = mni_layout(G, Q->mni_plan).total;
    Q->mni_off = arena.alloc(bytes);
    if (Q->mni_off == UINT64_MAX) return fail(PM_E_NOMEM, "arena too small for the MNI domains");
    auto release = [&]() {
        if (Q->mni_host) hipHostFree(Q->mni_host);
        if (Q->mni_cancel) hipHostFree(Q->mni_cancel);
        if (Q->mni_off != UINT64_MAX) arena.release(Q->mni_off);
        if (Q->ev_done) hipEventDestroy(Q->ev_done);
        if (Q->ev_start) hipEventDestroy(Q->ev_start);
        if (Q->ev_stop) hipEventDestroy(Q->ev_stop);
    };
    if (hipHostMalloc((void**)&Q->mni_host, 8 * std::max<size_t>(1, Q->mni_plan.outs.size()), 0) != hipSuccess ||
        hipHostMalloc((void**)&Q->mni_cancel, sizeof(int), hipHostMallocCoherent) != hipSuccess ||
        hipEventCreate(&Q->ev_start) != hipSuccess || hipEventCreate(&Q->ev_stop) != hipSuccess ||
        hipEventCreate(&Q->ev_done) != hipSuccess) {
        release();
        return fail(PM_E_DEVICE, "MNI query setup failed");
    }
    *(volatile int*)Q->mni_cancel = 0;
    Q->stats.plan_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    Q->stats.num_alt = (uint32_t)Q->mni_plan.alt.size();
    Q->stats.launches = 2;
    Q->stats.work_items = Q->mni_plan.tasks.size();
    Q->t_submit = t0;
    hipEventRecord(Q->ev_start, stream);
    rc = enqueue_mni(G, Q->mni_plan, Q->mni_off, Q->mni_host, Q->mni_cancel, stream);
    if (rc) {
        hipStreamSynchronize(stream);
        release();
        return rc;
    }
    hipEventRecord(Q->ev_stop, stream);
    hipEventRecord(Q->ev_done, stream);
    std::lock_guard<std::mutex> g(mu);
    const uint64_t tk = next_ticket++;
    G.inflight++;
    queries[tk] = std::move(Q);
    *ticket = tk;
    return PM_OK;
}

// Completion of an MNI query (called by wait() once its event has fired).
int Ctx_::finish_mni(Query& Q, int64_t* out) {
    float kms = 0;
    hipEventElapsedTime(&kms, Q.ev_start, Q.ev_stop);
    Q.stats.kernel_ms = kms;
    int rc = PM_OK;
    if (Q.cancelled) rc = fail(PM_E_CANCELLED, "query cancelled");
    if (rc == PM_OK && out)
        for (size_t i = 0; i < Q.mni_plan.qouts.size(); ++i) {
            int64_t m = INT64_MAX;
            for (uint32_t o : Q.mni_plan.qouts[i]) m = std::min<int64_t>(m, (int64_t)Q.mni_host[o]);
            out[i] = m;
        }
    Q.stats.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - Q.t_submit).count();
    last_stats = Q.stats;
    hipHostFree(Q.mni_host);
    hipHostFree(Q.mni_cancel);
    Q.mni_host = nullptr;
    Q.mni_cancel = nullptr;
    arena.release(Q.mni_off);
    Q.mni_off = UINT64_MAX;
    return rc;
}

}  // namespace pm

namespace pm {

namespace {

// Pattern key for sets and maps (canonical patterns only).
using PKey = std::tuple<int, uint32_t, bool, std::array<int8_t, 8>>;
PKey pkey(const Pat& p) { return PKey{p.k, p.em, p.vi, p.lab}; }

// The connected subpatterns with one edge fewer (Preliminaries, FSM:
// anti-monotonicity of MNI support): drop one edge; when that leaves a
// vertex without edges, drop the vertex too.  Drops that split the pattern
// into two parts with edges give no connected subpattern.
std::vector<Pat> edge_deletions(const Pat& q) {
    std::vector<Pat> out;
    for (int j = 1; j < q.k; ++j)
        for (int i = 0; i < j; ++i) {
            if (!has_edge(q.em, i, j)) continue;
            Pat r = q;
            r.em &= ~(1u << pair_bit(i, j));
            if (is_connected(r.k, r.em)) {
                out.push_back(canonical(r));
                continue;
            }
            int iso = -1;
            for (int w : {i, j}) {
                bool any = false;
                for (int x = 0; x < r.k; ++x)
                    if (x != w && has_edge(r.em, w, x)) any = true;
                if (!any) iso = w;
            }
            if (iso < 0 || r.k <= 2) continue;
            Pat s;
            s.k = r.k - 1;
            s.vi = false;
            int idx[8];
            for (int x = 0, y = 0; x < r.k; ++x) idx[x] = x == iso ? -1 : y++;
            for (int x = 0; x < r.k; ++x)
                if (idx[x] >= 0) s.lab[idx[x]] = r.lab[x];
            for (int b = 1; b < r.k; ++b)
                for (int a = 0; a < b; ++a)
                    if (idx[a] >= 0 && idx[b] >= 0 && has_edge(r.em, a, b))
                        s.em |= 1u << pair_bit(idx[a], idx[b]);
            if (is_connected(s.k, s.em)) out.push_back(canonical(s));
        }
    return out;
}

}  // namespace

// Level-wise frequent subgraph mining (Preliminaries, FSM): level e holds
// the labeled edge-induced connected patterns with e edges (at most KMAX
// vertices).  Level 1 is every labeled edge; level e + 1 extends each
// frequent pattern of level e by one edge, between two of its vertices or
// to a new labeled vertex, and keeps a candidate only when every connected
// subpattern with one edge fewer is frequent (MNI support is
// anti-monotone), before its support is computed.
int Ctx_::fsm_levelwise(GraphRes& G, uint32_t L, uint32_t max_edges, int64_t threshold, int morph,
                        std::vector<std::pair<Pat, int64_t>>* out) {
    out->clear();
    const uint64_t per_task = 4ull * ((G.n + 31) / 32);
    auto supports = [&](const std::vector<Pat>& cand, std::vector<int64_t>* sup) -> int {
        sup->assign(cand.size(), 0);
        const uint64_t budget = std::max<uint64_t>(arena.largest_free() / 4, 64ull << 20);
        const uint64_t batch = std::max<uint64_t>(1, budget / (64 * per_task + 4096));
        for (size_t b0 = 0; b0 < cand.size(); b0 += batch) {
            const size_t b1 = std::min<size_t>(cand.size(), b0 + batch);
            std::vector<Pat> part(cand.begin() + b0, cand.begin() + b1);
            MniPlan P;
            std::string err;
            int rc = mni_plan(part, morph, &P, &err);
            if (rc) return fail(rc, err);
            std::vector<int64_t> s;
            rc = run_mni_sync(G, P, &s);
            if (rc) return rc;
            std::copy(s.begin(), s.end(), sup->begin() + b0);
        }
        return PM_OK;
    };
    std::vector<Pat> level;
    for (uint32_t a = 0; a < L; ++a)
        for (uint32_t b = a; b < L; ++b) {
            Pat p;
            p.k = 2;
            p.em = 1;
            p.vi = false;
            p.lab[0] = (int8_t)a;
            p.lab[1] = (int8_t)b;
            level.push_back(canonical(p));
        }
    for (uint32_t e = 1; e <= max_edges && !level.empty(); ++e) {
        std::vector<int64_t> sup;
        int rc = supports(level, &sup);
        if (rc) return rc;
        std::set<PKey> frequent;
        std::vector<Pat> keep;
        for (size_t i = 0; i < level.size(); ++i)
            if (sup[i] >= threshold) {
                out->push_back({level[i], sup[i]});
                frequent.insert(pkey(level[i]));
                keep.push_back(level[i]);
            }
        if (e == max_edges) break;
        std::set<PKey> seen;
        std::vector<Pat> next;
        auto offer = [&](const Pat& q) {
            const Pat c = canonical(q);
            if (!seen.insert(pkey(c)).second) return;
            for (const Pat& r : edge_deletions(c))
                if (!frequent.count(pkey(r))) return;
            next.push_back(c);
        };
        for (const Pat& p : keep) {
            for (int j = 1; j < p.k; ++j)
                for (int i = 0; i < j; ++i)
                    if (!has_edge(p.em, i, j)) {
                        Pat q = p;
                        q.em |= 1u << pair_bit(i, j);
                        offer(q);
                    }
            if (p.k < KMAX)
                for (int i = 0; i < p.k; ++i)
                    for (uint32_t l = 0; l < L; ++l) {
                        Pat q = p;
                        q.k = p.k + 1;
                        q.lab[p.k] = (int8_t)l;
                        q.em |= 1u << pair_bit(i, p.k);
                        offer(q);
                    }
        }
        level.swap(next);
    }
    return PM_OK;
}

}  // namespace pm

using namespace pm;

extern "C" pm_status pm_fsm_levelwise(pm_ctx* ctx, uint32_t graph_id, uint32_t num_labels, uint32_t max_edges,
                                      int64_t threshold, int32_t morph, pm_pattern* out_pats,
                                      int64_t* out_support, uint64_t capacity, uint64_t* out_count) {
    if (!ctx || !out_count) return fail(PM_E_INVAL, "null argument");
    if (num_labels == 0 || num_labels > 255) return fail(PM_E_INVAL, "num_labels must be 1..255");
    if (max_edges == 0 || max_edges > (uint32_t)(KMAX * (KMAX - 1) / 2))
        return fail(PM_E_INVAL, "max_edges must be 1..10");
    if (morph != PM_MORPH_NONE && morph != PM_MORPH_NAIVE && morph != PM_MORPH_COST)
        return fail(PM_E_INVAL, "unknown morph mode");
    Ctx_& c = ctx->c;
    GraphRes* G;
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.graphs.find(graph_id);
        if (it == c.graphs.end()) return fail(PM_E_NOTFOUND, "unknown graph id");
        G = it->second.get();
    }
    if (!G->labeled) return fail(PM_E_INVAL, "level-wise FSM needs a labeled graph");
    if (G->max_label >= num_labels) return fail(PM_E_INVAL, "graph label outside 0..num_labels-1");
    if (hipSetDevice(c.device) != hipSuccess) return fail(PM_E_DEVICE, "hipSetDevice failed");
    std::vector<std::pair<Pat, int64_t>> res;
    int rc = c.fsm_levelwise(*G, num_labels, max_edges, threshold,
                             morph == PM_MORPH_NAIVE ? PM_MORPH_NAIVE : PM_MORPH_NONE, &res);
    if (rc) return rc;
    *out_count = res.size();
    if (capacity < res.size() || (!res.empty() && (!out_pats || !out_support)))
        return fail(PM_E_INVAL, "output capacity " + std::to_string(capacity) + " below the " +
                                    std::to_string(res.size()) + " frequent patterns");
    for (size_t i = 0; i < res.size(); ++i) {
        const Pat& p = res[i].first;
        pm_pattern& o = out_pats[i];
        o.k = (uint32_t)p.k;
        o.edge_mask = p.em;
        o.induce = PM_EDGE_INDUCED;
        for (int v = 0; v < 8; ++v) o.label[v] = v < p.k ? p.lab[v] : -1;
        out_support[i] = res[i].second;
    }
    return PM_OK;
}

namespace pm {

// Listing through morphing (Section 3.2.2, match conversion): the matches
// of an edge-induced pattern p are the vertex-induced matches of the
// patterns p + S on p's own vertices (S: the non-adjacent pairs whose
// images are adjacent), each converted by the identity map of p's vertices,
// so listing every p + S vertex-induced lists p edge-induced, each subgraph
// once.  One subgraph = one match up to p's automorphisms: the kernel keeps
// the lexicographically smallest.  Synchronous on the context's stream.
int Ctx_::list_matches(GraphRes& G, const Pat& p, int morph, uint32_t* out, uint64_t cap, uint64_t* count) {
    if (p.k < 2 || p.k > KMAX || !is_connected(p.k, p.em) || (p.em & ~full_mask(p.k)))
        return fail(PM_E_UNSUPPORTED, "listed patterns must be connected with 2..5 vertices");
    std::vector<Pat> route;
    if (morph == PM_MORPH_NAIVE && !p.vi && p.em != full_mask(p.k)) {
        std::vector<int> nonedge;
        for (int b = 0; b < p.k * (p.k - 1) / 2; ++b)
            if (!((p.em >> b) & 1)) nonedge.push_back(b);
        for (uint32_t S = 0; S < (1u << nonedge.size()); ++S) {
            Pat q = p;
            q.vi = true;
            for (size_t t = 0; t < nonedge.size(); ++t)
                if ((S >> t) & 1) q.em |= 1u << nonedge[t];
            route.push_back(q);
        }
    } else {
        route.push_back(p);
    }
    int rc = ensure_label_order(G);
    if (rc) return rc;
    // searches start at the pattern vertex of most edges
    int u = 0;
    for (int v = 1; v < p.k; ++v) {
        int dv = 0, du = 0;
        for (int w = 0; w < p.k; ++w) {
            dv += w != v && has_edge(p.em, v, w);
            du += w != u && has_edge(p.em, u, w);
        }
        if (dv > du) u = v;
    }
    std::vector<MTask> tasks;
    std::vector<uint8_t> steps(route.size() * KMAX);
    std::vector<uint64_t> prefix(route.size() + 1, 0);
    for (size_t t = 0; t < route.size(); ++t) {
        MTask T = search_task(route[t], u, &steps[t * KMAX]);
        if (T.label[0] >= 0 && G.labeled) {
            const uint32_t l = (uint32_t)T.label[0];
            T.pos_b = G.label_begin[l];
            T.pos_e = G.label_begin[l + 1];
        } else {
            T.pos_b = 0;
            T.pos_e = G.n;
        }
        prefix[t + 1] = prefix[t] + (T.pos_e - T.pos_b + MNI_CHUNK - 1) / MNI_CHUNK;
        tasks.push_back(T);
    }
    std::vector<uint8_t> aut;
    for (const Perm& g : automorphisms(p))
        for (int v = 0; v < KMAX; ++v) aut.push_back(v < p.k ? g[v] : 0);
    const uint32_t naut = (uint32_t)(aut.size() / KMAX);
    // device layout: tasks | steps | prefix | aut | count + head | out
    const uint64_t k = (uint64_t)p.k;
    uint64_t o = 0;
    const uint64_t o_tasks = o;
    o = r256(o + sizeof(MTask) * tasks.size());
    const uint64_t o_steps = o;
    o = r256(o + steps.size());
    const uint64_t o_prefix = o;
    o = r256(o + 8 * prefix.size());
    const uint64_t o_aut = o;
    o = r256(o + aut.size());
    const uint64_t o_cnt = o;
    o = r256(o + 16);
    const uint64_t o_out = o;
    const uint64_t room = arena.largest_free() / 2;
    const uint64_t dcap = std::min<uint64_t>(cap, room > o ? (room - o) / (4 * k) : 0);
    o = r256(o + 4 * k * std::max<uint64_t>(dcap, 1));
    const uint64_t off = arena.alloc(o);
    if (off == UINT64_MAX) return fail(PM_E_NOMEM, "arena too small for the listing");
    char* b = (char*)dptr(off);
    HIPCHK(hipSetDevice(device));
    unsigned long long hc = 0;
    auto run = [&]() -> int {
        HIPCHK(hipMemcpyAsync(b + o_tasks, tasks.data(), sizeof(MTask) * tasks.size(), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(b + o_steps, steps.data(), steps.size(), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(b + o_prefix, prefix.data(), 8 * prefix.size(), hipMemcpyHostToDevice, stream));
        HIPCHK(hipMemcpyAsync(b + o_aut, aut.data(), aut.size(), hipMemcpyHostToDevice, stream));
        if (launch_zero((uint32_t*)(b + o_cnt), 4, stream)) return fail(PM_E_DEVICE, "zero-fill launch failed");
        LArgs a{};
        a.g.rp = (const uint32_t*)dptr(G.off_rp);
        a.g.col = (const uint32_t*)dptr(G.off_col);
        a.g.split = (const uint32_t*)dptr(G.off_split);
        a.g.lab = G.labeled ? (const uint8_t*)dptr(G.off_lab) : nullptr;
        a.g.n = G.n;
        a.order = G.labeled ? (const uint32_t*)dptr(G.off_lorder) : nullptr;
        a.tasks = (const MTask*)(b + o_tasks);
        a.steps = (const uint8_t*)(b + o_steps);
        a.prefix = (const uint64_t*)(b + o_prefix);
        a.ntasks = (uint32_t)tasks.size();
        a.aut = (const uint8_t*)(b + o_aut);
        a.naut = naut;
        a.k = (uint32_t)k;
        a.out = (uint32_t*)(b + o_out);
        a.cap = dcap;
        a.count = (unsigned long long*)(b + o_cnt);
        a.head = (uint32_t*)(b + o_cnt + 8);
        if (prefix.back() && launch_list(a, num_cus * 8, stream)) return fail(PM_E_DEVICE, "listing launch failed");
        HIPCHK(hipMemcpyAsync(&hc, b + o_cnt, 8, hipMemcpyDeviceToHost, stream));
        HIPCHK(hipStreamSynchronize(stream));
        const uint64_t got = std::min<uint64_t>(hc, dcap);
        if (got && out) {
            HIPCHK(hipMemcpy(out, b + o_out, 4 * k * got, hipMemcpyDeviceToHost));
            for (uint64_t i = 0; i < got * k; ++i) out[i] = G.orig_id[out[i]];
        }
        return PM_OK;
    };
    rc = run();
    arena.release(off);
    if (rc) return rc;
    *count = hc;
    if (std::min<uint64_t>(hc, cap) > dcap)
        return fail(PM_E_NOMEM, "the arena holds only " + std::to_string(dcap) + " of the " +
                                    std::to_string(std::min<uint64_t>(hc, cap)) + " tuples asked for");
    return PM_OK;
}

}  // namespace pm

extern "C" pm_status pm_list(pm_ctx* ctx, uint32_t graph_id, const pm_pattern* pat, int32_t morph,
                             uint32_t* out_matches, uint64_t capacity, uint64_t* out_count) {
    if (!ctx || !pat || !out_count || (capacity && !out_matches)) return fail(PM_E_INVAL, "null argument");
    if (morph != PM_MORPH_NONE && morph != PM_MORPH_NAIVE && morph != PM_MORPH_COST)
        return fail(PM_E_INVAL, "unknown morph mode");
    Ctx_& c = ctx->c;
    GraphRes* G;
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.graphs.find(graph_id);
        if (it == c.graphs.end()) return fail(PM_E_NOTFOUND, "unknown graph id");
        G = it->second.get();
    }
    Pat p;
    std::string err;
    int rc = to_pat(*pat, &p, &err);
    if (rc) return fail(rc, err);
    for (int v = 0; v < p.k; ++v)
        if (p.lab[v] >= 0 && !G->labeled) return fail(PM_E_INVAL, "labeled pattern on an unlabeled graph");
    return c.list_matches(*G, p, morph == PM_MORPH_NAIVE ? PM_MORPH_NAIVE : PM_MORPH_NONE, out_matches, capacity,
                          out_count);
}
