// Host runtime and C-ABI of the pattern-morphing engine.
//
// Graph ingest (validation, degree-ordered relabelling, CSR build), the
// arena sub-allocator over the caller's device memory, query submission
// (morph plan, plan compile, device launch), completion and the integer
// conversion back to the requested patterns (Corollary 3.1 / Theorem 3.1 in
// counting form, checked int64).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "fsm.hpp"
#include "runtime.hpp"

namespace pm {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
    g_err = msg;
    return code;
}


// ---------------------------------------------------------------- arena

uint64_t Arena::alloc(uint64_t bytes) {
    std::lock_guard<std::mutex> g(mu);
    bytes = (bytes + 255) & ~uint64_t(255);
    if (bytes == 0) bytes = 256;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
        if (it->second >= bytes) {
            uint64_t off = it->first, sz = it->second;
            free_.erase(it);
            if (sz > bytes) free_[off + bytes] = sz - bytes;
            used_[off] = bytes;
            return off;
        }
    }
    return UINT64_MAX;
}

void Arena::release(uint64_t off) {
    std::lock_guard<std::mutex> g(mu);
    auto it = used_.find(off);
    if (it == used_.end()) return;
    uint64_t sz = it->second;
    used_.erase(it);
    auto nx = free_.lower_bound(off);
    if (nx != free_.end() && off + sz == nx->first) {
        sz += nx->second;
        free_.erase(nx);
    }
    auto pv = free_.lower_bound(off);
    if (pv != free_.begin()) {
        --pv;
        if (pv->first + pv->second == off) {
            pv->second += sz;
            return;
        }
    }
    free_[off] = sz;
}

uint64_t Arena::largest_free() {
    std::lock_guard<std::mutex> g(mu);
    uint64_t b = 0;
    for (auto& f : free_) b = std::max(b, f.second);
    return b;
}

// ---------------------------------------------------------------- graph

static void parallel_for(uint64_t n, const std::function<void(uint64_t, uint64_t)>& fn) {
    unsigned nt = std::max(1u, std::min(32u, std::thread::hardware_concurrency()));
    if (n < 65536) nt = 1;
    std::vector<std::thread> th;
    uint64_t chunk = (n + nt - 1) / nt;
    for (unsigned t = 0; t < nt; ++t) {
        uint64_t b = t * chunk, e = std::min(n, b + chunk);
        if (b >= e) break;
        th.emplace_back(fn, b, e);
    }
    for (auto& x : th) x.join();
}

std::vector<KItem> build_items(const std::vector<uint32_t>& rp, uint32_t n, uint64_t budget, uint32_t split,
                               uint32_t max_roots) {
    std::vector<KItem> items;
    // heaviest roots first (ids ascend with degree)
    int64_t r = (int64_t)n - 1;
    while (r >= 0) {
        uint32_t d = rp[r + 1] - rp[r];
        if (d > split) {
            for (uint32_t s = 0; s < d; s += split) items.push_back({(uint32_t)r, (uint32_t)r + 1, s, s + split});
            --r;
            continue;
        }
        int64_t end = r + 1;
        uint64_t sum = 0;
        uint32_t cnt = 0;
        while (r >= 0) {
            uint32_t dr = rp[r + 1] - rp[r];
            if (dr > split) break;
            if (cnt > 0 && (sum + dr > budget || cnt >= max_roots)) break;
            sum += dr;
            ++cnt;
            --r;
        }
        items.push_back({(uint32_t)(r + 1), (uint32_t)end, 0, 0xffffffffu});
    }
    return items;
}


// Work items of the triangle-core kernel.  A root's stream volume is the
// summed out-degree of its out-neighbours.  Consecutive roots with 2 ..
// CQ_SMAX out-neighbours are grouped until their volume reaches CQ_VOL (at
// most 256 roots an item); a root above CQ_VOL is cut into row slices of
// about CQ_VOL each (items {r, r+1, i0, i1}).  Roots with more than CQ_SMAX
// out-neighbours are listed apart for the general kernel.
static constexpr uint64_t CQ_VOL = 16384;
static void clique_items(GraphRes& G, const std::vector<uint32_t>& rp, const std::vector<uint32_t>& col,
                         const std::vector<uint32_t>& split) {
    G.clique_items.clear();
    G.clique_big.clear();
    uint32_t gb = 0;
    uint64_t gv = 0;
    bool open = false;
    auto close = [&](uint32_t end) {
        if (open) G.clique_items.push_back({gb, end, 0, UINT32_MAX});
        open = false;
        gv = 0;
    };
    for (uint32_t r = 0; r < G.n; ++r) {
        const uint32_t s = rp[r + 1] - split[r];
        if (s > CQ_SMAX) {
            close(r);
            G.clique_big.push_back(r);
            continue;
        }
        if (s < 2) continue;
        uint64_t vol = 0;
        for (uint32_t p = split[r]; p < rp[r + 1]; ++p) vol += rp[col[p] + 1] - split[col[p]];
        if (vol > CQ_VOL) {
            close(r);
            uint64_t acc = 0;
            uint32_t i0 = 0;
            for (uint32_t i = 0; i < s; ++i) {
                const uint32_t x = col[split[r] + i];
                acc += rp[x + 1] - split[x];
                if (acc >= CQ_VOL || i + 1 == s) {
                    G.clique_items.push_back({r, r + 1, i0, i + 1});
                    i0 = i + 1;
                    acc = 0;
                }
            }
            continue;
        }
        if (!open) {
            open = true;
            gb = r;
        }
        gv += vol;
        if (gv >= CQ_VOL || r + 1 - gb >= 256) close(r + 1);
    }
    close(G.n);
    // 4-clique kernel: light roots (3 .. C4_LIGHT_MAX out-neighbours) grouped
    // up to CQ_VOL of volume, heavier ones one an item, most volume first (to
    // C4_HEAVY_MAX, and to C4_ROOT_MAX in a launch of their own)
    G.c4_light.clear();
    G.c4_heavy.clear();
    G.c4_huge.clear();
    G.c4_big.clear();
    std::vector<std::pair<uint64_t, uint32_t>> hv, xv;
    open = false;
    gv = 0;
    auto close4 = [&](uint32_t end) {
        if (open) G.c4_light.push_back({gb, end, 0, 0});
        open = false;
        gv = 0;
    };
    for (uint32_t r = 0; r < G.n; ++r) {
        const uint32_t s = rp[r + 1] - split[r];
        // roots of two out-neighbours close no 4-clique, but the support
        // filling variant meets their one triangle
        if (s < 2) continue;
        uint64_t vol = 0;
        for (uint32_t p = split[r]; p < rp[r + 1]; ++p) vol += rp[col[p] + 1] - split[col[p]];
        if (s > C4_LIGHT_MAX) {
            close4(r);
            if (s > C4_ROOT_MAX) G.c4_big.push_back(r);
            else if (s > C4_HEAVY_MAX) xv.push_back({vol, r});
            else hv.push_back({vol, r});
            continue;
        }
        if (!open) {
            open = true;
            gb = r;
        }
        gv += vol;
        if (gv >= CQ_VOL || r + 1 - gb >= 256) close4(r + 1);
    }
    close4(G.n);
    auto by_volume = [](const auto& x, const auto& y) { return x.first > y.first; };
    std::stable_sort(hv.begin(), hv.end(), by_volume);
    std::stable_sort(xv.begin(), xv.end(), by_volume);
    for (const auto& h : hv) G.c4_heavy.push_back({h.second, h.second + 1, 0, 0});
    for (const auto& h : xv) G.c4_huge.push_back({h.second, h.second + 1, 0, 0});
}

int Ctx_::graph_load(uint32_t n, const uint32_t* rp, const uint32_t* col, const uint8_t* labels,
                     uint32_t* out_gid) {
    if (!rp || !col || !out_gid) return fail(PM_E_INVAL, "null graph array");
    if (n == 0) return fail(PM_E_INVAL, "empty graph");
    if (rp[0] != 0) return fail(PM_E_INVAL, "row_ptr[0] must be 0");
    for (uint32_t v = 0; v < n; ++v)
        if (rp[v + 1] < rp[v]) return fail(PM_E_INVAL, "row_ptr not monotone");
    uint64_t nnz = rp[n];
    if (nnz % 2) return fail(PM_E_INVAL, "odd number of adjacency entries: not symmetric");
    std::atomic<int> bad{0};
    std::atomic<uint64_t> bad_v{0};
    parallel_for(n, [&](uint64_t b, uint64_t e) {
        for (uint64_t v = b; v < e && !bad; ++v) {
            for (uint32_t p = rp[v]; p < rp[v + 1]; ++p) {
                uint32_t w = col[p];
                if (w >= n) { bad = 1; bad_v = v; break; }
                if (w == v) { bad = 2; bad_v = v; break; }
                if (p > rp[v] && col[p - 1] >= w) { bad = 3; bad_v = v; break; }
                // symmetric: v in N(w)
                const uint32_t* a = col + rp[w];
                uint32_t len = rp[w + 1] - rp[w];
                const uint32_t* f = std::lower_bound(a, a + len, (uint32_t)v);
                if (f == a + len || *f != v) { bad = 4; bad_v = v; break; }
            }
        }
    });
    static const char* why[] = {"", "neighbour id out of range", "self-loop",
                                "adjacency not strictly ascending (unsorted or duplicate)",
                                "adjacency not symmetric"};
    if (bad) return fail(PM_E_INVAL, std::string(why[bad.load()]) + " at vertex " + std::to_string(bad_v.load()));

    // degree-ordered relabelling: rank by (degree, id)
    std::vector<uint32_t> order(n);
    for (uint32_t v = 0; v < n; ++v) order[v] = v;
    std::stable_sort(order.begin(), order.end(), [&](uint32_t a, uint32_t b) {
        return (rp[a + 1] - rp[a]) < (rp[b + 1] - rp[b]);
    });
    std::vector<uint32_t> newid(n);
    for (uint32_t r = 0; r < n; ++r) newid[order[r]] = r;
    std::vector<uint32_t> nrp(n + 1, 0);
    for (uint32_t r = 0; r < n; ++r) nrp[r + 1] = nrp[r] + (rp[order[r] + 1] - rp[order[r]]);
    std::vector<uint32_t> ncol(nnz ? nnz : 1);
    parallel_for(n, [&](uint64_t b, uint64_t e) {
        for (uint64_t r = b; r < e; ++r) {
            uint32_t u = order[r];
            uint32_t o = nrp[r];
            for (uint32_t p = rp[u]; p < rp[u + 1]; ++p) ncol[o++] = newid[col[p]];
            std::sort(ncol.begin() + nrp[r], ncol.begin() + nrp[r + 1]);
        }
    });
    std::vector<uint8_t> nlab;
    uint32_t max_label = 0;
    if (labels) {
        nlab.resize(n);
        for (uint32_t r = 0; r < n; ++r) {
            nlab[r] = labels[order[r]];
            max_label = std::max<uint32_t>(max_label, nlab[r]);
        }
    }
    auto G = std::make_unique<GraphRes>();
    G->orig_id = order;
    G->n = n;
    G->m = nnz / 2;
    G->labeled = labels != nullptr;
    G->max_label = max_label;
    double sd2 = 0, so2 = 0, s_pq = 0, s_pd = 0, s_qq = 0, s_qd = 0;
    uint32_t maxd = 0, maxo = 0;
    for (uint32_t r = 0; r < n; ++r) {
        uint32_t d = nrp[r + 1] - nrp[r];
        const uint32_t* a = ncol.data() + nrp[r];
        uint32_t out = (uint32_t)((a + d) - std::upper_bound(a, a + d, r));
        maxd = std::max(maxd, d);
        maxo = std::max(maxo, out);
        double q = (double)(d - out);
        sd2 += (double)d * d;
        so2 += (double)out * out;
        s_pq += (double)out * q;
        s_pd += (double)out * d;
        s_qq += q * q;
        s_qd += q * d;
    }
    std::vector<uint32_t> nsplit(n);
    for (uint32_t r = 0; r < n; ++r) {
        const uint32_t* a = ncol.data() + nrp[r];
        uint32_t d = nrp[r + 1] - nrp[r];
        nsplit[r] = nrp[r] + (uint32_t)(std::upper_bound(a, a + d, r) - a);
    }
    G->max_deg = maxd;
    G->max_out = maxo;
    GraphStats& s = G->st;
    s.n = n;
    s.m = (double)G->m;
    s.avg_deg = n ? 2.0 * G->m / n : 0;
    s.nbr_deg = G->m ? sd2 / (2.0 * G->m) : 0;
    s.avg_out = n ? (double)G->m / n : 0;
    s.nbr_out = G->m ? so2 / (double)G->m : 0;
    s.max_deg = maxd;
    s.max_out = maxo;
    s.s_pp = so2;
    s.s_pq = s_pq;
    s.s_pd = s_pd;
    s.s_qq = s_qq;
    s.s_qd = s_qd;
    s.s_dd = sd2;
    {
        uint64_t h = 1469598103934665603ull;
        auto mix = [&](const void* p, size_t len) {
            const unsigned char* c = (const unsigned char*)p;
            for (size_t i = 0; i < len; ++i) h = (h ^ c[i]) * 1099511628211ull;
        };
        mix(&n, sizeof(n));
        mix(nrp.data(), 4ull * (n + 1));
        mix(ncol.data(), 4ull * nnz);
        if (labels) mix(nlab.data(), n);
        G->hash = h;
    }

    uint64_t need_rp = 4ull * (n + 1), need_col = 4ull * std::max<uint64_t>(nnz, 1),
             need_lab = labels ? n : 0, need_items = 0;
    G->off_rp = arena.alloc(need_rp);
    G->off_col = arena.alloc(need_col);
    G->off_split = arena.alloc(4ull * n);
    G->off_lab = labels ? arena.alloc(need_lab) : UINT64_MAX - 1;
    G->off_items = UINT64_MAX - 1;
    if (G->off_rp == UINT64_MAX || G->off_col == UINT64_MAX || G->off_lab == UINT64_MAX ||
        G->off_items == UINT64_MAX || G->off_split == UINT64_MAX) {
        for (uint64_t o : {G->off_rp, G->off_col, G->off_split, G->off_lab, G->off_items})
            if (o < UINT64_MAX - 1) arena.release(o);
        return fail(PM_E_NOMEM, "arena too small for the graph");
    }
    G->device_bytes = need_rp + need_col + 4ull * n + need_lab + need_items;
    HIPCHK(hipSetDevice(device));
    HIPCHK(hipMemcpyAsync(dptr(G->off_rp), nrp.data(), need_rp, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(dptr(G->off_col), ncol.data(), 4ull * nnz, hipMemcpyHostToDevice, stream));
    HIPCHK(hipMemcpyAsync(dptr(G->off_split), nsplit.data(), 4ull * n, hipMemcpyHostToDevice, stream));
    if (labels) HIPCHK(hipMemcpyAsync(dptr(G->off_lab), nlab.data(), n, hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
    // two-hop mass: summed degrees of the lower neighbours (entries before split)
    G->two_hop.assign(n, 0);
    G->low2.assign(n, 0);
    parallel_for(n, [&](uint64_t b, uint64_t e) {
        for (uint64_t r = b; r < e; ++r) {
            uint64_t w = 0;
            for (uint32_t p = nrp[r]; p < nsplit[r]; ++p) w += nrp[ncol[p] + 1] - nrp[ncol[p]];
            G->two_hop[r] = w;
            G->low2[r] = nsplit[r] - nrp[r] >= 2 ? 1 : 0;
        }
    });
    clique_items(*G, nrp, ncol, nsplit);
    {
        // the triangle and 4-clique kernels' items stay on the device with
        // the graph (read-only, shared by every launch set)
        const size_t nc = G->clique_items.size(), nl = G->c4_light.size(), nh = G->c4_heavy.size(),
                     nx = G->c4_huge.size();
        if (nc + nl + nh + nx) {
            G->off_cq = arena.alloc(16 * (nc + nl + nh + nx));
            if (G->off_cq == UINT64_MAX) {
                for (uint64_t o : {G->off_rp, G->off_col, G->off_split, G->off_lab, G->off_items})
                    if (o < UINT64_MAX - 1) arena.release(o);
                return fail(PM_E_NOMEM, "arena too small for the graph");
            }
            KItem* d = (KItem*)dptr(G->off_cq);
            if (nc) HIPCHK(hipMemcpyAsync(d, G->clique_items.data(), 16 * nc, hipMemcpyHostToDevice, stream));
            if (nl) HIPCHK(hipMemcpyAsync(d + nc, G->c4_light.data(), 16 * nl, hipMemcpyHostToDevice, stream));
            if (nh) HIPCHK(hipMemcpyAsync(d + nc + nl, G->c4_heavy.data(), 16 * nh, hipMemcpyHostToDevice, stream));
            if (nx)
                HIPCHK(hipMemcpyAsync(d + nc + nl + nh, G->c4_huge.data(), 16 * nx, hipMemcpyHostToDevice, stream));
            HIPCHK(hipStreamSynchronize(stream));
            G->d_cq = d;
            G->d_c4l = d + nc;
            G->d_c4h = d + nc + nl;
            G->d_c4x = d + nc + nl + nh;
            G->device_bytes += 16 * (nc + nl + nh + nx);
        }
    }
    // membership bitmaps of the highest-degree vertices (ids ascend with
    // degree, so they are a suffix): a probe of such a list costs one load
    // instead of a binary search.  At least HUB_BM_DEG neighbours, at most
    // HUB_BM_BYTES in all; skipped when the arena cannot hold them.
    G->hub0 = n;
    G->hub_words = (n + 31) / 32;
    {
        uint32_t h = n;
        while (h > 0 && nrp[h] - nrp[h - 1] >= HUB_BM_DEG) --h;
        const uint64_t row = 4ull * G->hub_words, cap = HUB_BM_BYTES / std::max<uint64_t>(row, 1);
        if (n - h > cap) h = (uint32_t)(n - cap);
        if (h < n) {
            const uint64_t bytes = row * (n - h);
            G->off_hubbm = arena.alloc(bytes);
            if (G->off_hubbm != UINT64_MAX) {
                KGraph kg{};
                kg.rp = (const uint32_t*)dptr(G->off_rp);
                kg.col = (const uint32_t*)dptr(G->off_col);
                kg.n = n;
                HIPCHK(hipMemsetAsync(dptr(G->off_hubbm), 0, bytes, stream));
                if (launch_hub_bitmaps(kg, (uint32_t*)dptr(G->off_hubbm), h, G->hub_words, stream)) {
                    arena.release(G->off_hubbm);
                    G->off_hubbm = UINT64_MAX;
                } else {
                    HIPCHK(hipStreamSynchronize(stream));
                    G->hub0 = h;
                    G->device_bytes += bytes;
                }
            }
        }
    }
    G->host_rp = std::move(nrp);
    if (labels) {
        // vertices by label (stable: degree order within a label), for the
        // FSM kernel's label-uniform wavefronts
        std::vector<uint32_t> cnt(257, 0);
        for (uint32_t r = 0; r < n; ++r) cnt[nlab[r] + 1]++;
        for (int l = 0; l < 256; ++l) cnt[l + 1] += cnt[l];
        G->label_begin.assign(cnt.begin(), cnt.end());
        G->label_order.resize(n);
        for (uint32_t r = 0; r < n; ++r) G->label_order[cnt[nlab[r]]++] = r;
    }
    std::lock_guard<std::mutex> g(mu);
    uint32_t gid = next_gid++;
    graphs[gid] = std::move(G);
    *out_gid = gid;
    return PM_OK;
}

int Ctx_::graph_unload(uint32_t gid) {
    std::lock_guard<std::mutex> g(mu);
    auto it = graphs.find(gid);
    if (it == graphs.end()) return fail(PM_E_NOTFOUND, "unknown graph id");
    if (it->second->inflight) return fail(PM_E_BUSY, "queries in flight on this graph");
    GraphRes& G = *it->second;
    for (uint64_t o : {G.off_rp, G.off_col, G.off_split, G.off_lab, G.off_items, G.off_support, G.off_cq,
                       G.off_lorder, G.off_hubbm})
        if (o < UINT64_MAX - 1) arena.release(o);
    for (auto& is : G.itemsets) arena.release(is.second.off);
    for (auto& ls : G.launches) free_launchset(ls.second.get());
    graphs.erase(it);
    return PM_OK;
}

// ---------------------------------------------------------------- queries

int to_pat(const pm_pattern& q, Pat* out, std::string* err) {
    if (q.k < 2 || q.k > (uint32_t)KMAX) {
        *err = "pattern size must be 2..5";
        return PM_E_UNSUPPORTED;
    }
    if (q.edge_mask & ~full_mask((int)q.k)) {
        *err = "edge_mask has bits beyond the k vertices";
        return PM_E_INVAL;
    }
    if (!is_connected((int)q.k, q.edge_mask)) {
        *err = "pattern is not connected";
        return PM_E_UNSUPPORTED;
    }
    if (q.induce > 1) {
        *err = "induce must be PM_EDGE_INDUCED or PM_VERTEX_INDUCED";
        return PM_E_INVAL;
    }
    out->k = (int)q.k;
    out->em = q.edge_mask;
    out->vi = q.induce == PM_VERTEX_INDUCED;
    for (int i = 0; i < 8; ++i) {
        int32_t l = i < (int)q.k ? q.label[i] : -1;
        if (l < -1 || l > 255) {
            *err = "label outside -1..255";
            return PM_E_INVAL;
        }
        out->lab[i] = (int8_t)(l < 0 ? -1 : (l > 127 ? 127 : l));
        if (l > 127) {
            *err = "labels above 127 are not supported";
            return PM_E_UNSUPPORTED;
        }
    }
    return PM_OK;
}


// Closed forms over triangle counts need every triangle met by the
// triangle pass that fills the per-edge counts (no root beyond CQ_SMAX).
bool Ctx_::tri_forms(const GraphRes& G) const {
    return clique_opt && support_opt && !G.clique_items.empty() && G.clique_big.empty();
}

const PlanInfo& Ctx_::plan_for(GraphRes& G, const Pat& p, int* rc, bool tri_ok) {
    std::lock_guard<std::mutex> g(plan_mu);
    const bool tri = tri_ok && tri_forms(G);
    auto& cache = tri ? G.plan_cache : G.plan_cache_notri;
    for (auto& e : cache)
        if (e.first == p) {
            *rc = PM_OK;
            return e.second;
        }
    PlanInfo pi;
    std::string err;
    *rc = compile_plan(p, G.st, &pi, &err, tri);
    if (*rc) g_err = err;
    cache.push_back({p, pi});
    return cache.back().second;
}

std::function<double(const Pat&)> Ctx_::cost_fn(GraphRes& G, bool tri_ok) {
    return [this, &G, tri_ok](const Pat& p) {
        int rc;
        const PlanInfo& pi = plan_for(G, p, &rc, tri_ok);
        return rc ? 1e300 : pi.total_cost;
    };
}

int Ctx_::plan_closure(GraphRes& G, const std::vector<Pat>& alt, std::vector<Pat>* closure,
                       std::vector<PlanInfo>* plans, bool tri_ok) {
    std::vector<Pat> cl = alt;
    std::vector<PlanInfo> pl;
    for (size_t i = 0; i < cl.size(); ++i) {
        int rc;
        PlanInfo pi = plan_for(G, cl[i], &rc, tri_ok);
        if (rc) return rc;
        for (auto& sq : pi.subs)
            if (std::find(cl.begin(), cl.end(), sq.first) == cl.end()) cl.push_back(sq.first);
        pl.push_back(pi);
    }
    std::vector<size_t> idx(cl.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    // plain plans, triangle-core plans, 4-clique plans, edge-core plans, then
    // two-hop plans:
    // each group can run in launches of its own
    auto group = [&](size_t a) {
        const DPlan& d = pl[a].d;
        if (d.cyc5) return 5;
        if (d.tagg) return 3;
        return d.agg_last ? 4
                          : (clique_ok(d) ? 1 : (clique4_ok(d) ? 2 : (edge_window_ok(d) || edge_cheap_ok(d) ? 3 : 0)));
    };
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return group(a) < group(b); });
    closure->clear();
    plans->clear();
    for (size_t i : idx) {
        closure->push_back(cl[i]);
        plans->push_back(pl[i]);
    }
    return PM_OK;
}

// Heavy roots of the two-hop launches: when every aggregation plan
// aggregates at its first level, roots whose two-hop mass (the summed
// degrees of their lower neighbours) is at least heavy_min_mass and at
// least their id (the range a window sweep may cover) over
// 2^heavy_span_shift run in agg_window_kernel, heaviest first.
// *p_agg = aggregation plans.
std::vector<uint32_t> Ctx_::heavy_roots(const GraphRes& G, const std::vector<PlanInfo>& plans,
                                        uint32_t* p_agg) const {
    std::vector<uint32_t> out;
    uint32_t pa = 0;
    *p_agg = 0;
    for (const PlanInfo& p : plans) {
        if (!p.d.agg_last) continue;
        if (p.d.ncore != 2 || p.d.bridge_src != 0) return out;
        ++pa;
    }
    *p_agg = pa;
    if (!pa || !heavy_roots_opt) return out;
    for (uint32_t r = 0; r < G.n; ++r) {
        const uint64_t w = G.two_hop[r];
        if (w >= heavy_min_mass && (w << heavy_span_shift) >= r) out.push_back(r);
    }
    std::stable_sort(out.begin(), out.end(),
                     [&](uint32_t x, uint32_t y) { return G.two_hop[x] > G.two_hop[y]; });
    return out;
}

// Heavy roots of edge-core plans: roots whose lower neighbours have a summed
// degree of at least heavy_min_mass, heaviest first (none when no such plan
// is present).
std::vector<uint32_t> Ctx_::edge_heavy_roots(const GraphRes& G, const std::vector<PlanInfo>& plans) const {
    std::vector<uint32_t> out;
    bool any = false;
    for (const PlanInfo& p : plans) any = any || (!p.d.agg_last && edge_window_ok(p.d));
    if (!any || !heavy_roots_opt) return out;
    for (uint32_t r = 0; r < G.n; ++r)
        if (G.two_hop[r] >= heavy_min_mass) out.push_back(r);
    std::stable_sort(out.begin(), out.end(),
                     [&](uint32_t x, uint32_t y) { return G.two_hop[x] > G.two_hop[y]; });
    return out;
}

// Work items of the heavy roots.  Two-hop roots are split by target-id range
// into about one slice per 2^22 of two-hop mass (items {r, 0, slice, slices};
// their workgroups hold a whole CU each, so a few hundred run at once);
// edge-core roots by level-1 candidates, 512 per item (items {r, 0, k0, k1}).
static std::vector<KItem> heavy_items(const GraphRes& G, const std::vector<uint32_t>& roots, bool two_hop) {
    std::vector<KItem> out;
    for (uint32_t r : roots) {
        if (two_hop) {
            const uint32_t ns = (uint32_t)std::min<uint64_t>(256, std::max<uint64_t>(1, G.two_hop[r] >> 22));
            for (uint32_t i = 0; i < ns; ++i) out.push_back({r, 0, i, ns});
        } else {
            const uint32_t d = G.host_rp[r + 1] - G.host_rp[r];
            for (uint32_t k = 0; k < d; k += 512) out.push_back({r, 0, k, k + 512});
        }
    }
    return out;
}

// Work items over every root except the heavy ones (ranges split around them).
static std::vector<KItem> items_without(const std::vector<KItem>& all, const std::vector<uint8_t>& heavy) {
    std::vector<KItem> out;
    for (const KItem& it : all) {
        uint32_t b = it.r0;
        for (uint32_t r = it.r0; r <= it.r1; ++r) {
            if (r == it.r1 || heavy[r]) {
                if (r > b) out.push_back({b, r, it.s0, it.s1});
                b = r + 1;
            }
        }
    }
    return out;
}


// Whether clique_kernel runs this plan on this graph: a plan summed over
// the edges of every triangle needs all triangles, so no root beyond the
// kernel's limit.
static bool clique_runs(const GraphRes& G, const DPlan& d) {
    const int k = clique_kind(d);
    return k == 1 || (k == 2 && G.clique_big.empty());
}

// Whether a launch set runs any plan in clique_kernel.
bool Ctx_::use_clique(const GraphRes& G, const std::vector<PlanInfo>& plans) const {
    if (!clique_opt || G.clique_items.empty()) return false;
    for (const PlanInfo& p : plans)
        if (clique_runs(G, p.d)) return true;
    return false;
}

// Whether a launch set runs any plan in clique4_kernel.
bool Ctx_::use_clique4(const GraphRes& G, const std::vector<PlanInfo>& plans) const {
    if (!clique_opt || (G.c4_light.empty() && G.c4_heavy.empty() && G.c4_huge.empty())) return false;
    for (const PlanInfo& p : plans)
        if (clique4_ok(p.d) || p.d.tagg == TAGG_K4EAR) return true;
    return false;
}

// Whether a launch set runs its edge-support plans on triangle supports
// (every triangle has to be met by clique_kernel: no root beyond CQ_SMAX).
bool Ctx_::use_support(const GraphRes& G, const std::vector<PlanInfo>& plans) const {
    if (!clique_opt || !support_opt || G.clique_items.empty() || !G.clique_big.empty()) return false;
    for (const PlanInfo& p : plans)
        if (p.d.tagg || (!clique_ok(p.d) && support_ok(p.d))) return true;
    return false;
}

// The graph's support counters (one u32 per adjacency entry), allocated on
// first use; every replay clears them before its triangle pass.
int Ctx_::ensure_support(GraphRes& G) {
    if (G.off_support != UINT64_MAX) return PM_OK;
    const uint64_t words = std::max<uint64_t>(1, 2 * G.m);
    G.off_support = arena.alloc(4 * words);
    if (G.off_support == UINT64_MAX) return fail(PM_E_NOMEM, "arena too small for the edge supports");
    return PM_OK;
}

// General-kernel items over the roots clique4_kernel leaves out.
std::vector<KItem> Ctx_::clique4_big_items(const GraphRes& G, const LaunchCfg& cfg) const {
    if (G.c4_big.empty()) return {};
    std::vector<uint8_t> other(G.n, 1);
    for (uint32_t r : G.c4_big) other[r] = 0;
    return items_without(build_items(G.host_rp, G.n, cfg.item_budget, cfg.item_split, 256), other);
}

// Items of the general kernel over the roots clique_kernel leaves out.
std::vector<KItem> Ctx_::clique_big_items(const GraphRes& G, const LaunchCfg& cfg) const {
    if (G.clique_big.empty()) return {};
    std::vector<uint8_t> other(G.n, 1);
    for (uint32_t r : G.clique_big) other[r] = 0;
    return items_without(build_items(G.host_rp, G.n, cfg.item_budget, cfg.item_split, 256), other);
}

uint64_t Ctx_::footprint(const GraphRes& G, const std::vector<PlanInfo>& plans, const LaunchCfg& cfg,
                         uint64_t* scratch_stride, bool* any_agg, bool heavy_ok) const {
    uint64_t stride = 1;
    bool agg = false;
    for (const PlanInfo& p : plans) {
        for (int j = 1; j < p.d.ncore; ++j) {
            const DLevel& L = p.d.lev[j];
            bool out_list = (L.adj & L.gt) != 0;
            stride = std::max<uint64_t>(stride, (out_list ? G.max_out : G.max_deg) + 64);
        }
        if (p.d.agg_last || p.d.cyc5 || p.d.tagg == TAGG_HOUSE) agg = true;
        if (p.d.local) {
            // bitmap rows: max_out rows of ceil(max_out/64) 64-bit words
            uint64_t words = (uint64_t)G.max_out * ((G.max_out + 63) / 64);
            stride = std::max<uint64_t>(stride, (2 * words + KMAX - 1) / KMAX + 64);
        }
    }
    stride = (stride + 63) & ~uint64_t(63);
    *scratch_stride = stride;
    *any_agg = agg;
    uint64_t b = 0;
    // plans, counters, heads, byte tally, and 256-byte rounding of each carve
    b += sizeof(DPlan) * plans.size() + 16 * plans.size() + 512 + 256 * 4;
    b += waves(cfg) * (uint64_t)KMAX * stride * 4;
    b += waves(cfg) * bitmap_words(G, plans) * 4;
    // per-vertex triangle counts of the closed forms (cleared with the counters)
    bool vt = false;
    for (const PlanInfo& p : plans) vt = vt || tagg_vtri(p.d.tagg) || p.d.tagg == TAGG_HOUSE;
    if (vt) b += (8ull * G.n + 255) & ~uint64_t(255);
    uint32_t pa = 0;
    const size_t hk = heavy_ok ? heavy_roots(G, plans, &pa).size() : 0;
    const size_t ek = heavy_ok ? edge_heavy_roots(G, plans).size() : 0;
    const uint64_t wstride = ((uint64_t)G.max_deg + 63) & ~uint64_t(63);
    if (hk) {
        // light items (at most one per root plus the hub slices), heavy items
        uint64_t items = G.n + heavy_items(G, heavy_roots(G, plans, &pa), true).size();
        for (uint32_t r = 0; r < G.n; ++r) items += (G.host_rp[r + 1] - G.host_rp[r]) / agg_split;
        b += 16 * items + 2 * 256;
    }
    if (ek) {
        uint64_t items = G.n + heavy_items(G, edge_heavy_roots(G, plans), false).size();
        for (uint32_t r = 0; r < G.n; ++r) items += (G.host_rp[r + 1] - G.host_rp[r]) / cfg.item_split;
        b += 16 * items + 2 * 256;
    }
    // per block: cursor, end and counter words per bridge or candidate
    if (hk || ek) b += (uint64_t)grid_blocks(cfg) * (2 + EW_TERMS) * wstride * 4 + 256;
    // general-kernel items of the roots the triangle and 4-clique kernels
    // leave out (their own items live with the graph)
    if (use_clique(G, plans) || use_support(G, plans)) b += 16 * clique_big_items(G, cfg).size() + 256;
    if (use_clique4(G, plans)) b += 16 * clique4_big_items(G, cfg).size() + 256;
    return b;
}

// Words of one wave's root bitmap (0 when no plan uses it).
uint64_t Ctx_::bitmap_words(const GraphRes& G, const std::vector<PlanInfo>& plans) const {
    bool any = false;
    for (const PlanInfo& p : plans) any = any || p.d.bm0;
    if (!any) return 0;
    return ((G.n + 31) / 32 + 63) & ~uint64_t(63);
}

// Whether a launch set in flight (cached and busy, or a query's own) points
// to the context's two-hop arrays.
bool Ctx_::ctx_agg_busy() {
    std::lock_guard<std::mutex> g(mu);
    for (auto& gr : graphs)
        for (auto& l : gr.second->launches)
            if (l.second->busy && l.second->agg_gen) return true;
    for (auto& q : queries)
        if (q.second->own && q.second->own->agg_gen) return true;
    return false;
}

void Ctx_::release_retired_agg() {
    if (agg_retired.empty() || ctx_agg_busy()) return;
    for (uint64_t off : agg_retired) arena.release(off);
    agg_retired.clear();
}

int Ctx_::ensure_agg(uint32_t n, const LaunchCfg& cfg) {
    uint64_t w = agg_waves(cfg, n);
    if (agg_off != UINT64_MAX && agg_n >= n && agg_w >= w) return PM_OK;
    if (agg_off != UINT64_MAX) {
        // launch sets built on these arrays are rebuilt on their next use;
        // the arrays go once no launch in flight reads them
        agg_retired.push_back(agg_off);
        agg_retired.push_back(agg_touch_off);
        agg_off = agg_touch_off = UINT64_MAX;
        ++agg_gen;
        release_retired_agg();
    }
    uint64_t need = w * (uint64_t)n * 4;
    agg_off = arena.alloc(need);
    agg_touch_off = arena.alloc(need);
    if (agg_off == UINT64_MAX || agg_touch_off == UINT64_MAX) {
        if (agg_off != UINT64_MAX) arena.release(agg_off);
        if (agg_touch_off != UINT64_MAX) arena.release(agg_touch_off);
        agg_off = agg_touch_off = UINT64_MAX;
        return fail(PM_E_NOMEM, "arena too small for the aggregation counters");
    }
    agg_n = n;
    agg_w = w;
    // the kernel returns every counter it touches to zero, so this runs once
    if (launch_zero((uint32_t*)dptr(agg_off), need / 4, stream)) return fail(PM_E_DEVICE, "zero-fill failed");
    HIPCHK(hipStreamSynchronize(stream));
    return PM_OK;
}

std::string Ctx_::closure_key(const GraphRes& G, const std::vector<Pat>& closure) const {
    std::string k = std::to_string(G.hash) + "|";
    for (const Pat& p : closure) {
        k += std::to_string(p.k) + ":" + std::to_string(p.em) + ":" + (p.vi ? "V" : "E");
        for (int i = 0; i < p.k; ++i) k += "," + std::to_string((int)p.lab[i]);
        k += ";";
    }
    return k;
}

LaunchCfg Ctx_::cfg_for(const GraphRes& G, const std::vector<Pat>& closure) const {
    auto it = tune_cache.find(closure_key(G, closure));
    if (it != tune_cache.end()) return it->second.first;
    return start_cfg(closure);
}

// Untuned launch parameters: the context's, except that a closure with
// 5-vertex patterns gets fine work items (its hub roots' subtrees dominate:
// R-MAT 12 5-MC 1,085 ms with 1024/512, 304 ms with 256/64), unless the
// caller set the item options.
LaunchCfg Ctx_::start_cfg(const std::vector<Pat>& closure) const {
    LaunchCfg c = default_cfg();
    int kmax = 0;
    for (const Pat& q : closure) kmax = std::max(kmax, (int)q.k);
    if (kmax >= 5 && !items_set) {
        c.item_budget = std::min<uint64_t>(c.item_budget, 256);
        c.item_split = std::min<uint32_t>(c.item_split, 64);
    }
    return c;
}

int Ctx_::get_items(GraphRes& G, const LaunchCfg& c, ItemSet** out) {
    auto key = std::make_pair(c.item_budget, c.item_split);
    auto it = G.itemsets.find(key);
    if (it != G.itemsets.end()) {
        *out = &it->second;
        return PM_OK;
    }
    std::vector<KItem> items = build_items(G.host_rp, G.n, c.item_budget, c.item_split, 256);
    ItemSet is;
    is.count = (uint32_t)items.size();
    is.off = arena.alloc(sizeof(KItem) * items.size());
    if (is.off == UINT64_MAX) return fail(PM_E_NOMEM, "arena too small for the work items");
    HIPCHK(hipMemcpyAsync(dptr(is.off), items.data(), sizeof(KItem) * items.size(), hipMemcpyHostToDevice, stream));
    HIPCHK(hipStreamSynchronize(stream));
    *out = &(G.itemsets[key] = is);
    return PM_OK;
}

void Ctx_::free_launchset(LaunchSet* ls) {
    if (!ls) return;
    if (ls->exec) hipGraphExecDestroy(ls->exec);
    if (ls->graph) hipGraphDestroy(ls->graph);
    if (ls->host && !ls->borrowed_host) hipHostFree(ls->host);
    if (ls->cancel_host && !ls->borrowed_host) hipHostFree(ls->cancel_host);
    ls->cancel_host = nullptr;
    ls->cancel_dev = nullptr;
    if (ls->off_mem != UINT64_MAX) arena.release(ls->off_mem);
    ls->exec = nullptr;
    ls->graph = nullptr;
    ls->host = nullptr;
    ls->off_mem = UINT64_MAX;
    ls->agg_gen = 0;
}

int Ctx_::make_launchset(GraphRes& G, const std::vector<PlanInfo>& plans, const LaunchCfg& cfg, LaunchSet* ls,
                         hipStream_t st, const AggArrays* agg) {
    const size_t np = plans.size();
    if (!st) st = stream;
    ls->np = np;
    ls->cfg = cfg;
    uint64_t need = footprint(G, plans, cfg, &ls->stride, &ls->any_agg, agg == nullptr);
    uint32_t p_agg = 0;
    const std::vector<uint32_t> heavy = agg == nullptr ? heavy_roots(G, plans, &p_agg) : std::vector<uint32_t>();
    const uint32_t hk = (uint32_t)heavy.size();
    const std::vector<uint32_t> eheavy = agg == nullptr ? edge_heavy_roots(G, plans) : std::vector<uint32_t>();
    const uint32_t ek = (uint32_t)eheavy.size();
    HIPCHK(hipSetDevice(device));
    if (ls->any_agg && !agg) {
        int rc = ensure_agg(G.n, cfg);
        if (rc) return rc;
    }
    if (ls->any_agg && agg && agg->n < G.n) return fail(PM_E_NOMEM, "slot aggregation arrays too small");
    ItemSet* is;
    int rc = get_items(G, cfg, &is);
    if (rc) return rc;
    // two-hop launches slice hub roots by target range; finer slices keep
    // each wave's window of its counter array cache-resident
    ItemSet* isa = is;
    if (ls->any_agg) {
        LaunchCfg ac = cfg;
        ac.item_split = agg_split;
        rc = get_items(G, ac, &isa);
        if (rc) return rc;
    }
    ls->agg_items = (const KItem*)dptr(isa->off);
    ls->agg_nitems = isa->count;
    std::vector<KItem> light, hitems;
    if (hk) {
        std::vector<uint8_t> is_heavy(G.n, 0);
        for (uint32_t r : heavy) is_heavy[r] = 1;
        // when every two-hop plan is the 4-cycle's pair count over bridges
        // below the root, a root with fewer than two lower neighbours adds
        // nothing: leave it out of the light items too
        bool c4only = true;
        for (const PlanInfo& p : plans)
            if (p.d.agg_last) c4only = c4only && c4_agg_plan(p.d);
        if (c4only)
            for (uint32_t r = 0; r < G.n; ++r)
                if (!G.low2[r]) is_heavy[r] = 1;
        hitems = heavy_items(G, heavy, true);
        light = items_without(build_items(G.host_rp, G.n, cfg.item_budget, agg_split, 256), is_heavy);
    }
    std::vector<KItem> elight, eitems;
    if (ek) {
        std::vector<uint8_t> is_heavy(G.n, 0);
        for (uint32_t r : eheavy) is_heavy[r] = 1;
        eitems = heavy_items(G, eheavy, false);
        elight = items_without(build_items(G.host_rp, G.n, cfg.item_budget, cfg.item_split, 256), is_heavy);
    }
    // serving slots (agg given) take the triangle and 4-clique kernels only
    // where no root is left to the general kernel: nothing to upload then
    const bool cq = use_clique(G, plans) && (agg == nullptr || G.clique_big.empty());
    const std::vector<KItem> cq_big = cq ? clique_big_items(G, cfg) : std::vector<KItem>();
    const bool c4 = use_clique4(G, plans) && (agg == nullptr || G.c4_big.empty());
    // supports: the graph's own array, or a serving slot's (slots run side
    // by side on one graph)
    const bool sup = use_support(G, plans) && (agg == nullptr || (agg->support && agg->support_words >= 2 * G.m));
    bool any_tagg = false, any_vtri = false;
    for (const PlanInfo& p : plans) {
        any_tagg = any_tagg || p.d.tagg != 0;
        any_vtri = any_vtri || tagg_vtri(p.d.tagg) || p.d.tagg == TAGG_HOUSE;
    }
    if (any_tagg && !sup) return fail(PM_E_DEVICE, "internal: a triangle-count plan without triangle counts");
    if (sup && !agg) {
        int rc2 = ensure_support(G);
        if (rc2) return rc2;
    }
    const bool cqs = cq || sup;
    const std::vector<KItem> c4_big = c4 ? clique4_big_items(G, cfg) : std::vector<KItem>();
    ls->off_mem = arena.alloc(need);
    if (ls->off_mem == UINT64_MAX) return fail(PM_E_NOMEM, "arena too small for the query scratch");
    char* base = (char*)dptr(ls->off_mem);
    uint64_t o = 0;
    auto carve = [&](uint64_t bytes) {
        char* p = base + o;
        o += (bytes + 255) & ~uint64_t(255);
        return p;
    };
    ls->dplans = (DPlan*)carve(sizeof(DPlan) * np);
    // counters, queue heads, byte tally and root bitmaps are cleared
    // together by the zero-fill at the head of every replay
    const uint64_t bm_words = bitmap_words(G, plans);
    const uint64_t zhead = (16 * np + 512 + 255) & ~uint64_t(255);
    const uint64_t zbm = (waves(cfg) * bm_words * 4 + 255) & ~uint64_t(255);
    const uint64_t zvt = any_vtri ? ((8ull * G.n + 255) & ~uint64_t(255)) : 0;
    const uint64_t zbytes = zhead + zbm + zvt;
    char* zb = carve(zbytes);
    ls->heavy_items = nullptr;
    ls->heavy_nitems = 0;
    uint32_t* wscr = nullptr;
    const uint64_t wstride = ((uint64_t)G.max_deg + 63) & ~uint64_t(63);
    if (hk || ek) wscr = (uint32_t*)carve((uint64_t)grid_blocks(cfg) * (2 + EW_TERMS) * wstride * 4);
    ls->edge_items = ls->edge_heavy = nullptr;
    ls->edge_nitems = ls->edge_nheavy = 0;
    if (ek) {
        KItem* li = (KItem*)carve(16 * std::max<size_t>(1, elight.size()));
        KItem* hi = (KItem*)carve(16 * eitems.size());
        if (!elight.empty())
            HIPCHK(hipMemcpyAsync(li, elight.data(), 16 * elight.size(), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(hi, eitems.data(), 16 * eitems.size(), hipMemcpyHostToDevice, st));
        ls->edge_items = li;
        ls->edge_nitems = (uint32_t)elight.size();
        ls->edge_heavy = hi;
        ls->edge_nheavy = (uint32_t)eitems.size();
    }
    if (hk) {
        KItem* li = (KItem*)carve(16 * std::max<size_t>(1, light.size()));
        KItem* hi = (KItem*)carve(16 * hitems.size());
        if (!light.empty())
            HIPCHK(hipMemcpyAsync(li, light.data(), 16 * light.size(), hipMemcpyHostToDevice, st));
        HIPCHK(hipMemcpyAsync(hi, hitems.data(), 16 * hitems.size(), hipMemcpyHostToDevice, st));
        ls->agg_items = li;
        ls->agg_nitems = (uint32_t)light.size();
        ls->heavy_items = hi;
        ls->heavy_nitems = (uint32_t)hitems.size();
    }
    ls->cq_items = ls->cq_big = nullptr;
    ls->cq_nitems = ls->cq_nbig = 0;
    ls->support = sup ? (agg ? agg->support : (uint32_t*)dptr(G.off_support)) : nullptr;
    ls->sup_words = sup ? std::max<uint64_t>(1, 2 * G.m) : 0;
    ls->sup_run = -1;
    ls->mirror = false;
    ls->c4_sup = false;
    ls->c4_fill_end = -1;
    if (cqs) {
        ls->cq_items = G.d_cq;
        ls->cq_nitems = (uint32_t)G.clique_items.size();
        if (!cq_big.empty()) {
            KItem* bi = (KItem*)carve(16 * cq_big.size());
            HIPCHK(hipMemcpyAsync(bi, cq_big.data(), 16 * cq_big.size(), hipMemcpyHostToDevice, st));
            ls->cq_big = bi;
            ls->cq_nbig = (uint32_t)cq_big.size();
        }
    }
    ls->c4_light = ls->c4_heavy = ls->c4_huge = ls->c4_big = nullptr;
    ls->c4_nlight = ls->c4_nheavy = ls->c4_nhuge = ls->c4_nbig = 0;
    if (c4) {
        ls->c4_light = G.d_c4l;
        ls->c4_nlight = (uint32_t)G.c4_light.size();
        ls->c4_heavy = G.d_c4h;
        ls->c4_nheavy = (uint32_t)G.c4_heavy.size();
        ls->c4_huge = G.d_c4x;
        ls->c4_nhuge = (uint32_t)G.c4_huge.size();
        if (!c4_big.empty()) {
            KItem* bi = (KItem*)carve(16 * c4_big.size());
            HIPCHK(hipMemcpyAsync(bi, c4_big.data(), 16 * c4_big.size(), hipMemcpyHostToDevice, st));
            ls->c4_big = bi;
            ls->c4_nbig = (uint32_t)c4_big.size();
        }
    }
    ls->zero_base = (uint32_t*)zb;
    ls->zero_words = zbytes / 4;
    ls->counters = (uint64_t*)zb;
    ls->heads = (uint32_t*)(zb + 16 * np);
    ls->bytes = (uint64_t*)(zb + 16 * np + 256);
    uint32_t* rootbm = bm_words ? (uint32_t*)(zb + zhead) : nullptr;
    ls->vtri = any_vtri ? (uint64_t*)(zb + zhead + zbm) : nullptr;
    ls->scratch = (uint32_t*)carve(waves(cfg) * (uint64_t)KMAX * ls->stride * 4);
    // footprint() must account for every carve above
    if (o > need) return fail(PM_E_DEVICE, "internal: launch scratch exceeds its footprint");
    std::vector<DPlan> hp(np);
    for (size_t i = 0; i < np; ++i) hp[i] = plans[i].d;
    if (agg && agg->stage) {
        // pinned staging: a pageable upload could wait for other streams
        if (agg->stage_bytes < sizeof(DPlan) * np) return fail(PM_E_NOMEM, "slot staging buffer too small");
        // no synchronisation: the slot's stream orders the upload before the
        // launches, and the slot reuses the staging only after its event
        memcpy(agg->stage, hp.data(), sizeof(DPlan) * np);
        HIPCHK(hipMemcpyAsync(ls->dplans, agg->stage, sizeof(DPlan) * np, hipMemcpyHostToDevice, st));
    } else {
        HIPCHK(hipMemcpyAsync(ls->dplans, hp.data(), sizeof(DPlan) * np, hipMemcpyHostToDevice, st));
        HIPCHK(hipStreamSynchronize(st));
    }
    if (agg && agg->host) {
        if (agg->host_words < 2 * np + 2 + MAX_RUNS) return fail(PM_E_NOMEM, "slot result buffer too small");
        ls->host = agg->host;
        ls->cancel_host = agg->cancel_host;
        ls->cancel_dev = agg->cancel_dev;
        ls->borrowed_host = true;
    } else {
        HIPCHK(hipHostMalloc((void**)&ls->host, 16 * np + 8 * (2 + MAX_RUNS), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void**)&ls->cancel_host, 64, hipHostMallocMapped | hipHostMallocCoherent));
        HIPCHK(hipHostGetDevicePointer((void**)&ls->cancel_dev, ls->cancel_host, 0));
    }
    __atomic_store_n(ls->cancel_host, 0, __ATOMIC_SEQ_CST);
    KArgs& a = ls->base;
    memset(&a, 0, sizeof(a));
    a.g.rp = (const uint32_t*)dptr(G.off_rp);
    a.g.col = (const uint32_t*)dptr(G.off_col);
    a.g.split = (const uint32_t*)dptr(G.off_split);
    a.g.lab = G.labeled ? (const uint8_t*)dptr(G.off_lab) : nullptr;
    a.g.n = G.n;
    if (G.off_hubbm != UINT64_MAX && hub_bitmaps_opt) {
        a.g.hubbm = (const uint32_t*)dptr(G.off_hubbm);
        a.g.hub0 = G.hub0;
        a.g.hub_words = G.hub_words;
    }
    a.items = (const KItem*)dptr(is->off);
    a.nitems = is->count;
    a.scratch = ls->scratch;
    a.buf_stride = ls->stride;
    a.bytes = ls->bytes;
    a.cancel = ls->cancel_dev;
    a.rootbm = rootbm;
    a.bm_words = bm_words;
    a.wscr = wscr;
    a.wscr_stride = wstride;
    a.wide = window_wide ? 1u : 0u;
    if (ls->any_agg) {
        if (agg) {
            a.aggcnt = agg->cnt;
            a.aggtouch = agg->touch;
            ls->agg_w = agg->waves;
        } else {
            a.aggcnt = (uint32_t*)dptr(agg_off);
            a.aggtouch = (uint32_t*)dptr(agg_touch_off);
            ls->agg_gen = agg_gen;
            ls->agg_w = agg_waves(cfg, G.n);
        }
    }
    ls->runs.clear();
    ls->run_agg.clear();
    // runs: plain plans; triangle-core plans (clique_kernel, CQ_PLANS a
    // launch, then the general kernel over the roots it leaves out);
    // edge-core plans (light roots, then heavy roots in LDS windows);
    // two-hop plans (light roots, then heavy roots)
    auto group = [&](int q) {
        if (plans[q].d.cyc5) return 6;
        if (plans[q].d.tagg) return 5;
        if (plans[q].d.agg_last) return 2;
        if (cq && clique_runs(G, plans[q].d)) return 3;
        if ((sup && support_ok(plans[q].d)) || (clique_opt && edge_cheap_ok(plans[q].d))) return 5;
        if (c4 && clique4_ok(plans[q].d)) return 4;
        return (ek && edge_window_ok(plans[q].d)) ? 1 : 0;
    };
    int i = 0;
    bool vtri_added = false;
    while (i < (int)np) {
        const int grp = group(i);
        int j = i;
        while (j < (int)np && group(j) == grp) ++j;
        if (grp == 0) {
            ls->runs.push_back({i, j});
            ls->run_agg.push_back(0);
        } else if (grp == 3) {
            for (int k = i; k < j; k += CQ_PLANS) {
                // the first triangle pass also fills the edge supports
                if (sup && ls->sup_run < 0) ls->sup_run = (int)ls->runs.size();
                ls->runs.push_back({k, std::min(j, k + CQ_PLANS)});
                ls->run_agg.push_back(5);
            }
            if (!cq_big.empty()) {
                ls->runs.push_back({i, j});
                ls->run_agg.push_back(6);
            }
        } else if (grp == 5) {
            bool need = false, tg = false;
            for (int k = i; k < j; ++k) {
                need = need || !edge_cheap_ok(plans[k].d);
                tg = tg || tagg_vtri(plans[k].d.tagg) || plans[k].d.tagg == TAGG_HOUSE;
            }
            if (need && ls->sup_run < 0) {
                // no triangle-core plan: a pass that only fills the supports
                ls->sup_run = (int)ls->runs.size();
                ls->runs.push_back({i, i});
                ls->run_agg.push_back(5);
            }
            if (tg && !vtri_added) {
                // per-vertex triangle counts from the supports (mirrored for
                // the house), once
                vtri_added = true;
                ls->runs.push_back({i, i});
                ls->run_agg.push_back(13);
            }
            for (int k = i; k < j; ++k)
                if (plans[k].d.tagg == TAGG_HOUSE) {
                    ls->mirror = true;
                    ls->runs.push_back({k, k + 1});
                    ls->run_agg.push_back(14);
                } else if (tagg_tri(plans[k].d.tagg)) {
                    ls->runs.push_back({k, k + 1});
                    ls->run_agg.push_back(15);
                } else if (plans[k].d.tagg == TAGG_K4EAR) {
                    // the 4-clique items of each size class
                    for (int code : {18, 17, 16}) {
                        const uint32_t n4 = code == 18 ? ls->c4_nhuge : (code == 17 ? ls->c4_nheavy : ls->c4_nlight);
                        if (!n4) continue;
                        ls->runs.push_back({k, k + 1});
                        ls->run_agg.push_back(code);
                    }
                }
            for (int k = i; k < j; k += CQ_PLANS) {
                ls->runs.push_back({k, std::min(j, k + CQ_PLANS)});
                ls->run_agg.push_back(10);
            }
        } else if (grp == 4) {
            // with no triangle pass before them, the first set of 4-clique
            // launches fills the edge supports while it builds its rows
            const bool fill = sup && ls->sup_run < 0;
            if (fill) {
                ls->c4_sup = true;
                ls->sup_run = (int)ls->runs.size();
            }
            for (int k = i; k < j; k += CQ_PLANS) {
                const std::pair<int, int> rr{k, std::min(j, k + CQ_PLANS)};
                if (ls->c4_nhuge) {
                    ls->runs.push_back(rr);
                    ls->run_agg.push_back(11);
                }
                if (ls->c4_nheavy) {
                    ls->runs.push_back(rr);
                    ls->run_agg.push_back(8);
                }
                if (ls->c4_nlight) {
                    ls->runs.push_back(rr);
                    ls->run_agg.push_back(7);
                }
                if (fill && k == i) ls->c4_fill_end = (int)ls->runs.size();
            }
            if (!c4_big.empty()) {
                ls->runs.push_back({i, j});
                ls->run_agg.push_back(9);
            }
        } else if (grp == 6) {
            ls->runs.push_back({i, j});
            ls->run_agg.push_back(12);
        } else if (grp == 1) {
            ls->runs.push_back({i, j});
            ls->run_agg.push_back(3);
            ls->runs.push_back({i, j});
            ls->run_agg.push_back(4);
        } else {
            ls->runs.push_back({i, j});
            ls->run_agg.push_back(1);
            if (hk) {
                ls->runs.push_back({i, j});
                ls->run_agg.push_back(2);
            }
        }
        i = j;
    }
    // pageable uploads above must finish before their host vectors go
    if (hk || ek || !cq_big.empty() || !c4_big.empty()) HIPCHK(hipStreamSynchronize(st));
    return PM_OK;
}

// The kernel a launch-set run uses (LaunchSet::run_agg codes).
const char* run_kernel_name(int kind) {
    switch (kind) {
        case 2: return "agg_window_kernel";
        case 4: return "edge_window_kernel";
        case 5: return "clique_kernel";
        case 7: case 8: case 11: return "clique4_kernel";
        case 10: return "support_kernel";
        case 12: return "cycle5_kernel";
        case 13: return "vtri_kernel";
        case 14: return "house_kernel";
        case 15: return "trisup_kernel";
        case 16: case 17: case 18: return "k4ear_kernel";
        default: return "match_kernel";
    }
}

// [zero-fill -> match launches -> copy-back]; with bytes_pass the same
// launches run in the byte-counting build and only the tally is copied
// (host slot 2*np+1), outside any timed region.
// Branch of a run when a captured launch set forks: 1 = triangle pass and
// edge supports (in order: the supports read what the pass writes), 2 =
// 4-cliques; 0 = the rest (general kernel and window kernels, which share
// the per-wavefront level buffers and window scratch).
static int run_branch(int kind) {
    if (kind == 5 || kind == 10 || (kind >= 13 && kind <= 18)) return 1;
    if (kind == 7 || kind == 8 || kind == 11) return 2;
    return 0;
}

int Ctx_::enqueue(LaunchSet& ls, hipStream_t s0, bool bytes_pass, hipEvent_t* run_ev, bool fork) {
    const LaunchCfg& cfg = ls.cfg;
    if (ls.runs.size() > MAX_RUNS) return fail(PM_E_DEVICE, "internal: too many launches in one set");
    // a serving slot's share of the launches sized by CU count (persistent
    // workgroups that hold CUs until their queue drains)
    auto shared = [&](int grid) { return cfg.share_div > 1 ? std::max(1, grid / cfg.share_div) : grid; };
    if (launch_zero(ls.zero_base, ls.zero_words, s0)) return fail(PM_E_DEVICE, "zero-fill launch failed");
    // the supports start from zero on every replay, also after a cancelled
    // one that stopped before reading them
    if (ls.support && launch_zero(ls.support, ls.sup_words, s0)) return fail(PM_E_DEVICE, "zero-fill launch failed");
    if (run_ev) HIPCHK(hipEventRecord(run_ev[0], s0));
    // house_kernel shares the per-wave dense counters with the two-hop and
    // 5-cycle launches of the main branch, and supports filled by 4-clique
    // launches are read on the triangle branch: no fork then
    fork = fork && !ls.mirror && !ls.c4_sup;
    bool used[3] = {true, false, false};
    if (fork) {
        for (int k = 0; k < 2; ++k) {
            if (!branch[k]) HIPCHK(hipStreamCreateWithFlags(&branch[k], hipStreamNonBlocking));
            if (!join_ev[k]) HIPCHK(hipEventCreateWithFlags(&join_ev[k], hipEventDisableTiming));
        }
        if (!fork_ev) HIPCHK(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
        HIPCHK(hipEventRecord(fork_ev, s0));
        for (size_t r = 0; r < ls.runs.size(); ++r) {
            const int br = run_branch(ls.run_agg[r]);
            if (br && !used[br]) {
                used[br] = true;
                HIPCHK(hipStreamWaitEvent(branch[br - 1], fork_ev, 0));
            }
        }
    }
    for (size_t r = 0; r < ls.runs.size(); ++r) {
        hipStream_t s = fork && run_branch(ls.run_agg[r]) ? branch[run_branch(ls.run_agg[r]) - 1] : s0;
        if (run_ev && r > 0) HIPCHK(hipEventRecord(run_ev[r], s));
        KArgs b = ls.base;
        b.bytes = ls.bytes + r;
        b.plans = ls.dplans + ls.runs[r].first;
        b.nplans = ls.runs[r].second - ls.runs[r].first;
        b.counters = ls.counters + 2 * ls.runs[r].first;
        b.head = ls.heads + r;
        int gb = grid_blocks(cfg);
        if (ls.run_agg[r] == 1) {
            b.items = ls.agg_items;
            b.nitems = ls.agg_nitems;
            gb = (int)std::max<uint64_t>(1, ls.agg_w / (block / 64));
        } else if (ls.run_agg[r] == 12) {
            gb = (int)std::max<uint64_t>(1, ls.agg_w / (block / 64));
            if (b.nitems && launch_cycle5(b, gb, bytes_pass, s)) return fail(PM_E_DEVICE, "kernel launch failed");
            continue;
        } else if (ls.run_agg[r] == 2) {
            b.items = ls.heavy_items;
            b.nitems = ls.heavy_nitems;
            if (b.nitems && launch_agg_window(b, std::min(gb, num_cus * agg_window_cu_blocks()), bytes_pass, s))
                return fail(PM_E_DEVICE, "kernel launch failed");
            continue;
        } else if (ls.run_agg[r] == 3) {
            b.items = ls.edge_items;
            b.nitems = ls.edge_nitems;
        } else if (ls.run_agg[r] == 5) {
            b.items = ls.cq_items;
            b.nitems = ls.cq_nitems;
            b.support = (int)r == ls.sup_run ? ls.support : nullptr;
            if (b.nitems && launch_clique(b, shared(clique_blocks(b.support != nullptr, b.g.n)), bytes_pass, s))
                return fail(PM_E_DEVICE, "kernel launch failed");
            continue;
        } else if (ls.run_agg[r] == 10) {
            b.support = ls.support;
            b.vtri = ls.vtri;
            b.mirror = ls.mirror ? 1u : 0u;
            if (launch_support(b, shared(support_blocks()), bytes_pass, s)) return fail(PM_E_DEVICE, "kernel launch failed");
            continue;
        } else if (ls.run_agg[r] == 13) {
            b.support = ls.support;
            b.vtri = ls.vtri;
            b.mirror = ls.mirror ? 1u : 0u;
            if (launch_vtri(b, shared(support_blocks()), bytes_pass, s)) return fail(PM_E_DEVICE, "kernel launch failed");
            continue;
        } else if (ls.run_agg[r] >= 16 && ls.run_agg[r] <= 18) {
            const int mode = ls.run_agg[r] - 16;
            b.items = mode == 0 ? ls.c4_light : (mode == 1 ? ls.c4_heavy : ls.c4_huge);
            b.nitems = mode == 0 ? ls.c4_nlight : (mode == 1 ? ls.c4_nheavy : ls.c4_nhuge);
            b.support = ls.support;
            if (b.nitems && launch_k4ear(b, shared(clique4_blocks(mode)), mode, bytes_pass, s))
                return fail(PM_E_DEVICE, "kernel launch failed");
            continue;
        } else if (ls.run_agg[r] == 15) {
            b.items = ls.cq_items;
            b.nitems = ls.cq_nitems;
            b.support = ls.support;
            // 48 KB of LDS a workgroup: three resident a CU
            if (b.nitems && launch_trisup(b, shared(num_cus * 3), bytes_pass, s)) return fail(PM_E_DEVICE, "kernel launch failed");
            continue;
        } else if (ls.run_agg[r] == 14) {
            b.support = ls.support;
            gb = (int)std::max<uint64_t>(1, ls.agg_w / (block / 64));
            if (b.nitems && launch_house(b, gb, bytes_pass, s)) return fail(PM_E_DEVICE, "kernel launch failed");
            continue;
        } else if (ls.run_agg[r] == 6) {
            b.items = ls.cq_big;
            b.nitems = ls.cq_nbig;
        } else if (ls.run_agg[r] == 7 || ls.run_agg[r] == 8 || ls.run_agg[r] == 11) {
            const int mode = ls.run_agg[r] == 7 ? 0 : (ls.run_agg[r] == 8 ? 1 : 2);
            b.items = mode == 0 ? ls.c4_light : (mode == 1 ? ls.c4_heavy : ls.c4_huge);
            b.nitems = mode == 0 ? ls.c4_nlight : (mode == 1 ? ls.c4_nheavy : ls.c4_nhuge);
            if (ls.c4_sup && (int)r >= ls.sup_run && (int)r < ls.c4_fill_end) b.support = ls.support;
            if (b.nitems && launch_clique4(b, shared(clique4_blocks(mode)), mode, bytes_pass, s))
                return fail(PM_E_DEVICE, "kernel launch failed");
            continue;
        } else if (ls.run_agg[r] == 9) {
            b.items = ls.c4_big;
            b.nitems = ls.c4_nbig;
        } else if (ls.run_agg[r] == 4) {
            b.items = ls.edge_heavy;
            b.nitems = ls.edge_nheavy;
            if (b.nitems && launch_edge_window(b, gb, bytes_pass, s)) return fail(PM_E_DEVICE, "kernel launch failed");
            continue;
        }
        if (b.nitems == 0) continue;
        if (launch_match(b, gb, block, bytes_pass, s)) return fail(PM_E_DEVICE, "kernel launch failed");
    }
    if (fork)
        for (int k = 0; k < 2; ++k)
            if (used[k + 1]) {
                HIPCHK(hipEventRecord(join_ev[k], branch[k]));
                HIPCHK(hipStreamWaitEvent(s0, join_ev[k], 0));
            }
    if (run_ev) HIPCHK(hipEventRecord(run_ev[ls.runs.size()], s0));
    if (bytes_pass) {
        HIPCHK(hipMemcpyAsync(ls.host + 2 * ls.np + 2, ls.bytes, 8 * MAX_RUNS, hipMemcpyDeviceToHost, s0));
        return PM_OK;
    }
    HIPCHK(hipMemcpyAsync(ls.host, ls.counters, 16 * ls.np, hipMemcpyDeviceToHost, s0));
    return PM_OK;
}

int Ctx_::run_eager_ms(GraphRes& G, const std::vector<PlanInfo>& plans, const LaunchCfg& c, double* ms) {
    LaunchSet ls;
    int rc = make_launchset(G, plans, c, &ls);
    if (rc) {
        free_launchset(&ls);
        return rc;
    }
    hipEvent_t e0, e1;
    hipEventCreate(&e0);
    hipEventCreate(&e1);
    hipEventRecord(e0, stream);
    rc = enqueue(ls, stream, false);
    hipEventRecord(e1, stream);
    hipError_t he = hipEventSynchronize(e1);
    float f = 0;
    hipEventElapsedTime(&f, e0, e1);
    hipEventDestroy(e0);
    hipEventDestroy(e1);
    free_launchset(&ls);
    if (he != hipSuccess) return fail(PM_E_DEVICE, std::string("tuning run failed: ") + hipGetErrorString(he));
    *ms = f;
    return rc;
}

int Ctx_::autotune(uint32_t gid, const pm_pattern* pats, uint32_t npat, int morph, int64_t* out_cfg,
                   double* out_ms) {
    GraphRes* G;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = graphs.find(gid);
        if (it == graphs.end()) return fail(PM_E_NOTFOUND, "unknown graph id");
        G = it->second.get();
    }
    std::vector<Pat> ps(npat);
    for (uint32_t i = 0; i < npat; ++i) {
        std::string err;
        int rc = to_pat(pats[i], &ps[i], &err);
        if (rc) return fail(rc, err);
    }
    MorphPlan mp;
    std::string err;
    int rc = morph_plan_count(ps, morph, &mp, &err, cost_fn(*G));
    if (rc) return fail(rc, err);
    std::vector<Pat> closure;
    std::vector<PlanInfo> plans;
    rc = plan_closure(*G, mp.alt, &closure, &plans);
    if (rc) return fail(rc, g_err);
    std::string key = closure_key(*G, closure);
    auto hit = tune_cache.find(key);
    if (hit == tune_cache.end()) {
        // coordinate descent over the launch parameters, timed on the graph
        LaunchCfg best = start_cfg(closure);
        double best_ms;
        rc = run_eager_ms(*G, plans, best, &best_ms);
        if (rc) return rc;
        const int bpcs[] = {1, 2, 4, 8};
        const uint64_t budgets[] = {256, 1024, 4096, 16384, 65536};
        const uint32_t splits[] = {32, 64, 512, 2048, 8192};
        for (int stage = 0; stage < 3; ++stage) {
            int nvals = stage == 0 ? 4 : 5;
            for (int v = 0; v < nvals; ++v) {
                LaunchCfg c = best;
                if (stage == 0) c.blocks_per_cu = bpcs[v];
                if (stage == 1) c.item_budget = budgets[v];
                if (stage == 2) c.item_split = splits[v];
                if (c.blocks_per_cu == best.blocks_per_cu && c.item_budget == best.item_budget &&
                    c.item_split == best.item_split)
                    continue;
                double ms;
                rc = run_eager_ms(*G, plans, c, &ms);
                if (rc == PM_E_NOMEM) continue;
                if (rc) return rc;
                if (ms < best_ms) {
                    best_ms = ms;
                    best = c;
                }
            }
        }
        hit = tune_cache.emplace(key, std::make_pair(best, best_ms)).first;
        if (!tune_file.empty()) {
            FILE* f = fopen(tune_file.c_str(), "a");
            if (f) {
                fprintf(f, "%d %llu %u %.6f %s\n", best.blocks_per_cu, (unsigned long long)best.item_budget,
                        best.item_split, best_ms, key.c_str());
                fclose(f);
            }
        }
    }
    if (out_cfg) {
        out_cfg[0] = hit->second.first.blocks_per_cu;
        out_cfg[1] = (int64_t)hit->second.first.item_budget;
        out_cfg[2] = hit->second.first.item_split;
    }
    if (out_ms) *out_ms = hit->second.second;
    return PM_OK;
}

void Ctx_::load_tune_file() {
    const char* env = getenv("PM_AUTOTUNE_CACHE");
    if (!env || !*env) return;
    tune_file = env;
    FILE* f = fopen(env, "r");
    if (!f) return;
    char line[65536];
    while (fgets(line, sizeof(line), f)) {
        int bpc;
        unsigned long long bud;
        unsigned spl;
        double ms;
        int off = 0;
        if (sscanf(line, "%d %llu %u %lf %n", &bpc, &bud, &spl, &ms, &off) != 4) continue;
        std::string key(line + off);
        while (!key.empty() && (key.back() == '\n' || key.back() == '\r')) key.pop_back();
        if (bpc < 1 || bpc > 64 || bud < 1 || spl < 64) continue;
        tune_cache[key] = {LaunchCfg{bpc, (uint64_t)bud, (uint32_t)spl}, ms};
    }
    fclose(f);
}

int Ctx_::submit(uint32_t gid, const pm_pattern* pats, uint32_t npat, int agg, int morph,
                 uint64_t* ticket) {
    auto t0 = std::chrono::steady_clock::now();
    if (!pats || !ticket || npat == 0) return fail(PM_E_INVAL, "null patterns or ticket");
    if (agg != PM_AGG_COUNT && agg != PM_AGG_MNI) return fail(PM_E_INVAL, "unknown aggregation");
    if (morph != PM_MORPH_NONE && morph != PM_MORPH_NAIVE && morph != PM_MORPH_COST)
        return fail(PM_E_INVAL, "unknown morph mode");
    GraphRes* G;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = graphs.find(gid);
        if (it == graphs.end()) return fail(PM_E_NOTFOUND, "unknown graph id");
        G = it->second.get();
    }
    auto Q = std::make_unique<Query>();
    Q->gid = gid;
    Q->npat = npat;
    std::vector<Pat> ps(npat);
    for (uint32_t i = 0; i < npat; ++i) {
        std::string err;
        int rc = to_pat(pats[i], &ps[i], &err);
        if (rc) return fail(rc, err);
        for (int v = 0; v < ps[i].k; ++v)
            if (ps[i].lab[v] >= 0 && !G->labeled) return fail(PM_E_INVAL, "labeled pattern on an unlabeled graph");
    }
    if (agg == PM_AGG_MNI) return submit_mni(*G, gid, ps, morph, ticket);
    std::string err;
    int rc = morph_plan_count(ps, morph, &Q->mp, &err, cost_fn(*G));
    if (rc) return fail(rc, err);
    rc = plan_closure(*G, Q->mp.alt, &Q->closure, &Q->plans);
    if (rc) return fail(rc, g_err);
    auto t1 = std::chrono::steady_clock::now();
    Q->stats.plan_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    Q->stats.num_alt = (uint32_t)Q->plans.size();
    Q->t_submit = t0;
    rc = launch(*G, *Q);
    if (rc) return rc;
    std::lock_guard<std::mutex> g(mu);
    uint64_t tk = next_ticket++;
    G->inflight++;
    queries[tk] = std::move(Q);
    *ticket = tk;
    return PM_OK;
}

// Frees every cached launch set that is not in flight, on every graph.
int Ctx_::evict_idle() {
    int k = 0;
    std::lock_guard<std::mutex> g(mu);
    for (auto& gr : graphs) {
        auto& L = gr.second->launches;
        for (auto it = L.begin(); it != L.end();) {
            if (!it->second->busy) {
                free_launchset(it->second.get());
                it = L.erase(it);
                ++k;
            } else {
                ++it;
            }
        }
    }
    return k;
}

int Ctx_::launch(GraphRes& G, Query& Q) {
    const LaunchCfg cfg = cfg_for(G, Q.closure);
    HIPCHK(hipSetDevice(device));
    LaunchSet* ls = nullptr;
    bool replay = use_graphs && !count_bytes && !launch_events;
    std::string key = closure_key(G, Q.closure) + "#" + std::to_string(cfg.blocks_per_cu) + "," +
                      std::to_string(cfg.item_budget) + "," + std::to_string(cfg.item_split) + "," +
                      std::to_string(agg_split) + "," + std::to_string(heavy_roots_opt) + "," +
                      std::to_string(heavy_min_mass) + "," + std::to_string(clique_opt) + "," +
                      std::to_string(heavy_span_shift) + "," + std::to_string(support_opt) + "," +
                      std::to_string(window_wide) + "," + std::to_string(hub_bitmaps_opt);
    if (replay) {
        auto it = G.launches.find(key);
        if (it != G.launches.end() && !it->second->busy && it->second->agg_gen &&
            it->second->agg_gen != agg_gen) {
            // built on two-hop arrays that have since been reallocated
            free_launchset(it->second.get());
            G.launches.erase(it);
            it = G.launches.end();
        }
        if (it != G.launches.end() && !it->second->busy) {
            ls = it->second.get();
        } else if (it == G.launches.end()) {
            auto nls = std::make_unique<LaunchSet>();
            int rc = make_launchset(G, Q.plans, cfg, nls.get());
            if (rc == PM_E_NOMEM) {
                // make room: drop cached launch sets that are not in flight
                free_launchset(nls.get());
                nls = std::make_unique<LaunchSet>();
                if (evict_idle() > 0) rc = make_launchset(G, Q.plans, cfg, nls.get());
            }
            if (rc) {
                free_launchset(nls.get());
                return rc;
            }
            // capture [zero-fill -> launches -> copy-back] once; replay later
            if (!cap_stream) HIPCHK(hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking));
            HIPCHK(hipStreamBeginCapture(cap_stream, hipStreamCaptureModeRelaxed));
            int erc = enqueue(*nls, cap_stream, false, nullptr, fork_launches);
            hipGraph_t graph = nullptr;
            hipError_t ce = hipStreamEndCapture(cap_stream, &graph);
            if (erc || ce != hipSuccess) {
                if (graph) hipGraphDestroy(graph);
                free_launchset(nls.get());
                return erc ? erc : fail(PM_E_DEVICE, std::string("graph capture failed: ") + hipGetErrorString(ce));
            }
            nls->graph = graph;
            hipError_t ie = hipGraphInstantiate(&nls->exec, graph, nullptr, nullptr, 0);
            if (ie != hipSuccess) {
                free_launchset(nls.get());
                return fail(PM_E_DEVICE, std::string("graph instantiate failed: ") + hipGetErrorString(ie));
            }
            ls = nls.get();
            G.launches[key] = std::move(nls);
        }
    }
    if (!ls) {
        Q.own = std::make_unique<LaunchSet>();
        int rc = make_launchset(G, Q.plans, cfg, Q.own.get());
        if (rc == PM_E_NOMEM) {
            free_launchset(Q.own.get());
            Q.own = std::make_unique<LaunchSet>();
            if (evict_idle() > 0) rc = make_launchset(G, Q.plans, cfg, Q.own.get());
        }
        if (rc) {
            free_launchset(Q.own.get());
            Q.own.reset();
            return rc;
        }
    }
    if (!Q.ev_start) {
        HIPCHK(hipEventCreate(&Q.ev_start));
        HIPCHK(hipEventCreate(&Q.ev_stop));
        HIPCHK(hipEventCreate(&Q.ev_done));
    }
    if (launch_events) {
        LaunchSet& L0 = ls ? *ls : *Q.own;
        Q.run_ev.assign(L0.runs.size() + 1, nullptr);
        for (auto& e : Q.run_ev) HIPCHK(hipEventCreate(&e));
        Q.run_kind = L0.run_agg;
    }
    Q.counted_bytes = !ls && count_bytes;
    if (Q.counted_bytes) {
        int rc = enqueue(*Q.own, stream, true);
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(Q.ev_start, stream));
    if (ls) {
        ls->busy = true;
        Q.ls = ls;
        *(volatile int*)ls->cancel_host = 0;
        HIPCHK(hipGraphLaunch(ls->exec, stream));
    } else {
        int rc = enqueue(*Q.own, stream, false, Q.run_ev.empty() ? nullptr : Q.run_ev.data());
        if (rc) return rc;
    }
    HIPCHK(hipEventRecord(Q.ev_stop, stream));
    HIPCHK(hipEventRecord(Q.ev_done, stream));
    LaunchSet& L = ls ? *ls : *Q.own;
    Q.stats.launches = (uint32_t)L.runs.size();
    Q.stats.work_items = (uint64_t)L.base.nitems * L.np;
    return PM_OK;
}

// Exact counts of the closure patterns from the 128-bit match totals of
// their plans (host words 2i, 2i+1), smallest patterns first because
// quotient plans subtract counts of smaller patterns.  st[i] is PM_OK,
// PM_E_OVERFLOW (the total exceeds 120 bits, the count exceeds int64, or a
// count it needs did) or PM_E_DEVICE (an internal inconsistency), with the
// message in err[i].
void closure_counts(const std::vector<Pat>& closure, const std::vector<PlanInfo>& plans, const uint64_t* host,
                    std::vector<__int128>* cnt_out, std::vector<int>* st_out, std::vector<std::string>* err_out) {
    const size_t np = plans.size();
    std::vector<__int128>& cnt = *cnt_out;
    std::vector<int>& st = *st_out;
    std::vector<std::string>& err = *err_out;
    cnt.assign(np, -1);
    st.assign(np, PM_OK);
    err.assign(np, std::string());
    std::vector<size_t> order(np);
    for (size_t i = 0; i < np; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) { return closure[a].k < closure[b].k; });
    for (size_t i : order) {
        const PlanInfo& pi = plans[i];
        const unsigned __int128 v = ((unsigned __int128)host[2 * i + 1] << 64) | host[2 * i];
        // below 2^120 every product with a plan multiplier (< 2^7) stays
        // inside the signed 128-bit range
        if (v >> 120) {
            st[i] = PM_E_OVERFLOW;
            err[i] = "match total exceeds 120 bits";
            continue;
        }
        __int128 c;
        if (pi.cyc5) {
            // pair sum minus the companion triangle plan's total
            const size_t j = pi.subs.empty() ? np
                                             : std::find(closure.begin(), closure.end(), pi.subs[0].first) -
                                                   closure.begin();
            if (j >= np || cnt[j] < 0) {
                st[i] = j < np && st[j] ? st[j] : PM_E_DEVICE;
                err[i] = j < np && st[j] ? err[j] : "internal: 5-cycle companion plan missing";
                continue;
            }
            c = (__int128)v - cnt[j];
            if (c < 0) {
                st[i] = PM_E_DEVICE;
                err[i] = "internal: negative 5-cycle count";
                continue;
            }
        } else if (pi.rewrite) {
            __int128 acc = (__int128)pi.hmult * (__int128)v;
            for (auto& sq : pi.subs) {
                size_t j = std::find(closure.begin(), closure.end(), sq.first) - closure.begin();
                if (j >= np) {
                    st[i] = PM_E_DEVICE;
                    err[i] = "internal: quotient sub-pattern missing";
                    break;
                }
                if (st[j]) {
                    st[i] = st[j];
                    err[i] = err[j];
                    break;
                }
                acc -= (__int128)sq.second * cnt[j];
            }
            if (st[i]) continue;
            if (acc < 0 || acc % pi.autp) {
                st[i] = PM_E_DEVICE;
                err[i] = "internal: quotient combination not exact";
                continue;
            }
            c = acc / pi.autp;
        } else {
            if (v % (unsigned __int128)pi.divisor) {
                st[i] = PM_E_DEVICE;
                err[i] = "internal: match total not divisible by the plan divisor";
                continue;
            }
            c = (__int128)(v / (unsigned __int128)pi.divisor);
        }
        if (c > (__int128)INT64_MAX) {
            st[i] = PM_E_OVERFLOW;
            err[i] = "count exceeds int64";
            continue;
        }
        cnt[i] = c;
    }
}

int Ctx_::wait(uint64_t ticket, int64_t* out, int64_t timeout_us) {
    Query* Q;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = queries.find(ticket);
        if (it == queries.end()) return fail(PM_E_NOTFOUND, "unknown ticket");
        Q = it->second.get();
    }
    auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        hipError_t e = hipEventQuery(Q->ev_done);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) return fail(PM_E_DEVICE, std::string("query failed: ") + hipGetErrorString(e));
        if (timeout_us >= 0) {
            double us = std::chrono::duration<double, std::micro>(std::chrono::steady_clock::now() - t0).count();
            if (us > (double)timeout_us) return fail(PM_E_TIMEOUT, "timeout");
        }
        std::this_thread::yield();
    }
    if (Q->mni) {
        const int rc = finish_mni(*Q, out);
        std::lock_guard<std::mutex> g(mu);
        hipEventDestroy(Q->ev_start);
        hipEventDestroy(Q->ev_stop);
        hipEventDestroy(Q->ev_done);
        auto git = graphs.find(Q->gid);
        if (git != graphs.end()) git->second->inflight--;
        queries.erase(ticket);
        return rc;
    }
    float kms = 0;
    hipEventElapsedTime(&kms, Q->ev_start, Q->ev_stop);
    Q->stats.kernel_ms = kms;
    size_t np = Q->plans.size();
    const uint64_t* host = Q->ls ? Q->ls->host : Q->own->host;
    std::vector<__int128> cnt;
    std::vector<int> cst;
    std::vector<std::string> cerr;
    closure_counts(Q->closure, Q->plans, host, &cnt, &cst, &cerr);
    int rc = PM_OK;
    for (size_t i = 0; i < np && rc == PM_OK; ++i)
        if (cst[i]) rc = fail(cst[i], cerr[i]);
    std::vector<int64_t> alt(Q->mp.alt.size(), 0);
    if (rc == PM_OK)
        for (size_t j = 0; j < alt.size(); ++j) {
            size_t i = std::find(Q->closure.begin(), Q->closure.end(), Q->mp.alt[j]) - Q->closure.begin();
            alt[j] = (int64_t)cnt[i];
        }
    std::vector<int64_t> res;
    if (rc == PM_OK && Q->cancelled) rc = fail(PM_E_CANCELLED, "query cancelled");
    if (rc == PM_OK) {
        std::string err;
        rc = unmorph(Q->mp, Q->npat, alt, &res, &err);
        if (rc) fail(rc, err);
    }
    if (rc == PM_OK && out) memcpy(out, res.data(), sizeof(int64_t) * Q->npat);
    Q->stats.alg_bytes = 0;
    last_launches.clear();
    {
        LaunchSet& L0 = Q->ls ? *Q->ls : *Q->own;
        for (size_t r = 0; r < L0.runs.size(); ++r) {
            pm_launch_stat ls_{};
            snprintf(ls_.kernel, sizeof(ls_.kernel), "%s", run_kernel_name(L0.run_agg[r]));
            ls_.alg_bytes = Q->counted_bytes ? host[2 * np + 2 + r] : 0;
            Q->stats.alg_bytes += ls_.alg_bytes;
            float ms = 0;
            if (Q->run_ev.size() > r + 1) hipEventElapsedTime(&ms, Q->run_ev[r], Q->run_ev[r + 1]);
            ls_.ms = ms;
            last_launches.push_back(ls_);
        }
    }
    for (auto& e : Q->run_ev) hipEventDestroy(e);
    Q->run_ev.clear();
    Q->stats.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - Q->t_submit).count();
    last_stats = Q->stats;
    last_alt = alt;
    // release
    {
        std::lock_guard<std::mutex> g(mu);
        if (Q->ls) Q->ls->busy = false;
        if (Q->own) free_launchset(Q->own.get());
        hipEventDestroy(Q->ev_start);
        hipEventDestroy(Q->ev_stop);
        hipEventDestroy(Q->ev_done);
        auto git = graphs.find(Q->gid);
        if (git != graphs.end()) git->second->inflight--;
        queries.erase(ticket);
    }
    release_retired_agg();
    return rc;
}

}  // namespace pm

// ================================================================ C-ABI

using namespace pm;


extern "C" {

pm_status pm_create(void* dev_arena, uint64_t arena_bytes, void* hip_stream, int device, pm_ctx** out) {
    if (!out || !dev_arena) return fail(PM_E_INVAL, "null arena or out");
    if (((uintptr_t)dev_arena) & 255) return fail(PM_E_INVAL, "arena must be 256-byte aligned");
    if (hipSetDevice(device) != hipSuccess) return fail(PM_E_DEVICE, "hipSetDevice failed");
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess) return fail(PM_E_DEVICE, "hipGetDeviceProperties failed");
    pm_ctx* c = new pm_ctx();
    c->c.device = device;
    c->c.stream = (hipStream_t)hip_stream;
    c->c.arena.base = (uintptr_t)dev_arena;
    c->c.arena.size = arena_bytes;
    c->c.arena.free_[0] = arena_bytes & ~uint64_t(255);
    c->c.num_cus = prop.multiProcessorCount;
    c->c.load_tune_file();
    noalloc_init(device);
    *out = c;
    return PM_OK;
}

pm_status pm_destroy(pm_ctx* ctx) {
    if (!ctx) return PM_E_INVAL;
    hipStreamSynchronize(ctx->c.stream);
    for (auto& g : ctx->c.graphs)
        for (auto& ls : g.second->launches) ctx->c.free_launchset(ls.second.get());
    if (ctx->c.cap_stream) hipStreamDestroy(ctx->c.cap_stream);
    delete ctx;
    return PM_OK;
}

pm_status pm_graph_load(pm_ctx* ctx, uint32_t n, const uint32_t* row_ptr, const uint32_t* col,
                        const uint8_t* labels, uint32_t* out_graph_id) {
    if (!ctx) return fail(PM_E_INVAL, "null ctx");
    try {
        return ctx->c.graph_load(n, row_ptr, col, labels, out_graph_id);
    } catch (const std::exception& e) {
        return fail(PM_E_NOMEM, std::string("host allocation failed: ") + e.what());
    }
}

pm_status pm_graph_unload(pm_ctx* ctx, uint32_t gid) {
    if (!ctx) return fail(PM_E_INVAL, "null ctx");
    return ctx->c.graph_unload(gid);
}

pm_status pm_graph_stats(pm_ctx* ctx, uint32_t gid, pm_graph_info* out) {
    if (!ctx || !out) return fail(PM_E_INVAL, "null argument");
    std::lock_guard<std::mutex> g(ctx->c.mu);
    auto it = ctx->c.graphs.find(gid);
    if (it == ctx->c.graphs.end()) return fail(PM_E_NOTFOUND, "unknown graph id");
    const GraphRes& G = *it->second;
    out->n = G.n;
    out->m = G.m;
    out->max_degree = G.max_deg;
    out->max_out_degree = G.max_out;
    out->labeled = G.labeled;
    out->device_bytes = G.device_bytes;
    return PM_OK;
}

pm_status pm_query_footprint(pm_ctx* ctx, uint32_t gid, const pm_pattern* pats, uint32_t npat, int32_t agg,
                             int32_t morph, uint64_t* out_bytes) {
    if (!ctx || !pats || !out_bytes) return fail(PM_E_INVAL, "null argument");
    GraphRes* G;
    {
        std::lock_guard<std::mutex> g(ctx->c.mu);
        auto it = ctx->c.graphs.find(gid);
        if (it == ctx->c.graphs.end()) return fail(PM_E_NOTFOUND, "unknown graph id");
        G = it->second.get();
    }
    if (agg != PM_AGG_COUNT && agg != PM_AGG_MNI) return fail(PM_E_INVAL, "unknown aggregation");
    std::vector<Pat> ps(npat);
    for (uint32_t i = 0; i < npat; ++i) {
        std::string err;
        int rc = to_pat(pats[i], &ps[i], &err);
        if (rc) return fail(rc, err);
    }
    if (agg == PM_AGG_MNI) {
        MniPlan P;
        std::string err;
        int rc = mni_plan(ps, morph == PM_MORPH_NAIVE ? PM_MORPH_NAIVE : PM_MORPH_NONE, &P, &err);
        if (rc) return fail(rc, err);
        *out_bytes = ctx->c.mni_footprint(*G, P);
        return PM_OK;
    }
    MorphPlan mp;
    std::string err;
    int rc = morph_plan_count(ps, morph, &mp, &err, ctx->c.cost_fn(*G));
    if (rc) return fail(rc, err);
    std::vector<PlanInfo> plans;
    std::vector<Pat> closure;
    rc = ctx->c.plan_closure(*G, mp.alt, &closure, &plans);
    if (rc) return fail(rc, g_err);
    uint64_t stride;
    bool any_agg;
    *out_bytes = ctx->c.footprint(*G, plans, ctx->c.cfg_for(*G, closure), &stride, &any_agg);
    return PM_OK;
}

pm_status pm_submit(pm_ctx* ctx, uint32_t gid, const pm_pattern* pats, uint32_t npat, int32_t agg,
                    int32_t morph, uint64_t* out_ticket) {
    if (!ctx) return fail(PM_E_INVAL, "null ctx");
    try {
        return ctx->c.submit(gid, pats, npat, agg, morph, out_ticket);
    } catch (const std::exception& e) {
        return fail(PM_E_NOMEM, std::string("host allocation failed: ") + e.what());
    }
}

pm_status pm_wait(pm_ctx* ctx, uint64_t ticket, int64_t* out_values, int64_t timeout_us) {
    if (!ctx) return fail(PM_E_INVAL, "null ctx");
    return ctx->c.wait(ticket, out_values, timeout_us);
}

pm_status pm_last_query_stats(pm_ctx* ctx, pm_query_stats* out) {
    if (!ctx || !out) return fail(PM_E_INVAL, "null argument");
    *out = ctx->c.last_stats;
    return PM_OK;
}

pm_status pm_last_launch_stats(pm_ctx* ctx, pm_launch_stat* out, uint32_t cap, uint32_t* n) {
    if (!ctx || !n) return fail(PM_E_INVAL, "null argument");
    const auto& L = ctx->c.last_launches;
    *n = (uint32_t)L.size();
    if (cap < L.size() || (!out && !L.empty())) return fail(PM_E_INVAL, "capacity below the number of launches");
    for (size_t i = 0; i < L.size(); ++i) out[i] = L[i];
    return PM_OK;
}

pm_status pm_cancel(pm_ctx* ctx, uint64_t ticket) {
    if (!ctx) return fail(PM_E_INVAL, "null ctx");
    std::lock_guard<std::mutex> g(ctx->c.mu);
    auto it = ctx->c.queries.find(ticket);
    if (it == ctx->c.queries.end()) return fail(PM_E_NOTFOUND, "unknown ticket");
    Query& Q = *it->second;
    LaunchSet* ls = Q.ls ? Q.ls : Q.own.get();
    if (ls && ls->cancel_host) __atomic_store_n(ls->cancel_host, 1, __ATOMIC_SEQ_CST);
    if (Q.mni_cancel) __atomic_store_n(Q.mni_cancel, 1, __ATOMIC_SEQ_CST);
    Q.cancelled = true;
    return PM_OK;
}

pm_status pm_morph_plan(const pm_pattern* pats, uint32_t npat, int32_t agg, int32_t morph, pm_pattern* out_alt,
                        uint32_t* inout_nalt, int64_t* out_matrix) {
    if (!pats || !inout_nalt) return fail(PM_E_INVAL, "null argument");
    if (agg != PM_AGG_COUNT && agg != PM_AGG_MNI) return fail(PM_E_INVAL, "unknown aggregation");
    std::vector<Pat> ps(npat);
    for (uint32_t i = 0; i < npat; ++i) {
        std::string err;
        int rc = to_pat(pats[i], &ps[i], &err);
        if (rc) return fail(rc, err);
    }
    MorphPlan mp;
    std::string err;
    if (agg == PM_AGG_MNI) {
        // Theorem 3.2: the patterns whose domains are joined (by union) into
        // each query's domains; the matrix marks which
        MniPlan P;
        int rc = mni_plan(ps, morph == PM_MORPH_NAIVE || morph == PM_MORPH_COST ? PM_MORPH_NAIVE : PM_MORPH_NONE,
                          &P, &err);
        if (rc) return fail(rc, err);
        mp.alt = P.alt;
        mp.matrix.assign((size_t)npat * P.alt.size(), 0);
        for (uint32_t i = 0; i < npat; ++i)
            for (uint32_t j : P.qalts[i]) mp.matrix[(size_t)i * P.alt.size() + j] = 1;
    } else {
        int rc = morph_plan_count(ps, morph, &mp, &err);
        if (rc) return fail(rc, err);
    }
    uint32_t na = (uint32_t)mp.alt.size();
    if (*inout_nalt < na || !out_alt) {
        *inout_nalt = na;
        return fail(PM_E_INVAL, "out_alt capacity too small");
    }
    *inout_nalt = na;
    for (uint32_t j = 0; j < na; ++j) {
        pm_pattern& o = out_alt[j];
        o.k = (uint32_t)mp.alt[j].k;
        o.edge_mask = mp.alt[j].em;
        o.induce = mp.alt[j].vi ? PM_VERTEX_INDUCED : PM_EDGE_INDUCED;
        for (int i = 0; i < 8; ++i) o.label[i] = mp.alt[j].lab[i];
    }
    if (out_matrix)
        for (size_t i = 0; i < mp.matrix.size(); ++i) out_matrix[i] = mp.matrix[i];
    return PM_OK;
}

pm_status pm_morph_plan_costs(const pm_pattern* pats, uint32_t npat, const pm_pattern* cost_pats,
                              const double* costs, uint32_t ncost, pm_pattern* out_alt, uint32_t* inout_nalt,
                              int64_t* out_matrix) {
    if (!pats || !inout_nalt || (ncost && (!cost_pats || !costs))) return fail(PM_E_INVAL, "null argument");
    std::vector<Pat> ps(npat), cp(ncost);
    for (uint32_t i = 0; i < npat; ++i) {
        std::string err;
        int rc = to_pat(pats[i], &ps[i], &err);
        if (rc) return fail(rc, err);
    }
    for (uint32_t i = 0; i < ncost; ++i) {
        std::string err;
        int rc = to_pat(cost_pats[i], &cp[i], &err);
        if (rc) return fail(rc, err);
        cp[i] = canonical(cp[i]);
    }
    // patterns without a listed cost are never worth matching
    auto cost = [&](const Pat& q) {
        const Pat c = canonical(q);
        for (uint32_t i = 0; i < ncost; ++i)
            if (cp[i] == c) return costs[i];
        return 1e30;
    };
    MorphPlan mp;
    std::string err;
    int rc = morph_plan_mixed(ps, cost, &mp, &err);
    if (rc) return fail(rc, err);
    const uint32_t na = (uint32_t)mp.alt.size();
    if (*inout_nalt < na || !out_alt) {
        *inout_nalt = na;
        return fail(PM_E_INVAL, "out_alt capacity too small");
    }
    *inout_nalt = na;
    for (uint32_t j = 0; j < na; ++j) {
        pm_pattern& o = out_alt[j];
        o.k = (uint32_t)mp.alt[j].k;
        o.edge_mask = mp.alt[j].em;
        o.induce = mp.alt[j].vi ? PM_VERTEX_INDUCED : PM_EDGE_INDUCED;
        for (int i = 0; i < 8; ++i) o.label[i] = mp.alt[j].lab[i];
    }
    if (out_matrix)
        for (size_t i = 0; i < mp.matrix.size(); ++i) out_matrix[i] = mp.matrix[i];
    return PM_OK;
}

const char* pm_last_error(void) { return g_err.c_str(); }

const char* pm_status_str(pm_status s) {
    switch (s) {
        case PM_OK: return "PM_OK";
        case PM_E_INVAL: return "PM_E_INVAL";
        case PM_E_NOMEM: return "PM_E_NOMEM";
        case PM_E_OVERFLOW: return "PM_E_OVERFLOW";
        case PM_E_UNSUPPORTED: return "PM_E_UNSUPPORTED";
        case PM_E_DEVICE: return "PM_E_DEVICE";
        case PM_E_BUSY: return "PM_E_BUSY";
        case PM_E_TIMEOUT: return "PM_E_TIMEOUT";
        case PM_E_CANCELLED: return "PM_E_CANCELLED";
        case PM_E_NOTFOUND: return "PM_E_NOTFOUND";
        default: return "PM_E_UNKNOWN";
    }
}

pm_status pm_set_option(pm_ctx* ctx, const char* key, int64_t value) {
    if (!ctx || !key) return fail(PM_E_INVAL, "null argument");
    std::string k(key);
    Ctx_& c = ctx->c;
    if (k == "count_bytes") c.count_bytes = value != 0;
    else if (k == "blocks_per_cu" && value >= 1 && value <= 64) c.blocks_per_cu = (int)value;
    else if (k == "item_budget" && value >= 1) {
        c.item_budget = (uint64_t)value;
        c.items_set = true;
    } else if (k == "item_split" && value >= 16) {
        c.item_split = (uint32_t)value;
        c.items_set = true;
    }
    else if (k == "agg_waves" && value >= 1) c.agg_waves_opt = (uint64_t)value;
    else if (k == "agg_split" && value >= 64 && value <= 0x7fffffff) c.agg_split = (uint32_t)value;
    else if (k == "heavy_roots" && (value == 0 || value == 1)) c.heavy_roots_opt = value != 0;
    else if (k == "heavy_min_mass" && value >= 1) c.heavy_min_mass = (uint64_t)value;
    else if (k == "clique_kernel" && (value == 0 || value == 1)) c.clique_opt = value != 0;
    else if (k == "edge_support" && (value == 0 || value == 1)) c.support_opt = value != 0;
    else if (k == "heavy_span_shift" && value >= 0 && value <= 32) c.heavy_span_shift = (uint32_t)value;
    else if (k == "hipgraph") c.use_graphs = value != 0;
    else if (k == "window_counters" && (value == 16 || value == 32)) c.window_wide = value == 32;
    else if (k == "launch_events" && (value == 0 || value == 1)) c.launch_events = value != 0;
    else if (k == "fork_launches" && (value == 0 || value == 1)) c.fork_launches = value != 0;
    else if (k == "hub_bitmaps" && (value == 0 || value == 1)) c.hub_bitmaps_opt = value != 0;
    else return fail(PM_E_INVAL, "unknown option or value out of range: " + k);
    return PM_OK;
}

pm_status pm_plan_describe(pm_ctx* ctx, uint32_t gid, const pm_pattern* pat, char* buf, uint64_t cap) {
    if (!ctx || !pat || !buf || !cap) return fail(PM_E_INVAL, "null argument");
    GraphRes* G;
    {
        std::lock_guard<std::mutex> g(ctx->c.mu);
        auto it = ctx->c.graphs.find(gid);
        if (it == ctx->c.graphs.end()) return fail(PM_E_NOTFOUND, "unknown graph id");
        G = it->second.get();
    }
    Pat p;
    std::string err;
    int rc = to_pat(*pat, &p, &err);
    if (rc) return fail(rc, err);
    int prc;
    const PlanInfo& pi = ctx->c.plan_for(*G, p, &prc);
    if (prc) return prc;
    std::string s = pi.describe();
    snprintf(buf, cap, "%s", s.c_str());
    return PM_OK;
}

pm_status pm_serve(pm_ctx* ctx, const pm_serve_request* reqs, uint32_t nreq, const pm_serve_config* cfg,
                   pm_serve_result* out_results, pm_serve_stats* out_stats) {
    if (!ctx) return fail(PM_E_INVAL, "null ctx");
    try {
        return ctx->c.serve(reqs, nreq, cfg, out_results, out_stats);
    } catch (const std::exception& e) {
        return fail(PM_E_NOMEM, std::string("host allocation failed: ") + e.what());
    }
}

pm_status pm_autotune(pm_ctx* ctx, uint32_t gid, const pm_pattern* pats, uint32_t npat, int32_t morph,
                      int64_t* out_cfg, double* out_ms) {
    if (!ctx || !pats || npat == 0) return fail(PM_E_INVAL, "null argument");
    try {
        return ctx->c.autotune(gid, pats, npat, morph, out_cfg, out_ms);
    } catch (const std::exception& e) {
        return fail(PM_E_NOMEM, std::string("host allocation failed: ") + e.what());
    }
}

// ---- labeled 3-edge FSM: dense slot order --------------------------------
// [triangles: sorted label triples] [3-edge paths: label 4-tuples up to
// reversal, the lexicographically smaller orientation] [3-stars: centre
// label, sorted leaf triple]; each block in lexicographic order.
static uint64_t fsm_tri(uint32_t L) { return (uint64_t)L * (L + 1) * (L + 2) / 6; }
static uint64_t fsm_p4(uint32_t L) { return ((uint64_t)L * L * L * L + (uint64_t)L * L) / 2; }

struct FsmTables {
    uint32_t L = 0;
    std::vector<int32_t> tricode, p4code, s3code;
    std::vector<std::array<int, 5>> slots;  // kind (0 tri, 1 path, 2 star), labels
};

static void fsm_tables(uint32_t L, FsmTables* t) {
    t->L = L;
    t->tricode.assign((size_t)L * L * L, -1);
    t->p4code.assign((size_t)L * L * L * L, -1);
    t->s3code.assign((size_t)L * L * L * L, -1);
    t->slots.clear();
    for (uint32_t a = 0; a < L; ++a)
        for (uint32_t b = a; b < L; ++b)
            for (uint32_t c = b; c < L; ++c) {
                t->tricode[(a * L + b) * L + c] = (int32_t)t->slots.size();
                t->slots.push_back({0, (int)a, (int)b, (int)c, -1});
            }
    for (uint32_t a = 0; a < L; ++a)
        for (uint32_t b = 0; b < L; ++b)
            for (uint32_t c = 0; c < L; ++c)
                for (uint32_t d = 0; d < L; ++d) {
                    std::array<uint32_t, 4> f{a, b, c, d}, r{d, c, b, a};
                    if (r < f) continue;  // not canonical
                    int32_t slot = (int32_t)t->slots.size();
                    t->slots.push_back({1, (int)a, (int)b, (int)c, (int)d});
                    int pal = (f == r) ? 1 : 0;
                    t->p4code[((a * L + b) * L + c) * L + d] = slot << 2 | pal;
                    t->p4code[((d * L + c) * L + b) * L + a] = slot << 2 | (pal ? 0 : 2) | pal;
                }
    for (uint32_t c = 0; c < L; ++c)
        for (uint32_t x = 0; x < L; ++x)
            for (uint32_t y = x; y < L; ++y)
                for (uint32_t z = y; z < L; ++z) {
                    t->s3code[((c * L + x) * L + y) * L + z] = (int32_t)t->slots.size();
                    t->slots.push_back({2, (int)c, (int)x, (int)y, (int)z});
                }
}

uint64_t pm_fsm_num_slots(uint32_t num_labels) {
    if (num_labels == 0 || num_labels > (uint32_t)FSM_LMAX) return 0;
    return fsm_tri(num_labels) + fsm_p4(num_labels) + (uint64_t)num_labels * fsm_tri(num_labels);
}

pm_status pm_fsm_slot(uint32_t num_labels, uint64_t slot, pm_pattern* out) {
    if (!out || num_labels == 0 || num_labels > (uint32_t)FSM_LMAX) return fail(PM_E_INVAL, "bad label count");
    if (slot >= pm_fsm_num_slots(num_labels)) return fail(PM_E_INVAL, "slot out of range");
    // the slot table of each label count is built once per process
    static std::mutex mu;
    static std::map<uint32_t, std::unique_ptr<FsmTables>> cache;
    const FsmTables* t;
    {
        std::lock_guard<std::mutex> g(mu);
        auto& e = cache[num_labels];
        if (!e) {
            e = std::make_unique<FsmTables>();
            fsm_tables(num_labels, e.get());
        }
        t = e.get();
    }
    const auto& s = t->slots[slot];
    for (int i = 0; i < 8; ++i) out->label[i] = -1;
    out->induce = PM_EDGE_INDUCED;
    if (s[0] == 0) {  // triangle 0-1-2
        out->k = 3;
        out->edge_mask = 0x7;
        for (int i = 0; i < 3; ++i) out->label[i] = s[1 + i];
    } else if (s[0] == 1) {  // path 0-1-2-3: edges (0,1) (1,2) (2,3)
        out->k = 4;
        out->edge_mask = (1u << pair_bit(0, 1)) | (1u << pair_bit(1, 2)) | (1u << pair_bit(2, 3));
        for (int i = 0; i < 4; ++i) out->label[i] = s[1 + i];
    } else {  // star centred at 0
        out->k = 4;
        out->edge_mask = (1u << pair_bit(0, 1)) | (1u << pair_bit(0, 2)) | (1u << pair_bit(0, 3));
        for (int i = 0; i < 4; ++i) out->label[i] = s[1 + i];
    }
    return PM_OK;
}

// Morphed FSM (Theorem 3.2): every slot's edge-induced pattern takes its
// domains as unions over its vertex-induced superpatterns' domains, through
// the MNI search kernels, in batches of slots whose bitmaps fit a quarter of
// the free arena.
static pm_status fsm_morphed(Ctx_& c, GraphRes& G, const FsmTables& T, uint32_t L, int64_t threshold,
                             int64_t* out_support, uint8_t* out_frequent,
                             std::chrono::steady_clock::time_point t0) {
    const uint64_t nslots = T.slots.size();
    const uint64_t per_task = 4ull * ((G.n + 31) / 32);
    const uint64_t budget = std::max<uint64_t>(c.arena.largest_free() / 4, 64ull << 20);
    // a slot needs at most 8 superpatterns x 4 columns of searches
    const uint64_t batch = std::max<uint64_t>(1, budget / (32 * per_task + 4096));
    float kms = 0;
    uint32_t launches = 0;
    for (uint64_t s0 = 0; s0 < nslots; s0 += batch) {
        const uint64_t s1 = std::min<uint64_t>(nslots, s0 + batch);
        std::vector<Pat> ps;
        for (uint64_t s = s0; s < s1; ++s) {
            pm_pattern q;
            pm_fsm_slot(L, s, &q);
            Pat p;
            std::string err;
            to_pat(q, &p, &err);
            ps.push_back(p);
        }
        MniPlan P;
        std::string err;
        int rc = mni_plan(ps, PM_MORPH_NAIVE, &P, &err);
        if (rc) return fail(rc, err);
        std::vector<int64_t> sup;
        hipEvent_t e0 = nullptr, e1 = nullptr;
        hipEventCreate(&e0);
        hipEventCreate(&e1);
        hipEventRecord(e0, c.stream);
        rc = c.run_mni_sync(G, P, &sup);
        hipEventRecord(e1, c.stream);
        hipEventSynchronize(e1);
        float ms = 0;
        hipEventElapsedTime(&ms, e0, e1);
        hipEventDestroy(e0);
        hipEventDestroy(e1);
        if (rc) return rc;
        kms += ms;
        launches += 2;
        for (uint64_t s = s0; s < s1; ++s) {
            out_support[s] = sup[s - s0];
            if (out_frequent) out_frequent[s] = sup[s - s0] >= threshold ? 1 : 0;
        }
    }
    pm_query_stats st{};
    st.kernel_ms = kms;
    st.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st.launches = launches;
    st.num_alt = (uint32_t)nslots;
    c.last_stats = st;
    return PM_OK;
}

pm_status pm_fsm(pm_ctx* ctx, uint32_t gid, uint32_t num_labels, int64_t threshold, int32_t morph,
                 int64_t* out_support, uint8_t* out_frequent, uint64_t nslots) {
    if (!ctx || !out_support) return fail(PM_E_INVAL, "null argument");
    if (num_labels == 0 || num_labels > (uint32_t)FSM_LMAX)
        return fail(PM_E_UNSUPPORTED, "pm_fsm supports 1..16 labels");
    if (nslots != pm_fsm_num_slots(num_labels)) return fail(PM_E_INVAL, "nslots must equal pm_fsm_num_slots");
    if (morph != PM_MORPH_NONE && morph != PM_MORPH_NAIVE && morph != PM_MORPH_COST)
        return fail(PM_E_INVAL, "unknown morph mode");
    Ctx_& c = ctx->c;
    GraphRes* G;
    {
        std::lock_guard<std::mutex> g(c.mu);
        auto it = c.graphs.find(gid);
        if (it == c.graphs.end()) return fail(PM_E_NOTFOUND, "unknown graph id");
        G = it->second.get();
    }
    if (!G->labeled) return fail(PM_E_INVAL, "pm_fsm needs a labeled graph");
    if (G->max_label >= num_labels) return fail(PM_E_INVAL, "graph label outside 0..num_labels-1");
    auto t0 = std::chrono::steady_clock::now();
    FsmTables T;
    fsm_tables(num_labels, &T);
    if (morph == PM_MORPH_NAIVE) return fsm_morphed(c, *G, T, num_labels, threshold, out_support, out_frequent, t0);
    const uint64_t n = G->n;
    const int grid = std::max(1, c.num_cus * 4);
    const uint64_t threads = (uint64_t)grid * 256;
    const uint64_t LL = (uint64_t)FSM_LMAX * FSM_LMAX;
    uint64_t sz_hist = n * FSM_LMAX * 4, sz_pres = n * 3 * 4, sz_b = n * LL, sz_bm = n * FSM_LMAX * 4;
    uint64_t sz_tab = 4 * (T.tricode.size() + T.p4code.size() + T.s3code.size());
    uint64_t sz_ord = 4 * n;
    uint64_t sz_tri = 32 * n;
    uint64_t sz_cnt = nslots * 16, sz_scr = threads * FSM_SCRATCH_WORDS * 8;
    uint64_t need = 0;
    for (uint64_t x : {sz_hist, sz_pres, sz_b, sz_b, sz_bm, sz_tab, sz_cnt, sz_scr, sz_ord, sz_tri})
        need += (x + 255) & ~uint64_t(255);
    uint64_t off = c.arena.alloc(need);
    if (off == UINT64_MAX) return fail(PM_E_NOMEM, "arena too small for FSM tables");
    char* base = (char*)c.dptr(off);
    uint64_t o = 0;
    auto carve = [&](uint64_t bytes) {
        char* p = base + o;
        o += (bytes + 255) & ~uint64_t(255);
        return p;
    };
    FsmArgs a;
    a.rp = (const uint32_t*)c.dptr(G->off_rp);
    a.col = (const uint32_t*)c.dptr(G->off_col);
    a.lab = (const uint8_t*)c.dptr(G->off_lab);
    a.n = G->n;
    a.L = (int)num_labels;
    a.hist = (uint32_t*)carve(sz_hist);
    a.pres = (uint32_t*)carve(sz_pres);
    a.bcnt = (uint8_t*)carve(sz_b);
    a.bfrag = (uint8_t*)carve(sz_b);
    a.bmask = (uint32_t*)carve(sz_bm);
    char* tab = carve(sz_tab);
    a.tricode = (const int32_t*)tab;
    a.p4code = a.tricode + T.tricode.size();
    a.s3code = a.p4code + T.p4code.size();
    a.counts = (uint32_t*)carve(sz_cnt);
    a.scratch = (uint64_t*)carve(sz_scr);
    uint32_t* ord = (uint32_t*)carve(sz_ord);
    a.order = ord;
    a.tri = (unsigned long long*)carve(sz_tri);
    a.split = (const uint32_t*)c.dptr(G->off_split);
    // ids ascend with degree: the hubs are a suffix of the id range
    a.hub0 = (uint32_t)n;
    while (a.hub0 > 0 && G->host_rp[a.hub0] - G->host_rp[a.hub0 - 1] >= FSM_HUB) --a.hub0;
    std::vector<int32_t> tabs;
    tabs.insert(tabs.end(), T.tricode.begin(), T.tricode.end());
    tabs.insert(tabs.end(), T.p4code.begin(), T.p4code.end());
    tabs.insert(tabs.end(), T.s3code.begin(), T.s3code.end());
    int rc = PM_OK;
    std::vector<uint32_t> counts(nslots * 4);
    hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    do {
        if (hipMemcpyAsync(tab, tabs.data(), 4 * tabs.size(), hipMemcpyHostToDevice, c.stream) != hipSuccess ||
            hipMemcpyAsync(ord, G->label_order.data(), sz_ord, hipMemcpyHostToDevice, c.stream) != hipSuccess ||
            launch_zero(a.counts, nslots * 4, c.stream)) {
            rc = fail(PM_E_DEVICE, "FSM setup failed");
            break;
        }
        for (auto& e : ev) hipEventCreate(&e);
        if (launch_fsm(a, grid, c.stream, ev)) {
            rc = fail(PM_E_DEVICE, "FSM kernel launch failed");
            break;
        }
        if (hipMemcpyAsync(counts.data(), a.counts, sz_cnt, hipMemcpyDeviceToHost, c.stream) != hipSuccess) {
            rc = fail(PM_E_DEVICE, "FSM copy-back failed");
            break;
        }
        hipError_t se = hipStreamSynchronize(c.stream);
        if (se != hipSuccess) {
            rc = fail(PM_E_DEVICE, std::string("FSM kernels failed: ") + hipGetErrorString(se));
            break;
        }
    } while (0);
    float kms = 0;
    c.last_launches.clear();
    if (rc == PM_OK && ev[0] && ev[5]) {
        hipEventElapsedTime(&kms, ev[0], ev[5]);
        // algorithmic bytes per launch: every array a kernel reads or writes,
        // with the fixed-size per-vertex records of a neighbour counted once
        // per adjacency entry that reaches them (m2 = adjacency entries)
        const uint64_t m2 = G->host_rp[n];
        // the vertices below and from a.hub0 (fsm_main and fsm_hub split them)
        const uint64_t nl = a.hub0, nh = n - a.hub0, ml = G->host_rp[a.hub0], mh = m2 - ml;
        auto main_bytes = [](uint64_t nv, uint64_t me) {
            return nv * (4 + 8 + 1 + 4 * FSM_LMAX + 12 + 32) + me * (2 * (4 + 1 + 12) + 4 * FSM_LMAX);
        };
        const uint64_t per[5] = {
            // hist: row offsets, lists, neighbour labels; writes histogram,
            // presence masks and the cleared triangle masks
            n * (8 + 4 * FSM_LMAX + 12 + 32) + m2 * (4 + 1),
            // tri: out-lists streamed against the root's hashed out-list,
            // corner label pairs written
            n * (8 + 4 + 32) + m2 * (4 + 1),
            // btab: per vertex b, its neighbours' histograms and masks; writes
            // b's (lc, ld) masks, counts and witness counts
            n * (8 + 4 * FSM_LMAX + FSM_LMAX * FSM_LMAX * 2) + m2 * (4 + 1 + 4 * FSM_LMAX + 12),
            // main (and hub, over their own vertices): per vertex its
            // records; per adjacency entry the neighbour's label and presence
            // masks in two passes and its (lc, ld) mask row in the path-end pass
            main_bytes(nl, ml), main_bytes(nh, mh)};
        static const char* names[5] = {"fsm_hist", "fsm_tri", "fsm_btab", "fsm_main", "fsm_hub"};
        for (int i = 0; i < 5; ++i) {
            pm_launch_stat ls_{};
            snprintf(ls_.kernel, sizeof(ls_.kernel), "%s", names[i]);
            ls_.alg_bytes = per[i];
            float ms = 0;
            hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
            ls_.ms = ms;
            c.last_launches.push_back(ls_);
        }
    }
    for (auto& e : ev)
        if (e) hipEventDestroy(e);
    c.arena.release(off);
    if (rc) return rc;
    // support = smallest domain over the distinct (non-automorphic) columns
    for (uint64_t s = 0; s < nslots; ++s) {
        const auto& sl = T.slots[s];
        const uint32_t* cc = &counts[s * 4];
        uint32_t sup;
        if (sl[0] == 0) {
            sup = cc[0];
            if (sl[2] != sl[1]) sup = std::min(sup, cc[1]);
            if (sl[3] != sl[2]) sup = std::min(sup, cc[2]);
        } else if (sl[0] == 1) {
            bool pal = sl[1] == sl[4] && sl[2] == sl[3];
            sup = std::min(cc[0], cc[1]);
            if (!pal) sup = std::min(sup, std::min(cc[2], cc[3]));
        } else {
            sup = std::min(cc[0], cc[1]);
            if (sl[3] != sl[2]) sup = std::min(sup, cc[2]);
            if (sl[4] != sl[3]) sup = std::min(sup, cc[3]);
        }
        out_support[s] = sup;
        if (out_frequent) out_frequent[s] = (int64_t)sup >= threshold ? 1 : 0;
    }
    pm_query_stats st{};
    st.kernel_ms = kms;
    st.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    st.launches = a.hub0 < n ? 5 : 4;
    st.num_alt = (uint32_t)nslots;
    c.last_stats = st;
    return PM_OK;
}

}  // extern "C"
