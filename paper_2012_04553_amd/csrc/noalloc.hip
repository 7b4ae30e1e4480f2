// Allocation-free counting: pm_count_noalloc.
//
// The same counts as pm_submit + pm_wait (COUNT aggregation), for callers
// that cannot allocate device memory.  Every device buffer the matching
// launch needs beyond the resident graph and the caller's output - the
// device plans, the 128-bit counters, the work-queue head, the root work
// items and the per-wavefront level buffers - lives in `scratch`, one
// file-scope device array of NOALLOC_BYTES per GPU, held from the library's
// load until the process ends.  Host code never passes the array's name to
// a kernel or a copy: its device address is taken once per device with
// hipGetSymbolAddress (when a context is created on that device) and only
// that address is used.
//
// Every plan of the query's closure runs in the general matching kernel
// (match_kernel), in one launch: plans that need the two-hop counter
// arrays, the root bitmaps or the bitmap-clique rows are not chosen here.
// The number of wavefronts follows from what is left of the array after
// the plans, counters and items; a query that does not fit is rejected
// with PM_E_NOMEM before anything is launched.
//
// Calls on one device share the array and keep the last call's contents;
// the counters and the queue head are cleared by a fill kernel at the start
// of every call.  Calls from this process are serialised per device; calls
// from other processes that overlap on the same GPU race.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "runtime.hpp"

namespace pm {

namespace {

constexpr uint64_t NOALLOC_BYTES = 64ull << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
constexpr uint32_t NOALLOC_MAX_PLANS = 64;

__device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

struct DevScratch {
    std::mutex mu;                 // serialises the calls of this process
    void* ptr = nullptr;           // device address of `scratch` on this device
    hipError_t status = hipErrorNotInitialized;
    bool tried = false;
};
DevScratch g_dev[NOALLOC_MAX_DEVICES];
std::mutex g_init_mu;

uint64_t round256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// The cheapest plan the general kernel runs alone (no two-hop aggregation,
// no root bitmap, no bitmap clique rows) and that needs no other pattern's
// count (no quotient rewrite), so the query's plans are its alternatives.
int general_plan(const Pat& p, const GraphStats& gs, PlanInfo* out, std::string* err) {
    std::vector<PlanInfo> all;
    int rc = candidate_plans(p, gs, &all, err);
    if (rc) return rc;
    int best = -1;
    for (size_t i = 0; i < all.size(); ++i) {
        const DPlan& d = all[i].d;
        if (d.agg_last || d.bm0 || d.local || all[i].rewrite) continue;
        if (best < 0 || all[i].est_cost < all[best].est_cost) best = (int)i;
    }
    if (best < 0) {
        *err = "no plan of this pattern runs in the general kernel";
        return PM_E_UNSUPPORTED;
    }
    *out = all[best];
    return PM_OK;
}

}  // namespace

void noalloc_init(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return;
    std::lock_guard<std::mutex> g(g_init_mu);
    DevScratch& D = g_dev[device];
    if (D.tried) return;
    D.tried = true;
    // the caller (pm_create) has made `device` current
    void* p = nullptr;
    D.status = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (D.status == hipSuccess) D.ptr = p;
}

static int count_noalloc(Ctx_& C, uint32_t gid, const pm_pattern* pats, uint32_t npat, int morph, int64_t* out) {
    if (!pats || !out || npat == 0) return fail(PM_E_INVAL, "null patterns or output");
    if (morph != PM_MORPH_NONE && morph != PM_MORPH_NAIVE && morph != PM_MORPH_COST)
        return fail(PM_E_INVAL, "unknown morph mode");
    if (C.device < 0 || C.device >= NOALLOC_MAX_DEVICES) return fail(PM_E_INVAL, "device index out of range");
    DevScratch& D = g_dev[C.device];
    if (!D.ptr)
        return fail(PM_E_DEVICE, std::string("static scratch address unavailable: ") + hipGetErrorString(D.status));
    GraphRes* G;
    {
        std::lock_guard<std::mutex> g(C.mu);
        auto it = C.graphs.find(gid);
        if (it == C.graphs.end()) return fail(PM_E_NOTFOUND, "unknown graph id");
        G = it->second.get();
    }
    std::vector<Pat> ps(npat);
    for (uint32_t i = 0; i < npat; ++i) {
        std::string err;
        int rc = to_pat(pats[i], &ps[i], &err);
        if (rc) return fail(rc, err);
        for (int v = 0; v < ps[i].k; ++v)
            if (ps[i].lab[v] >= 0 && !G->labeled) return fail(PM_E_INVAL, "labeled pattern on an unlabeled graph");
    }
    // morph plan, then one general-kernel plan per alternative pattern
    MorphPlan mp;
    std::string err;
    int rc = morph_plan_count(ps, morph, &mp, &err, C.cost_fn(*G));
    if (rc) return fail(rc, err);
    const std::vector<Pat>& closure = mp.alt;
    if (closure.size() > NOALLOC_MAX_PLANS)
        return fail(PM_E_NOMEM, "query needs " + std::to_string(closure.size()) +
                                    " plans; the static scratch holds at most " + std::to_string(NOALLOC_MAX_PLANS));
    std::vector<PlanInfo> plans;
    for (size_t i = 0; i < closure.size(); ++i) {
        PlanInfo pi;
        rc = general_plan(closure[i], G->st, &pi, &err);
        if (rc) return fail(rc, err);
        plans.push_back(pi);
    }
    const uint32_t np = (uint32_t)plans.size();
    uint64_t stride = 1;
    for (const PlanInfo& p : plans)
        for (int j = 1; j < p.d.ncore; ++j) {
            const DLevel& L = p.d.lev[j];
            const bool out_list = (L.adj & L.gt) != 0;
            stride = std::max<uint64_t>(stride, (uint64_t)(out_list ? G->max_out : G->max_deg) + 64);
        }
    stride = (stride + 63) & ~uint64_t(63);
    const LaunchCfg cfg = C.default_cfg();
    std::vector<KItem> items = build_items(G->host_rp, G->n, cfg.item_budget, cfg.item_split, 256);
    // layout: plans | counters | head + byte tally | items | level buffers
    const uint64_t o_plans = 0;
    const uint64_t o_cnt = round256(o_plans + sizeof(DPlan) * np);
    const uint64_t o_head = round256(o_cnt + 16ull * np);
    const uint64_t o_items = round256(o_head + 16);
    const uint64_t o_buf = round256(o_items + sizeof(KItem) * items.size());
    const uint64_t per_wave = (uint64_t)KMAX * stride * 4;
    const uint64_t left = o_buf < NOALLOC_BYTES ? NOALLOC_BYTES - o_buf : 0;
    const uint64_t block_waves = (uint64_t)C.block / 64;
    uint64_t waves = std::min<uint64_t>(C.waves(cfg), left / per_wave);
    waves -= waves % block_waves;
    if (waves == 0)
        return fail(PM_E_NOMEM, "the static scratch (" + std::to_string(NOALLOC_BYTES >> 20) +
                                    " MiB) cannot hold one workgroup's level buffers (" +
                                    std::to_string(block_waves * per_wave) + " bytes) after " +
                                    std::to_string(o_buf) + " bytes of plans and items");
    std::vector<DPlan> dp(np);
    for (uint32_t i = 0; i < np; ++i) dp[i] = plans[i].d;
    std::vector<uint64_t> host(2ull * np + 2, 0);

    std::lock_guard<std::mutex> dg(D.mu);
    HIPCHK(hipSetDevice(C.device));
    uint8_t* base = (uint8_t*)D.ptr;
    KArgs a{};
    a.g.rp = (const uint32_t*)C.dptr(G->off_rp);
    a.g.col = (const uint32_t*)C.dptr(G->off_col);
    a.g.split = (const uint32_t*)C.dptr(G->off_split);
    a.g.lab = G->labeled ? (const uint8_t*)C.dptr(G->off_lab) : nullptr;
    a.g.n = G->n;
    a.plans = (const DPlan*)(base + o_plans);
    a.nplans = (int32_t)np;
    a.nitems = (uint32_t)items.size();
    a.items = (const KItem*)(base + o_items);
    a.counters = (uint64_t*)(base + o_cnt);
    a.head = (uint32_t*)(base + o_head);
    a.bytes = (uint64_t*)(base + o_head + 8);
    a.scratch = (uint32_t*)(base + o_buf);
    a.buf_stride = stride;
    hipStream_t s = C.stream;
    HIPCHK(hipMemcpyAsync(base + o_plans, dp.data(), sizeof(DPlan) * np, hipMemcpyHostToDevice, s));
    if (!items.empty())
        HIPCHK(hipMemcpyAsync(base + o_items, items.data(), sizeof(KItem) * items.size(), hipMemcpyHostToDevice, s));
    // counters, head and tally start at zero on every call
    if (launch_zero((uint32_t*)(base + o_cnt), (o_items - o_cnt) / 4, s))
        return fail(PM_E_DEVICE, "zero-fill launch failed");
    if (!items.empty() && launch_match(a, (int)(waves / block_waves), C.block, false, s))
        return fail(PM_E_DEVICE, "kernel launch failed");
    HIPCHK(hipMemcpyAsync(host.data(), base + o_cnt, 16ull * np, hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));

    std::vector<__int128> cnt;
    std::vector<int> st;
    std::vector<std::string> cerr;
    closure_counts(closure, plans, host.data(), &cnt, &st, &cerr);
    for (uint32_t i = 0; i < np; ++i)
        if (st[i]) return fail(st[i], cerr[i]);
    std::vector<int64_t> alt(mp.alt.size());
    for (size_t j = 0; j < alt.size(); ++j) {
        const size_t i = std::find(closure.begin(), closure.end(), mp.alt[j]) - closure.begin();
        alt[j] = (int64_t)cnt[i];
    }
    std::vector<int64_t> res;
    rc = unmorph(mp, npat, alt, &res, &err);
    if (rc) return fail(rc, err);
    memcpy(out, res.data(), sizeof(int64_t) * npat);
    return PM_OK;
}

}  // namespace pm

extern "C" pm_status pm_count_noalloc(pm_ctx* ctx, uint32_t graph_id, const pm_pattern* pats, uint32_t npat,
                                      int32_t morph, int64_t* out_values) {
    if (!ctx) return pm::fail(PM_E_INVAL, "null context");
    return pm::count_noalloc(ctx->c, graph_id, pats, npat, morph, out_values);
}
