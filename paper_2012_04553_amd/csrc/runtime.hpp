// Host runtime state of a pm_ctx.
#pragma once
#include <hip/hip_runtime.h>

#include <chrono>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "internal.hpp"
#include "kernels.hpp"
#include "mni.hpp"

namespace pm {

extern thread_local std::string g_err;
int fail(int code, const std::string& msg);

#define HIPCHK(x)                                                                          \
    do {                                                                                   \
        hipError_t e_ = (x);                                                               \
        if (e_ != hipSuccess) return fail(PM_E_DEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

int to_pat(const pm_pattern& q, Pat* out, std::string* err);

// MNI domain searches of a query (mni_host.cpp): deduplicated column
// searches, and per query pattern one output per vertex, the union of some
// searches' bitmaps.
struct MniPlan {
    std::vector<MTask> tasks;
    std::vector<uint32_t> list;                 // search indices of the outputs
    std::vector<MOut> outs;
    std::vector<std::vector<uint32_t>> qouts;   // per query pattern: its outputs
    std::vector<Pat> alt;                       // distinct patterns searched
    std::vector<std::vector<uint32_t>> qalts;   // per query pattern: indices into alt
};
// morph: PM_MORPH_NONE (direct) or PM_MORPH_NAIVE (edge-induced patterns
// through their vertex-induced superpatterns, Theorem 3.2)
int mni_plan(const std::vector<Pat>& qs, int morph, MniPlan* out, std::string* err);

struct PlanInfo;
// Work items over the roots: consecutive roots of about `budget` adjacency
// entries (at most max_roots), roots above `split` cut into level-1 slices.
std::vector<KItem> build_items(const std::vector<uint32_t>& rp, uint32_t n, uint64_t budget, uint32_t split,
                               uint32_t max_roots);
// The allocation-free entry point's static scratch array: its device address
// is taken once per device when a context is created there.
void noalloc_init(int device);
void closure_counts(const std::vector<Pat>& closure, const std::vector<PlanInfo>& plans, const uint64_t* host,
                    std::vector<__int128>* cnt, std::vector<int>* st, std::vector<std::string>* err);

// First-fit sub-allocator over the caller's device arena (offsets).
struct Arena {
    uintptr_t base = 0;
    uint64_t size = 0;
    std::map<uint64_t, uint64_t> free_;  // offset -> bytes
    std::map<uint64_t, uint64_t> used_;
    std::mutex mu;
    uint64_t alloc(uint64_t bytes);       // UINT64_MAX when full
    void release(uint64_t off);
    uint64_t largest_free();
};

// Work items of one (root budget, hub slice) configuration, on the device.
struct ItemSet {
    uint64_t off = UINT64_MAX;
    uint32_t count = 0;
};

constexpr size_t MAX_RUNS = 32;   // launches of one launch set (byte tallies, events)

struct LaunchCfg {
    int blocks_per_cu = 4;
    uint64_t item_budget = 4096;
    uint32_t item_split = 2048;
    int grid_override = 0;   // > 0: blocks of the match launch (a GPU share)
    int share_div = 0;       // > 1: the fixed-grid LDS launches take 1/share_div of their grids
};

// Device state of one (graph, plan closure, launch configuration): plans,
// counters, queue heads, scratch, pinned result buffer, and the captured
// hipGraph that replays [zero-fill -> match launches -> copy-back].
struct LaunchSet {
    uint64_t off_mem = UINT64_MAX;
    size_t np = 0;
    DPlan* dplans = nullptr;
    uint64_t* counters = nullptr;
    uint32_t* zero_base = nullptr;   // counters + heads + bytes + root bitmaps, cleared together
    uint64_t zero_words = 0;
    uint32_t* heads = nullptr;
    uint64_t* bytes = nullptr;
    uint32_t* scratch = nullptr;
    uint64_t stride = 0;
    bool any_agg = false;
    KArgs base{};
    std::vector<std::pair<int, int>> runs;   // contiguous plan ranges, one launch each
    std::vector<int> run_agg;                // 0 plain, 1 two-hop, 2 heavy two-hop roots,
                                             // 3 edge-core light roots, 4 edge-core heavy roots,
                                             // 5 triangle-core (clique_kernel), 6 their larger roots,
                                             // 7/8 4-cliques (clique4_kernel, light/heavy roots),
                                             // 9 their larger roots, 10 edge-support plans,
                                             // 11 4-cliques (clique4_kernel, largest roots),
                                             // 12 5-cycles (cycle5_kernel), 13 per-vertex
                                             // triangle counts (vtri_kernel), 14 the
                                             // house's 4-cycle sums (house_kernel),
                                             // 15 per-triangle sums (trisup_kernel)
    const KItem* agg_items = nullptr;        // work items of the two-hop launches
    uint32_t agg_nitems = 0;
    const KItem* heavy_items = nullptr;      // heavy two-hop roots, one item each
    uint32_t heavy_nitems = 0;
    const KItem* edge_items = nullptr;       // edge-core plans: light roots
    const KItem* edge_heavy = nullptr;       //                  heavy roots, one item each
    uint32_t edge_nitems = 0, edge_nheavy = 0;
    const KItem* cq_items = nullptr;         // triangle-core plans: clique_kernel items
    const KItem* cq_big = nullptr;           //   and general-kernel items of the larger roots
    uint32_t cq_nitems = 0, cq_nbig = 0;
    const KItem* c4_light = nullptr;         // 4-clique plans: wavefront roots,
    const KItem* c4_heavy = nullptr;         //   workgroup roots,
    const KItem* c4_huge = nullptr;          //   workgroup roots above C4_HEAVY_MAX,
    const KItem* c4_big = nullptr;           //   general-kernel items of the larger roots
    uint32_t c4_nlight = 0, c4_nheavy = 0, c4_nhuge = 0, c4_nbig = 0;
    uint32_t* support = nullptr;             // edge supports (the graph's), when used
    int sup_run = -1;                        // the triangle run that fills them
    uint64_t sup_words = 0;                  // their words (2m), cleared at the head of a replay
    uint64_t* vtri = nullptr;                // per vertex: twice its triangle count (closed forms)
    bool mirror = false;                     // supports mirrored to both list ends (house plans)
    bool c4_sup = false;                     // the 4-clique launches [sup_run, c4_fill_end) fill them
    int c4_fill_end = -1;
    uint64_t* host = nullptr;                // pinned: 2*np counter words + byte tally
    uint64_t agg_w = 0;                      // wavefronts of the aggregation launches
    int* cancel_host = nullptr;              // pinned coherent flag polled by the kernel
    int* cancel_dev = nullptr;
    bool borrowed_host = false;              // host/cancel buffers owned by a serving slot
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool busy = false;
    uint64_t agg_gen = 0;                    // generation of the context's two-hop arrays it
                                             // points to (0: uses none, or a slot's own)
    LaunchCfg cfg;
};

struct GraphRes {
    uint32_t n = 0;
    uint64_t m = 0;
    bool labeled = false;
    uint32_t max_label = 0;
    uint32_t max_deg = 0, max_out = 0;
    GraphStats st;
    uint64_t off_rp = UINT64_MAX, off_col = UINT64_MAX, off_split = UINT64_MAX, off_lab = UINT64_MAX,
             off_items = UINT64_MAX;
    uint64_t off_support = UINT64_MAX;       // edge supports, u32 per adjacency entry (on first use)
    uint64_t off_cq = UINT64_MAX;            // device copies of the items below
    const KItem* d_cq = nullptr;
    const KItem* d_c4l = nullptr;
    const KItem* d_c4h = nullptr;
    const KItem* d_c4x = nullptr;
    uint64_t device_bytes = 0;
    std::vector<uint32_t> host_rp;           // degree-ordered row offsets (item building)
    std::vector<uint32_t> orig_id;           // degree-ordered id -> the caller's id
    std::vector<uint32_t> label_order;       // labeled graphs: vertices sorted by label
    std::vector<uint64_t> two_hop;           // per vertex: summed degrees of its lower neighbours
    std::vector<uint8_t> low2;               // per vertex: 1 with two or more lower neighbours
    std::vector<KItem> clique_items;         // triangle-core kernel items
    std::vector<uint32_t> clique_big;        // roots with more than CQ_SMAX out-neighbours
    std::vector<KItem> c4_light, c4_heavy, c4_huge;   // 4-clique kernel items
    std::vector<uint32_t> c4_big;            // roots with more than C4_ROOT_MAX out-neighbours
    std::map<std::pair<uint64_t, uint32_t>, ItemSet> itemsets;
    std::map<std::string, std::unique_ptr<LaunchSet>> launches;
    std::vector<std::pair<Pat, PlanInfo>> plan_cache;
    std::vector<std::pair<Pat, PlanInfo>> plan_cache_notri;   // without triangle-count closed forms
    uint64_t off_lorder = UINT64_MAX;        // label-sorted vertex order on the device (first MNI use)
    uint64_t off_hubbm = UINT64_MAX;         // membership bitmaps of the vertices hub0 .. n-1
    uint32_t hub0 = 0, hub_words = 0;
    std::vector<uint32_t> label_begin;       // labeled graphs: first position of each label in label_order
    uint64_t hash = 0;                       // FNV-1a of the degree-ordered CSR (+labels)
    int inflight = 0;
};

struct Query {
    uint32_t gid = 0;
    uint32_t npat = 0;
    MorphPlan mp;
    std::vector<Pat> closure;        // patterns matched on the device
    std::vector<PlanInfo> plans;     // one per closure entry
    LaunchSet* ls = nullptr;                 // cached launch set (busy while in flight)
    std::unique_ptr<LaunchSet> own;          // or one made for this query alone
    bool counted_bytes = false;
    bool cancelled = false;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr, ev_done = nullptr;
    pm_query_stats stats{};
    std::chrono::steady_clock::time_point t_submit;
    std::vector<hipEvent_t> run_ev;          // launch_events: one before each launch, one after the last
    std::vector<int> run_kind;               // LaunchSet::run_agg of each launch
    // MNI queries: domain searches, their arena region, pinned column sizes
    // and cancel flag
    bool mni = false;
    MniPlan mni_plan;
    uint64_t mni_off = UINT64_MAX;
    unsigned long long* mni_host = nullptr;
    int* mni_cancel = nullptr;
};

struct Ctx_ {
    int device = 0;
    hipStream_t stream = nullptr;
    Arena arena;
    int num_cus = 1;
    int blocks_per_cu = 4;
    int block = 256;
    uint64_t item_budget = 4096;
    uint32_t item_split = 2048;
    bool count_bytes = false;
    uint64_t agg_waves_opt = 2048;
    uint32_t agg_split = 256;
    bool heavy_roots_opt = true;
    uint64_t heavy_min_mass = 16384;
    bool clique_opt = true;
    uint32_t heavy_span_shift = 6;   // two-hop heavy roots: mass << shift >= id
    bool support_opt = true;
    bool window_wide = false;        // agg_window_kernel: 32-bit counters always
    bool launch_events = false;      // eager launches with an event between launches
    std::vector<pm_launch_stat> last_launches;
    bool use_graphs = true;
    hipStream_t cap_stream = nullptr;
    // captured launch sets fork the LDS-kernel launches (triangle pass and
    // edge supports; 4-cliques) onto two branches beside the general-kernel
    // launches, which share the per-wavefront buffers and stay in order
    hipStream_t branch[2] = {nullptr, nullptr};
    hipEvent_t fork_ev = nullptr, join_ev[2] = {nullptr, nullptr};
    bool fork_launches = false;      // measured slower at R-MAT 20 (127 vs 120 ms a step)
    bool hub_bitmaps_opt = true;     // probes of hub lists through the graph's membership bitmaps
    std::map<std::string, std::pair<LaunchCfg, double>> tune_cache;
    std::string tune_file;
    std::mutex mu, plan_mu;
    std::map<uint32_t, std::unique_ptr<GraphRes>> graphs;
    std::map<uint64_t, std::unique_ptr<Query>> queries;
    uint32_t next_gid = 1;
    uint64_t next_ticket = 1;
    uint64_t agg_off = UINT64_MAX, agg_touch_off = UINT64_MAX;
    // the two-hop arrays are reallocated when a graph needs more; launch
    // sets (and their captured graphs) built on older arrays are rebuilt,
    // and older arrays are released once nothing in flight uses them
    uint64_t agg_gen = 1;
    std::vector<uint64_t> agg_retired;
    bool ctx_agg_busy();
    void release_retired_agg();
    uint32_t agg_n = 0;
    uint64_t agg_w = 0;
    pm_query_stats last_stats{};
    std::vector<int64_t> last_alt;

    void* dptr(uint64_t off) const { return (void*)(arena.base + off); }
    int grid_blocks(const LaunchCfg& c) const {
        return c.grid_override > 0 ? c.grid_override : num_cus * c.blocks_per_cu;
    }
    uint64_t waves(const LaunchCfg& c) const { return (uint64_t)grid_blocks(c) * (block / 64); }
    // clique_kernel: 40 KB of LDS a workgroup, four resident a CU; with
    // edge supports 41 KB (counters in the hash slots), three, or 65 KB on
    // graphs above CQ_PACK_MAX vertices, two
    int clique_blocks(bool sup, uint32_t n) const { return num_cus * (!sup ? 4 : (n <= CQ_PACK_MAX ? 3 : 2)); }
    int support_blocks() const { return num_cus * 8; }
    // clique4_kernel: wavefront roots 14 KB of LDS a workgroup, eight
    // resident a CU; workgroup roots 44 KB, three; the largest 152 KB, one
    int clique4_blocks(int mode) const { return num_cus * (mode == 0 ? 8 : (mode == 1 ? 3 : 1)); }
    // wavefronts of the two-hop aggregation launches on an n-vertex graph:
    // each holds two dense u32[n] arrays, so their number follows from a
    // memory budget (a quarter of the arena, at most 8 GiB)
    uint64_t agg_waves(const LaunchCfg& c, uint32_t n) const {
        const uint64_t budget = std::min<uint64_t>(8ull << 30, arena.size / 4);
        const uint64_t by_mem = std::max<uint64_t>(64, budget / (8ull * std::max<uint32_t>(n, 1)));
        return std::min<uint64_t>(std::min<uint64_t>(agg_waves_opt, waves(c)), by_mem);
    }
    LaunchCfg default_cfg() const { return LaunchCfg{blocks_per_cu, item_budget, item_split}; }
    LaunchCfg start_cfg(const std::vector<Pat>& closure) const;
    bool items_set = false;          // item_budget / item_split set through pm_set_option
    std::string closure_key(const GraphRes& G, const std::vector<Pat>& closure) const;
    LaunchCfg cfg_for(const GraphRes& G, const std::vector<Pat>& closure) const;
    int get_items(GraphRes& G, const LaunchCfg& c, ItemSet** out);
    // agg: per-wave dense counter arrays (aggcnt, aggtouch, waves) for the
    // aggregation launches, or null to use the context's shared ones
    struct AggArrays {
        uint32_t* cnt = nullptr;
        uint32_t* touch = nullptr;
        uint64_t waves = 0;
        uint32_t n = 0;
        // optional pinned buffers reused across launch sets (pinned host
        // allocation and release synchronise the device)
        uint64_t* host = nullptr;
        uint64_t host_words = 0;
        int* cancel_host = nullptr;
        int* cancel_dev = nullptr;
        void* stage = nullptr;         // pinned staging for the plan upload
        uint64_t stage_bytes = 0;
        uint32_t* support = nullptr;   // the slot's edge supports (u32 per adjacency entry)
        uint64_t support_words = 0;
    };
    int make_launchset(GraphRes& G, const std::vector<PlanInfo>& plans, const LaunchCfg& c, LaunchSet* ls,
                       hipStream_t s = nullptr, const AggArrays* agg = nullptr);
    std::function<double(const Pat&)> cost_fn(GraphRes& G, bool tri_ok = true);
    int serve(const pm_serve_request* reqs, uint32_t nreq, const pm_serve_config* cfg, pm_serve_result* res,
              pm_serve_stats* stats);
    void free_launchset(LaunchSet* ls);
    int enqueue(LaunchSet& ls, hipStream_t s, bool bytes_pass, hipEvent_t* run_ev = nullptr, bool fork = false);
    int run_eager_ms(GraphRes& G, const std::vector<PlanInfo>& plans, const LaunchCfg& c, double* ms);
    int autotune(uint32_t gid, const pm_pattern* pats, uint32_t npat, int morph, int64_t* out_cfg, double* out_ms);
    void load_tune_file();
    int graph_load(uint32_t n, const uint32_t* rp, const uint32_t* col, const uint8_t* labels, uint32_t* gid);
    int graph_unload(uint32_t gid);
    // tri_ok: the launch may use the graph's per-edge triangle counts (not in
    // serving slots, which share the graph); the closed forms over them are
    // chosen only when the options and the graph allow it too (tri_forms)
    const PlanInfo& plan_for(GraphRes& G, const Pat& p, int* rc, bool tri_ok = true);
    bool tri_forms(const GraphRes& G) const;
    // alternative patterns plus every sub-pattern their quotient plans need,
    // aggregation plans last (they run in a launch of their own)
    int plan_closure(GraphRes& G, const std::vector<Pat>& alt, std::vector<Pat>* closure,
                     std::vector<PlanInfo>* plans, bool tri_ok = true);
    uint64_t footprint(const GraphRes& G, const std::vector<PlanInfo>& plans, const LaunchCfg& c,
                       uint64_t* stride, bool* any_agg, bool heavy_ok = true) const;
    std::vector<uint32_t> heavy_roots(const GraphRes& G, const std::vector<PlanInfo>& plans,
                                      uint32_t* p_agg) const;
    std::vector<uint32_t> edge_heavy_roots(const GraphRes& G, const std::vector<PlanInfo>& plans) const;
    int ensure_agg(uint32_t n, const LaunchCfg& c);
    uint64_t bitmap_words(const GraphRes& G, const std::vector<PlanInfo>& plans) const;
    bool use_clique(const GraphRes& G, const std::vector<PlanInfo>& plans) const;
    std::vector<KItem> clique_big_items(const GraphRes& G, const LaunchCfg& cfg) const;
    bool use_clique4(const GraphRes& G, const std::vector<PlanInfo>& plans) const;
    bool use_support(const GraphRes& G, const std::vector<PlanInfo>& plans) const;
    int ensure_support(GraphRes& G);
    std::vector<KItem> clique4_big_items(const GraphRes& G, const LaunchCfg& cfg) const;
    int submit(uint32_t gid, const pm_pattern* pats, uint32_t npat, int agg, int morph, uint64_t* ticket);
    // MNI queries (mni_host.cpp)
    uint64_t mni_footprint(const GraphRes& G, const MniPlan& P) const;
    int ensure_label_order(GraphRes& G);
    int enqueue_mni(GraphRes& G, const MniPlan& P, uint64_t base, unsigned long long* host, const int* cancel,
                    hipStream_t s);
    int run_mni_sync(GraphRes& G, const MniPlan& P, std::vector<int64_t>* sup);
    int submit_mni(GraphRes& G, uint32_t gid, const std::vector<Pat>& ps, int morph, uint64_t* ticket);
    int finish_mni(Query& Q, int64_t* out);
    int fsm_levelwise(GraphRes& G, uint32_t L, uint32_t max_edges, int64_t threshold, int morph,
                      std::vector<std::pair<Pat, int64_t>>* out);
    int list_matches(GraphRes& G, const Pat& p, int morph, uint32_t* out, uint64_t cap, uint64_t* count);
    int launch(GraphRes& G, Query& Q);
    int evict_idle();
    int wait(uint64_t ticket, int64_t* out, int64_t timeout_us);
};

}  // namespace pm

struct pm_ctx {
    pm::Ctx_ c;
};
