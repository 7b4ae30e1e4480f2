// Serving loop: continuous batching of pattern-set queries over resident
// graphs (host side of pm_serve).
//
// One host thread runs the loop.  Each iteration (1) makes visible the
// requests whose scheduled arrival has passed, (2) retires finished slots
// (event query), converting the batch's closure counts into every request's
// values with that request's own morph plan, and (3) admits new batches.
// Every request is planned once when it arrives (morph plan and compiled
// plans of its alternatives), which gives its estimated kernel work (the
// planner's cost model).  Admission is cheapest first: the pending request
// of least estimated work heads a batch, joined by other pending requests
// on the same graph whose estimate is at most four times the head's (or
// than SMALL_WORK), up to max_batch, so a light request never waits inside
// a heavy batch.  The
// batch is admitted when a slot is free and its footprint fits the
// remaining byte budget.  With a deadline, a batch that timed out teaches
// the loop the estimated work of its costliest request, per graph and
// largest pattern size (the cost model ranks plans within such a class far
// better than across them): a later request of that class estimated at that
// much or more is shed at once (PM_E_TIMEOUT, counted in `shed`) instead of
// holding a slot until the deadline, once the class has timed out twice and
// unless a request of that class at least as costly has completed in time (a
// cheap batch can time out behind heavy neighbours on the device); one in
// SHED_PROBE of the requests it would shed is admitted anyway.
// Every slot owns a HIP stream (default priority), dense two-hop counter
// arrays and edge-support counters, so batches in different slots run
// concurrently on the device without sharing mutable memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <thread>

#include <cstdio>

#include "runtime.hpp"

namespace pm {

namespace {

struct Batch {
    std::vector<uint32_t> reqs;
    std::vector<MorphPlan> mps;       // per request
    std::vector<Pat> closure;
    std::vector<PlanInfo> plans;
    LaunchSet ls;
    uint64_t bytes = 0;
    double admitted = 0;
    double cost = 0;                  // estimated kernel work of its requests
    bool cancelled = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    uint64_t agg_off = UINT64_MAX, agg_touch_off = UINT64_MAX;
    uint64_t sup_off = UINT64_MAX;   // edge supports for the triangle-count closed forms
    uint64_t* host = nullptr;     // pinned result words, reused by every batch
    int* cancel_host = nullptr;   // pinned coherent cancel flag
    int* cancel_dev = nullptr;
    hipEvent_t done = nullptr;
    void* stage = nullptr;        // pinned plan staging
    std::unique_ptr<Batch> batch;
};

constexpr uint64_t SLOT_STAGE_BYTES = 1024 * sizeof(DPlan);

constexpr uint64_t SLOT_HOST_WORDS = 2 * 1024 + 8;

// estimated work below which requests count as equally cheap for batching
constexpr double SMALL_WORK = 1e6;

// one in this many requests that shedding would end is admitted instead
constexpr uint32_t SHED_PROBE = 16;

using Clock = std::chrono::steady_clock;

// closure counts -> per-request values and statuses: a request fails (with
// PM_E_OVERFLOW, say) only when a count it needs does
void batch_values(const Batch& B, std::vector<std::vector<int64_t>>* out, std::vector<int>* status,
                  std::vector<std::string>* errs) {
    std::vector<__int128> cnt;
    std::vector<int> st;
    std::vector<std::string> cerr;
    closure_counts(B.closure, B.plans, B.ls.host, &cnt, &st, &cerr);
    out->assign(B.reqs.size(), {});
    status->assign(B.reqs.size(), PM_OK);
    errs->assign(B.reqs.size(), std::string());
    for (size_t r = 0; r < B.reqs.size(); ++r) {
        const MorphPlan& mp = B.mps[r];
        std::vector<int64_t> alt(mp.alt.size());
        for (size_t j = 0; j < alt.size() && !(*status)[r]; ++j) {
            size_t i = std::find(B.closure.begin(), B.closure.end(), mp.alt[j]) - B.closure.begin();
            if (i >= cnt.size()) {
                (*status)[r] = PM_E_DEVICE;
                (*errs)[r] = "internal: alternative pattern missing from the batch";
            } else if (st[i]) {
                (*status)[r] = st[i];
                (*errs)[r] = cerr[i];
            } else {
                alt[j] = (int64_t)cnt[i];
            }
        }
        if ((*status)[r]) continue;
        size_t npat = mp.alt.empty() ? 0 : mp.matrix.size() / mp.alt.size();
        (*status)[r] = unmorph(mp, npat, alt, &(*out)[r], &(*errs)[r]);
    }
}

}  // namespace

int Ctx_::serve(const pm_serve_request* reqs, uint32_t nreq, const pm_serve_config* cfg, pm_serve_result* res,
                pm_serve_stats* stats) {
    if (!reqs || !cfg || !res || nreq == 0) return fail(PM_E_INVAL, "null argument");
    if (cfg->max_slots < 1 || cfg->max_batch < 1) return fail(PM_E_INVAL, "max_slots and max_batch must be >= 1");
    HIPCHK(hipSetDevice(device));
    // validate requests and resolve graphs
    uint32_t maxn = 0;
    uint64_t maxm = 0;
    std::vector<GraphRes*> gr(nreq, nullptr);
    std::vector<std::vector<Pat>> pats(nreq);
    for (uint32_t i = 0; i < nreq; ++i) {
        memset(&res[i], 0, sizeof(res[i]));
        const pm_serve_request& q = reqs[i];
        if (q.npat < 1 || q.npat > PM_SERVE_MAX_PATTERNS) return fail(PM_E_INVAL, "request npat out of range");
        if (i && q.arrival_s < reqs[i - 1].arrival_s) return fail(PM_E_INVAL, "arrivals must be non-decreasing");
        auto it = graphs.find(q.graph_id);
        if (it == graphs.end()) return fail(PM_E_NOTFOUND, "unknown graph id in request");
        gr[i] = it->second.get();
        maxn = std::max(maxn, gr[i]->n);
        maxm = std::max<uint64_t>(maxm, gr[i]->m);
        pats[i].resize(q.npat);
        for (uint32_t k = 0; k < q.npat; ++k) {
            std::string err;
            int rc = to_pat(q.pats[k], &pats[i][k], &err);
            if (rc) {
                res[i].status = rc;
                break;
            }
            for (int v = 0; v < pats[i][k].k; ++v)
                if (pats[i][k].lab[v] >= 0 && !gr[i]->labeled) res[i].status = PM_E_INVAL;
        }
    }
    // work items of every graph built up front (their upload synchronises)
    for (uint32_t i = 0; i < nreq; ++i) {
        ItemSet* is;
        int irc = get_items(*gr[i], default_cfg(), &is);
        if (irc) return irc;
    }
    // slots: stream + two-hop counter arrays sized for the largest graph
    const uint64_t slot_agg_waves = 64;
    std::vector<Slot> slots(cfg->max_slots);
    int rc = PM_OK;
    bool serve_tri = clique_opt && support_opt;
    for (Slot& s : slots) {
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess) {
            rc = fail(PM_E_DEVICE, "stream creation failed");
            break;
        }
        uint64_t need = slot_agg_waves * (uint64_t)maxn * 4;
        s.agg_off = arena.alloc(need);
        s.agg_touch_off = arena.alloc(need);
        if (s.agg_off == UINT64_MAX || s.agg_touch_off == UINT64_MAX) {
            rc = fail(PM_E_NOMEM, "arena too small for the serving slots");
            break;
        }
        if (launch_zero((uint32_t*)dptr(s.agg_off), need / 4, s.stream)) {
            rc = fail(PM_E_DEVICE, "zero-fill failed");
            break;
        }
        // each slot its own edge supports, so that batches on one graph run
        // side by side (every replay clears the words it uses first); with
        // no room for them the slots plan without the closed forms
        if (serve_tri) {
            s.sup_off = arena.alloc(4 * std::max<uint64_t>(1, 2 * maxm));
            if (s.sup_off == UINT64_MAX) serve_tri = false;
        }
        if (hipHostMalloc((void**)&s.host, 8 * SLOT_HOST_WORDS, hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc((void**)&s.cancel_host, 64, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess ||
            hipHostGetDevicePointer((void**)&s.cancel_dev, s.cancel_host, 0) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(&s.stage, SLOT_STAGE_BYTES, hipHostMallocDefault) != hipSuccess) {
            rc = fail(PM_E_DEVICE, "slot setup failed");
            break;
        }
        HIPCHK(hipStreamSynchronize(s.stream));
    }
    auto cleanup = [&]() {
        for (Slot& s : slots) {
            if (s.batch) {
                if (s.cancel_host) __atomic_store_n(s.cancel_host, 1, __ATOMIC_SEQ_CST);
                hipStreamSynchronize(s.stream);
                free_launchset(&s.batch->ls);
            }
        }
        for (Slot& s : slots) {
            if (s.agg_off != UINT64_MAX) arena.release(s.agg_off);
            if (s.agg_touch_off != UINT64_MAX) arena.release(s.agg_touch_off);
            if (s.sup_off != UINT64_MAX) arena.release(s.sup_off);
            if (s.done) hipEventDestroy(s.done);
            if (s.host) hipHostFree(s.host);
            if (s.cancel_host) hipHostFree(s.cancel_host);
            if (s.stage) hipHostFree(s.stage);
            if (s.stream) hipStreamDestroy(s.stream);
        }
    };
    if (rc) {
        cleanup();
        return rc;
    }
    if (!serve_tri)
        for (Slot& s : slots)
            if (s.sup_off != UINT64_MAX) {
                arena.release(s.sup_off);
                s.sup_off = UINT64_MAX;
            }

    std::deque<uint32_t> pending;
    // per request: its morph plan and estimated kernel work (planned once)
    std::vector<MorphPlan> rmp(nreq);
    std::vector<double> rcost(nreq, -1.0);
    // per (graph, largest pattern size): least estimated work of a request
    // that headed a timed-out batch's work (its costliest request)
    std::vector<int> rk(nreq, 0);
    for (uint32_t i = 0; i < nreq; ++i)
        for (const Pat& q : pats[i]) rk[i] = std::max(rk[i], (int)q.k);
    std::map<std::pair<const GraphRes*, int>, double> timeout_cost;
    // per class: the largest estimated work of a request that completed in
    // time; a request no costlier than that is never shed (a timeout of a
    // cheap batch behind heavy neighbours on the device says little about it)
    std::map<std::pair<const GraphRes*, int>, double> done_cost;
    // per class: timeouts learnt (shedding starts at the second), and the
    // requests shedding has passed over; every SHED_PROBE-th of those is
    // admitted anyway (and never shed later), so that a class whose first
    // timeouts were bad luck can show otherwise
    std::map<std::pair<const GraphRes*, int>, int> timeouts_n;
    std::map<std::pair<const GraphRes*, int>, uint32_t> shed_seen;
    std::vector<uint8_t> probe(nreq, 0);
    uint64_t shed = 0;
    uint32_t next = 0, finished = 0;
    uint64_t used = 0, batches = 0;
    double inflight_sum = 0;
    uint64_t admissions = 0;
    const Clock::time_point t0 = Clock::now();
    auto now_s = [&]() { return std::chrono::duration<double>(Clock::now() - t0).count(); };
    // requests already failed at validation
    for (uint32_t i = 0; i < nreq; ++i)
        if (res[i].status) {
            res[i].latency_s = 0;
            ++finished;
        }
    double last_done = 0;
    while (finished < nreq && rc == PM_OK) {
        const double t = now_s();
        while (next < nreq && reqs[next].arrival_s <= t) {
            const uint32_t r = next++;
            if (res[r].status) continue;
            std::string err;
            GraphRes& G = *gr[r];
            int prc = morph_plan_count(pats[r], reqs[r].morph, &rmp[r], &err, cost_fn(G, serve_tri));
            std::vector<Pat> cl;
            std::vector<PlanInfo> pl;
            if (!prc) prc = plan_closure(G, rmp[r].alt, &cl, &pl, serve_tri);
            if (prc == PM_E_NOMEM || prc == PM_E_DEVICE) {
                rc = prc;
                break;
            }
            if (prc) {
                res[r].status = prc;
                res[r].latency_s = now_s() - reqs[r].arrival_s;
                ++finished;
                continue;
            }
            double c = 0;
            for (const PlanInfo& p : pl) c += p.est_cost;
            rcost[r] = c;
            pending.push_back(r);
        }
        if (rc) break;
        bool progressed = false;
        // retire finished batches; cancel those past the deadline
        for (Slot& s : slots) {
            if (!s.batch) continue;
            hipError_t e = hipEventQuery(s.done);
            if (e == hipErrorNotReady) {
                if (cfg->deadline_s > 0 && !s.batch->cancelled && t - s.batch->admitted > cfg->deadline_s) {
                    __atomic_store_n(s.batch->ls.cancel_host, 1, __ATOMIC_SEQ_CST);
                    s.batch->cancelled = true;
                }
                continue;
            }
            Batch& B = *s.batch;
            const double tdone = now_s();
            std::vector<std::vector<int64_t>> vals;
            std::vector<int> rst;
            std::vector<std::string> rerr;
            const int brc = e == hipSuccess ? (B.cancelled ? PM_E_TIMEOUT : PM_OK) : PM_E_DEVICE;
            if (brc == PM_E_TIMEOUT) {
                // the costliest request of the batch takes the blame
                uint32_t worst = B.reqs[0];
                for (uint32_t r : B.reqs)
                    if (rcost[r] > rcost[worst]) worst = r;
                // unless a request of its class at least as costly has
                // completed in time: then the device was busy with others
                auto key = std::make_pair((const GraphRes*)gr[worst], rk[worst]);
                auto dc = done_cost.find(key);
                if (dc == done_cost.end() || rcost[worst] > dc->second) {
                    auto it = timeout_cost.find(key);
                    if (it == timeout_cost.end()) timeout_cost[key] = rcost[worst];
                    else it->second = std::min(it->second, rcost[worst]);
                    ++timeouts_n[key];
                }
            }
            if (brc == PM_OK) batch_values(B, &vals, &rst, &rerr);
            for (size_t r = 0; r < B.reqs.size(); ++r) {
                pm_serve_result& R = res[B.reqs[r]];
                R.status = brc ? brc : rst[r];
                if (R.status == PM_OK) {
                    const uint32_t q = B.reqs[r];
                    double& dc = done_cost[std::make_pair((const GraphRes*)gr[q], rk[q])];
                    dc = std::max(dc, rcost[q]);
                }
                R.latency_s = tdone - reqs[B.reqs[r]].arrival_s;
                R.service_s = tdone - B.admitted;
                R.batch_size = (uint32_t)B.reqs.size();
                if (R.status == PM_OK)
                    for (size_t k = 0; k < vals[r].size(); ++k) R.values[k] = vals[r][k];
                ++finished;
            }
            last_done = std::max(last_done, tdone);
            if (cfg->progress_every && finished / cfg->progress_every !=
                                           (finished - B.reqs.size()) / cfg->progress_every)
                fprintf(stderr, "pm_serve: %u of %u requests finished at %.2f s\n", (unsigned)finished,
                        (unsigned)nreq, tdone);
            used -= B.bytes;
            free_launchset(&B.ls);
            s.batch.reset();
            progressed = true;
            if (e != hipSuccess) {
                rc = fail(PM_E_DEVICE, std::string("serving batch failed: ") + hipGetErrorString(e));
                break;
            }
        }
        // admit batches while a slot is free and the budget allows
        while (!pending.empty() && rc == PM_OK) {
            Slot* free_slot = nullptr;
            int busy = 0;
            for (Slot& s : slots) {
                if (s.batch) ++busy;
                else if (!free_slot) free_slot = &s;
            }
            if (!free_slot) break;
            // shed what an observed timeout says cannot finish in time
            if (cfg->deadline_s > 0 && !timeout_cost.empty()) {
                bool any = false;
                for (auto it = pending.begin(); it != pending.end();) {
                    const auto key = std::make_pair((const GraphRes*)gr[*it], rk[*it]);
                    auto tc = timeout_cost.find(key);
                    auto dc = done_cost.find(key);
                    bool cut = !probe[*it] && tc != timeout_cost.end() && timeouts_n[key] >= 2 &&
                               rcost[*it] >= tc->second && (dc == done_cost.end() || rcost[*it] > dc->second);
                    if (cut && ++shed_seen[key] % SHED_PROBE == 0) {
                        probe[*it] = 1;
                        cut = false;
                    }
                    if (cut) {
                        res[*it].status = PM_E_TIMEOUT;
                        res[*it].latency_s = now_s() - reqs[*it].arrival_s;
                        ++finished;
                        ++shed;
                        any = true;
                        it = pending.erase(it);
                    } else {
                        ++it;
                    }
                }
                if (any) progressed = true;
                if (pending.empty()) break;
            }
            // the cheapest pending request heads the batch (earliest first
            // among equals); others on its graph of at most four times its
            // estimated work join, cheapest first
            uint32_t head = pending.front();
            for (uint32_t r : pending)
                if (rcost[r] < rcost[head]) head = r;
            GraphRes& G = *gr[head];
            const double t_setup = now_s();
            auto B = std::make_unique<Batch>();
            B->reqs.push_back(head);
            {
                std::vector<uint32_t> cand;
                for (uint32_t r : pending)
                    if (r != head && gr[r] == &G && rcost[r] <= 4 * std::max(rcost[head], SMALL_WORK)) cand.push_back(r);
                std::stable_sort(cand.begin(), cand.end(), [&](uint32_t x, uint32_t y) { return rcost[x] < rcost[y]; });
                for (uint32_t r : cand) {
                    if (B->reqs.size() >= cfg->max_batch) break;
                    B->reqs.push_back(r);
                }
            }
            // union the requests' alternatives (morph plans made on arrival)
            std::vector<Pat> alts;
            for (uint32_t r : B->reqs) {
                B->mps.push_back(rmp[r]);
                B->cost += rcost[r];
                for (const Pat& a : rmp[r].alt)
                    if (std::find(alts.begin(), alts.end(), a) == alts.end()) alts.push_back(a);
            }
            int prc = plan_closure(G, alts, &B->closure, &B->plans, serve_tri);
            if (prc) {
                rc = prc;
                break;
            }
            LaunchCfg lc = cfg_for(G, B->closure);
            // a persistent launch holds its CUs until its queue drains: give
            // each slot a share of the GPU so batches really run side by side
            lc.grid_override = std::max(1, (int)(num_cus * 2 / cfg->max_slots));
            lc.share_div = (int)cfg->max_slots;
            uint64_t stride;
            bool any_agg;
            B->bytes = footprint(G, B->plans, lc, &stride, &any_agg, false);
            if (B->bytes > cfg->budget_bytes) {
                for (uint32_t r : B->reqs) {
                    res[r].status = PM_E_NOMEM;
                    res[r].latency_s = now_s() - reqs[r].arrival_s;
                    pending.erase(std::find(pending.begin(), pending.end(), r));
                    ++finished;
                }
                continue;
            }
            if (used + B->bytes > cfg->budget_bytes) break;  // wait for memory
            AggArrays ag;
            ag.cnt = (uint32_t*)dptr(free_slot->agg_off);
            ag.touch = (uint32_t*)dptr(free_slot->agg_touch_off);
            ag.waves = slot_agg_waves;
            ag.n = maxn;
            ag.host = free_slot->host;
            ag.host_words = SLOT_HOST_WORDS;
            ag.cancel_host = free_slot->cancel_host;
            ag.cancel_dev = free_slot->cancel_dev;
            ag.stage = free_slot->stage;
            ag.stage_bytes = SLOT_STAGE_BYTES;
            if (free_slot->sup_off != UINT64_MAX) {
                ag.support = (uint32_t*)dptr(free_slot->sup_off);
                ag.support_words = std::max<uint64_t>(1, 2 * maxm);
            }
            int mrc = make_launchset(G, B->plans, lc, &B->ls, free_slot->stream, &ag);
            if (mrc == PM_E_NOMEM) {
                free_launchset(&B->ls);
                if (busy == 0) {
                    rc = mrc;
                    break;
                }
                break;  // wait for in-flight batches to release memory
            }
            if (mrc) {
                free_launchset(&B->ls);
                rc = mrc;
                break;
            }
            if (enqueue(B->ls, free_slot->stream, false) ||
                hipEventRecord(free_slot->done, free_slot->stream) != hipSuccess) {
                free_launchset(&B->ls);
                rc = fail(PM_E_DEVICE, "serving launch failed");
                break;
            }
            const double ta = now_s();
            B->admitted = ta;
            for (uint32_t r : B->reqs) {
                res[r].queue_s = ta - reqs[r].arrival_s;
                res[r].setup_s = ta - t_setup;
                pending.erase(std::find(pending.begin(), pending.end(), r));
            }
            used += B->bytes;
            ++batches;
            inflight_sum += busy + 1;
            ++admissions;
            free_slot->batch = std::move(B);
            progressed = true;
        }
        if (!progressed) {
            // nothing to do: sleep until the next arrival or a short poll
            double wait = 50e-6;
            if (next < nreq) wait = std::min(wait, std::max(0.0, reqs[next].arrival_s - now_s()));
            if (wait > 2e-6) std::this_thread::sleep_for(std::chrono::duration<double>(wait));
        }
    }
    cleanup();
    if (rc) return rc;
    // statistics
    std::vector<double> lat;
    double total_matches = 0, setup_sum = 0, service_sum = 0;
    uint64_t failed = 0, timeouts = 0;
    for (uint32_t i = 0; i < nreq; ++i) {
        if (res[i].status) {
            ++failed;
            if (res[i].status == PM_E_TIMEOUT) ++timeouts;
            continue;
        }
        lat.push_back(res[i].latency_s);
        setup_sum += res[i].setup_s;
        service_sum += res[i].service_s;
        for (uint32_t k = 0; k < reqs[i].npat; ++k) total_matches += (double)res[i].values[k];
    }
    std::sort(lat.begin(), lat.end());
    if (stats) {
        memset(stats, 0, sizeof(*stats));
        auto rank = [&](double q) {
            if (lat.empty()) return 0.0;
            size_t k = (size_t)std::ceil(q * lat.size());
            if (k < 1) k = 1;
            return lat[std::min(k, lat.size()) - 1];
        };
        stats->p50_s = rank(0.50);
        stats->p99_s = rank(0.99);
        double sum = 0;
        for (double x : lat) sum += x;
        stats->mean_s = lat.empty() ? 0 : sum / lat.size();
        stats->max_s = lat.empty() ? 0 : lat.back();
        stats->makespan_s = last_done - reqs[0].arrival_s;
        stats->matches_per_s = stats->makespan_s > 0 ? total_matches / stats->makespan_s : 0;
        stats->mean_inflight = admissions ? inflight_sum / admissions : 0;
        stats->batches = batches;
        stats->completed = nreq - failed;
        stats->failed = failed;
        stats->timeouts = timeouts;
        stats->mean_setup_s = lat.empty() ? 0 : setup_sum / lat.size();
        stats->mean_service_s = lat.empty() ? 0 : service_sum / lat.size();
        stats->sustained_qps = stats->makespan_s > 0 ? (double)stats->completed / stats->makespan_s : 0;
        stats->shed = shed;
    }
    return PM_OK;
}

}  // namespace pm

