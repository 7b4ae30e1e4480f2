/*
 * pm.h -- C-ABI of the MI355X pattern-morphing subgraph-counting engine.
 *
 * The operations follow the paper's statement of the problem (Pattern
 * Morphing for Efficient Graph Mining, Jamshidi & Vora):
 *   - a data graph is a simple undirected graph, optionally vertex-labeled
 *     (Preliminaries, "Graph Isomorphism");
 *   - a query is a set of patterns, each vertex- or edge-induced and labeled
 *     or not (Preliminaries, "Pattern Semantics");
 *   - the result is one aggregation value per pattern: the number of
 *     distinct matched subgraphs (Motif Counting) or the minimum-node-image
 *     support (Frequent Subgraph Mining) (Preliminaries, "Graph Mining
 *     Applications");
 *   - morphing rewrites the query into an alternative pattern set and
 *     converts the results back (Section 3.2, Theorems 3.1/3.2,
 *     Corollary 3.1; Section 4.1 "external module" (a) and (b)).
 *
 * Conventions.
 *   - Every function returns pm_status: 0 = PM_OK, negative = error.  No C++
 *     exception crosses this boundary.  On error the thread-local message is
 *     available from pm_last_error().
 *   - "device pointer" = memory of the HIP device the context was created
 *     on; "host pointer" = ordinary process memory.  Every pointer argument
 *     is a host pointer unless stated otherwise.
 *   - Vertex ids are uint32.  Counts are exact int64; any value (or any
 *     intermediate of the morph conversion) outside int64 is reported as
 *     PM_E_OVERFLOW rather than wrapped.
 *   - A pattern edge between pattern vertices i < j is bit j*(j-1)/2 + i of
 *     pm_pattern.edge_mask.
 */
#ifndef PM_H
#define PM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pm_ctx pm_ctx;
typedef int32_t pm_status;

enum {
    PM_OK = 0,
    PM_E_INVAL = -1,        /* malformed argument, graph or pattern          */
    PM_E_NOMEM = -2,        /* the caller's arena cannot hold the request    */
    PM_E_OVERFLOW = -3,     /* a count or conversion left int64               */
    PM_E_UNSUPPORTED = -4,  /* e.g. disconnected pattern, k outside 2..5      */
    PM_E_DEVICE = -5,       /* a HIP runtime call failed                      */
    PM_E_BUSY = -6,         /* graph unload while queries are in flight       */
    PM_E_TIMEOUT = -7,      /* pm_wait timed out (the query keeps running)    */
    PM_E_CANCELLED = -8,    /* the query was cancelled by pm_cancel           */
    PM_E_NOTFOUND = -9      /* unknown graph id or ticket                     */
};

/* Induced-ness of a pattern (Preliminaries, "Pattern Semantics"): a
 * vertex-induced pattern carries an anti-edge on every non-adjacent pair,
 * an edge-induced pattern carries none. */
enum { PM_EDGE_INDUCED = 0, PM_VERTEX_INDUCED = 1 };

/* Aggregation (Section 3.2.3): COUNT = number of distinct matched subgraphs
 * (#matches / #label-preserving automorphisms); MNI = minimum node image
 * support (smallest per-pattern-vertex domain, Preliminaries, FSM). */
enum { PM_AGG_COUNT = 0, PM_AGG_MNI = 1 };

/* Morph mode: NONE matches the query patterns as given ("No PMR",
 * Section 4.2); NAIVE matches the alternative set of Section 4.2's "Naive
 * PMR": vertex-induced patterns become their same-size edge-induced
 * superpatterns plus the clique, converted back by Corollary 3.1; COST
 * ("Cost-Based PMR", Section 4.1) picks the cheapest alternative set under
 * the engine's cost model (plan work estimated from the graph's degree
 * statistics): over the queries' same-size superpatterns each is matched
 * vertex-induced, edge-induced or not at all, so vertex- and edge-induced
 * alternatives mix (Table 4: an edge-induced 4-cycle may become the
 * vertex-induced 4-cycle, the edge-induced diamond and the 4-clique), see
 * pm_morph_plan_costs.  pm_morph_plan has no graph and treats COST as
 * NAIVE. */
enum { PM_MORPH_NONE = 0, PM_MORPH_NAIVE = 1, PM_MORPH_COST = 2 };

typedef struct {
    uint32_t k;          /* number of pattern vertices, 2..5                 */
    uint32_t edge_mask;  /* bit j*(j-1)/2+i set = edge (i, j); connected     */
    uint32_t induce;     /* PM_EDGE_INDUCED or PM_VERTEX_INDUCED             */
    int32_t label[8];    /* label of each pattern vertex, -1 = any label     */
} pm_pattern;

typedef struct {
    uint32_t n;             /* vertices                                      */
    uint64_t m;             /* undirected edges                              */
    uint32_t max_degree;
    uint32_t max_out_degree; /* in the degree-ordered orientation            */
    uint32_t labeled;       /* 1 when labels were given                      */
    uint64_t device_bytes;  /* arena bytes held by the resident graph        */
} pm_graph_info;

typedef struct {
    double plan_ms;          /* host planning (morph + plan compile)         */
    double kernel_ms;        /* device time of the matching launch(es)       */
    double total_ms;         /* submit -> results ready, incl. unmorph       */
    uint64_t alg_bytes;      /* algorithmic bytes of the executed plans      */
    uint64_t work_items;     /* work items processed                         */
    uint32_t num_alt;        /* patterns actually matched                    */
    uint32_t launches;       /* kernel launches of the query                 */
} pm_query_stats;

/* Create a context on HIP device `device`.  `dev_arena` (device pointer,
 * `arena_bytes` long, 256-byte aligned) is memory the caller owns (e.g. a
 * torch tensor); every device allocation of the engine is carved from it,
 * so it must outlive the context.  `hip_stream` is a hipStream_t owned by
 * the caller on which all work is issued (NULL = the null stream).
 * Errors: PM_E_INVAL (null out, misaligned arena), PM_E_DEVICE. */
pm_status pm_create(void* dev_arena, uint64_t arena_bytes, void* hip_stream,
                    int device, pm_ctx** out);

/* Waits for in-flight work, then frees host state.  The arena and stream
 * stay the caller's. */
pm_status pm_destroy(pm_ctx* ctx);

/* Load a graph: `row_ptr` (n+1 entries) and `col` (row_ptr[n] entries) are
 * a host CSR of a simple undirected graph: each row strictly ascending, no
 * self-loops, symmetric.  `labels` (n bytes) may be NULL.  The arrays are
 * copied: the engine validates them, relabels vertices by (degree, id)
 * rank (degree-ordered CSR), and keeps the result resident in the arena.
 * Vertex ids in results (none for COUNT/MNI) refer to the caller's ids.
 * Errors: PM_E_INVAL (asymmetric, unsorted, self-loop, duplicate, id out of
 * range, row_ptr[n] >= 2^32), PM_E_NOMEM, PM_E_DEVICE. */
pm_status pm_graph_load(pm_ctx* ctx, uint32_t n, const uint32_t* row_ptr,
                        const uint32_t* col, const uint8_t* labels,
                        uint32_t* out_graph_id);

/* Release a graph.  PM_E_BUSY while queries on it are in flight. */
pm_status pm_graph_unload(pm_ctx* ctx, uint32_t graph_id);

pm_status pm_graph_stats(pm_ctx* ctx, uint32_t graph_id, pm_graph_info* out);

/* Arena bytes a query would need beyond the resident graph. */
pm_status pm_query_footprint(pm_ctx* ctx, uint32_t graph_id,
                             const pm_pattern* pats, uint32_t npat, int32_t agg,
                             int32_t morph, uint64_t* out_bytes);

/* Submit a query (asynchronous).  `pats` is copied.  The ticket identifies
 * it for pm_wait / pm_cancel.
 *   agg = PM_AGG_COUNT: one count per pattern; `morph` as documented above.
 *   agg = PM_AGG_MNI: one MNI support per pattern (Preliminaries, FSM): the
 *     smallest over the pattern's vertices of the number of data vertices
 *     some match maps that vertex to.  PM_MORPH_NAIVE takes an edge-induced
 *     pattern's domains as unions of the domains of its vertex-induced
 *     superpatterns on the same vertices, each read through the column
 *     permutation (Theorem 3.2); vertex-induced patterns and cliques are
 *     searched directly (a union has no inverse).  PM_MORPH_NONE and
 *     PM_MORPH_COST search every pattern directly (with existence searches
 *     the morphed route never does less work).  Patterns have 2..5 vertices.
 * Errors: PM_E_INVAL, PM_E_UNSUPPORTED, PM_E_NOTFOUND (graph), PM_E_NOMEM
 * (footprint exceeds the free arena). */
pm_status pm_submit(pm_ctx* ctx, uint32_t graph_id, const pm_pattern* pats,
                    uint32_t npat, int32_t agg, int32_t morph,
                    uint64_t* out_ticket);

/* Wait for a query; on PM_OK writes npat int64 values (counts or MNI
 * supports, in the order submitted) to `out_values` (host) and releases the
 * ticket.  timeout_us < 0 waits forever.  PM_E_TIMEOUT leaves the ticket
 * valid.  PM_E_OVERFLOW / PM_E_CANCELLED release it. */
pm_status pm_wait(pm_ctx* ctx, uint64_t ticket, int64_t* out_values,
                  int64_t timeout_us);

/* Optional statistics of the last pm_wait'ed query (call before the next). */
pm_status pm_last_query_stats(pm_ctx* ctx, pm_query_stats* out);

/* Per-launch statistics of the last pm_wait'ed counting query: one entry per
 * kernel launch of its launch set, in launch order.  alg_bytes is the
 * launch's algorithmic bytes when option "count_bytes" was set (else 0);
 * ms its device time between HIP events recorded on the context's stream
 * before and after it when option "launch_events" was set (else 0).
 * Errors: PM_E_INVAL when `cap` is below *n (then only *n is written). */
typedef struct {
    char kernel[32];         /* kernel name                                  */
    uint64_t alg_bytes;
    double ms;
} pm_launch_stat;
pm_status pm_last_launch_stats(pm_ctx* ctx, pm_launch_stat* out, uint32_t cap, uint32_t* n);

/* Request cancellation: the query's kernels stop taking work items (a
 * host-visible flag polled once per item) and the later pm_wait returns
 * PM_E_CANCELLED.  PM_E_NOTFOUND for an unknown ticket. */
pm_status pm_cancel(pm_ctx* ctx, uint64_t ticket);

/* Host-only morph planning (Section 4.1 (a); Section 4.2 "Naive PMR").
 * For the `npat` query patterns (all with the same k, unlabeled or
 * labeled), writes the alternative patterns to `out_alt` (capacity
 * *inout_nalt, updated to the count used) and the integer conversion
 * matrix to `out_matrix` (row-major npat x nalt, host): value(query i) =
 * sum_j out_matrix[i*nalt + j] * count(alt j).  For PM_AGG_MNI the
 * alternatives are the patterns whose domains pm_submit searches (with
 * PM_MORPH_NAIVE or PM_MORPH_COST: each edge-induced query's vertex-induced
 * superpatterns on the same vertices, Theorem 3.2; otherwise the queries
 * themselves), and out_matrix[i*nalt + j] is 1 when alternative j's domains
 * enter query i's union, else 0.  Errors: PM_E_INVAL (capacity),
 * PM_E_UNSUPPORTED. */
pm_status pm_morph_plan(const pm_pattern* pats, uint32_t npat, int32_t agg,
                        int32_t morph, pm_pattern* out_alt, uint32_t* inout_nalt,
                        int64_t* out_matrix);

/* Host-only cost-based morph planning with caller-given costs (Section 4.1's
 * optimizer; the mixed alternative sets of Table 4).  Over the queries'
 * same-size superpatterns, each pattern is matched vertex-induced,
 * edge-induced or not at all, minimising the summed cost, such that every
 * query's count follows (Theorem 3.1, Corollary 3.1): an edge-induced
 * query may become its vertex-induced form plus edge-induced
 * superpatterns, a vertex-induced one its edge-induced superpatterns, or a
 * query may stay as given.  `cost_pats[i]` (its `induce` says how it would
 * be matched) costs `costs[i]`; unlisted patterns are never chosen unless
 * no set avoids them.  pm_submit with PM_MORPH_COST runs the same search
 * with costs from the engine's plan cost model on the graph.  Output as
 * pm_morph_plan (COUNT).  Errors: PM_E_INVAL, PM_E_UNSUPPORTED. */
pm_status pm_morph_plan_costs(const pm_pattern* pats, uint32_t npat,
                              const pm_pattern* cost_pats, const double* costs,
                              uint32_t ncost, pm_pattern* out_alt,
                              uint32_t* inout_nalt, int64_t* out_matrix);

/* Listing (enumeration aggregation; Section 3.2.2, match conversion):
 * every distinct matched subgraph of `pat` on the graph, once, as the
 * caller's ids of the images of pattern vertices 0..k-1 (one match per
 * subgraph: the smallest of its images under the pattern's automorphisms).
 * With PM_MORPH_NAIVE an edge-induced pattern is listed through its
 * vertex-induced patterns p + S on the same vertices (S: non-adjacent pairs
 * of p whose images are adjacent), each of whose matches converts to a
 * match of p by the identity map of p's vertices; otherwise (and for
 * vertex-induced patterns and cliques) the pattern is listed directly.
 * Synchronous.  Writes min(*out_count, capacity) tuples of k uint32 to
 * out_matches (host, capacity * k entries) and the number of subgraphs to
 * *out_count.  Order is unspecified.  Errors: PM_E_INVAL,
 * PM_E_UNSUPPORTED, PM_E_NOTFOUND, PM_E_NOMEM (also when the tuples to
 * write do not fit half the free arena; *out_count is still set). */
pm_status pm_list(pm_ctx* ctx, uint32_t graph_id, const pm_pattern* pat, int32_t morph,
                  uint32_t* out_matches, uint64_t capacity, uint64_t* out_count);

/* Labeled 3-edge frequent subgraph mining with MNI support (Preliminaries,
 * FSM).  Computes the support of every edge-induced labeled pattern with 3
 * edges (the triangle, the 3-edge path and the 3-star) over the graph's
 * `num_labels` labels, in the dense slot order documented with
 * pm_fsm_slot(); `out_support` (host, nslots int64) receives the supports;
 * `out_frequent` (host, nslots bytes, may be NULL) receives support >=
 * threshold.  morph = PM_MORPH_NONE (and PM_MORPH_COST) computes the
 * supports from the edge-induced patterns directly, with membership tests
 * over per-vertex neighbour-label tables; PM_MORPH_NAIVE computes every
 * slot's domains as unions of its vertex-induced superpatterns' domains
 * (Theorem 3.2) with the existence searches of pm_submit's MNI route, in
 * batches that fit the arena.  Errors: PM_E_INVAL (unlabeled graph, a label
 * >= num_labels, nslots != pm_fsm_num_slots), PM_E_NOMEM (arena). */
pm_status pm_fsm(pm_ctx* ctx, uint32_t graph_id, uint32_t num_labels,
                 int64_t threshold, int32_t morph, int64_t* out_support,
                 uint8_t* out_frequent, uint64_t nslots);

/* Level-wise frequent subgraph mining (Preliminaries, FSM) with MNI
 * support.  Level 1 holds every labeled edge (labels 0..num_labels-1);
 * level e+1 extends each frequent pattern of level e by one edge (between
 * two of its vertices, or to a new vertex of any label, at most 5 vertices)
 * and keeps a candidate only when each of its connected subpatterns with
 * one edge fewer is frequent (MNI support is anti-monotone), before its
 * support is computed with pm_submit's MNI route (`morph` as there).
 * Frequent = support >= threshold.  Writes every frequent edge-induced
 * pattern with 1..max_edges edges, in canonical form, level by level, to
 * out_pats / out_support (host, `capacity` entries) and their number to
 * *out_count.  Errors: PM_E_INVAL (unlabeled graph, label >= num_labels,
 * max_edges outside 1..10, capacity below *out_count: nothing is written
 * but *out_count), PM_E_NOMEM. */
pm_status pm_fsm_levelwise(pm_ctx* ctx, uint32_t graph_id, uint32_t num_labels,
                           uint32_t max_edges, int64_t threshold, int32_t morph,
                           pm_pattern* out_pats, int64_t* out_support,
                           uint64_t capacity, uint64_t* out_count);

/* Number of FSM slots for `num_labels` labels, and the pattern of slot s. */
uint64_t pm_fsm_num_slots(uint32_t num_labels);
pm_status pm_fsm_slot(uint32_t num_labels, uint64_t slot, pm_pattern* out);

/* Engine options (tuning knobs of the implementation, not of the method):
 *   "count_bytes"   0/1: before each query run an untimed pass of the same
 *                   kernel that tallies algorithmic bytes (see
 *                   pm_last_query_stats);
 *   "blocks_per_cu" persistent blocks per compute unit (1..64);
 *   "item_budget"   adjacency entries per root-range work item (>= 1,
 *                   default 4096; untuned sets with 5-vertex patterns use
 *                   256 unless this or "item_split" was set);
 *   "item_split"    level-1 slice length for high-degree roots (>= 16,
 *                   default 2048; 64 for untuned 5-vertex sets, as above);
 *   "agg_waves"     upper bound on the wavefronts of two-hop aggregation
 *                   launches (>= 1, default 2048); each such wave holds
 *                   8 bytes per vertex, and their total is also kept within
 *                   a quarter of the arena (at most 8 GiB);
 *   "agg_split"     target-range slices of a high-degree root in two-hop
 *                   aggregation launches: one slice per this many
 *                   adjacency entries (>= 64, default 256);
 *   "heavy_roots"   0/1 (default 1): roots with a large two-hop mass (the
 *                   summed degrees of their lower neighbours) of two-hop
 *                   plans that aggregate at their first level, and of
 *                   edge-core plans whose terms intersect N(v0) and N(v1),
 *                   are counted by workgroups sweeping LDS windows;
 *   "heavy_min_mass" two-hop mass from which a root counts as heavy
 *                   (>= 1, default 16384);
 *   "heavy_span_shift" a two-hop root also needs its mass times
 *                   2^shift to reach its id, which bounds the id range its
 *                   window sweep covers (0..32, default 6);
 *   "clique_kernel" 0/1 (default 1): triangle-core and ordered 4-clique
 *                   plans run in the LDS hash kernels (roots up to 1024
 *                   and 512 out-neighbours; larger ones in the general
 *                   kernel), edge-core plans with cheap terms per edge;
 *   "edge_support"  0/1 (default 1): edge-core plans whose set-size term
 *                   is the whole common neighbourhood (the diamond) take
 *                   it from per-edge triangle counts, and eight unlabeled
 *                   edge-induced patterns (the triangle, the tailed
 *                   triangle, the bowtie, the triangle with a two-edge
 *                   path, the house, the diamond with a pendant at a tip,
 *                   the fan of three triangles, the 4-clique with an ear)
 *                   are counted in closed form from them instead of being
 *                   enumerated.  The counts are filled by the 4-clique or
 *                   the triangle launches (needs "clique_kernel" and no
 *                   root above 1024 out-neighbours; one u32 per adjacency
 *                   entry of the graph, allocated on first use and cleared
 *                   at the head of every replay);
 *   "hipgraph"      0/1 (default 1): capture a query set's launches in a
 *                   hipGraph on first use and replay it afterwards;
 *   "window_counters" 16 or 32 (default 16): counter width of the two-hop
 *                   window kernel when every degree fits 16 bits (32 is
 *                   always used otherwise);
 *   "launch_events" 0/1 (default 0): launch eagerly (no hipGraph) with a HIP
 *                   event between launches, for per-launch device times in
 *                   pm_last_launch_stats;
 *   "fork_launches" 0/1 (default 0): captured launch sets run the triangle
 *                   and edge-support launches and the 4-clique launches on
 *                   two more branches of the hipGraph, beside the general
 *                   kernel's launches (not for sets with a house plan or
 *                   whose 4-clique launches fill the edge supports);
 *   "hub_bitmaps"   0/1 (default 1): probes of the adjacency lists of the
 *                   highest-degree vertices (64 neighbours or more, up to
 *                   512 MiB of n-bit bitmaps built at graph load) answer
 *                   from the bitmaps instead of by binary search.
 * Errors: PM_E_INVAL for an unknown key or a value out of range. */
pm_status pm_set_option(pm_ctx* ctx, const char* key, int64_t value);

/* Batching: tune the launch of one query set on one graph.  Times the
 * whole multi-pattern launch under a coordinate search over blocks per
 * compute unit {1,2,4,8}, root budget per work item {256,1K,4K,16K,64K}
 * adjacency entries and hub slice {32,64,512,2K,8K}, and keeps the fastest for
 * that (graph, matched pattern set): later pm_submit calls of the same set
 * use it.  Results are cached per context and, when the environment
 * variable PM_AUTOTUNE_CACHE names a file, appended there and reloaded by
 * later contexts.  `out_cfg` (3 int64, may be NULL) receives the chosen
 * values, `out_ms` (may be NULL) the tuned kernel time in milliseconds.
 * Errors: as pm_submit. */
pm_status pm_autotune(pm_ctx* ctx, uint32_t graph_id, const pm_pattern* pats,
                      uint32_t npat, int32_t morph, int64_t* out_cfg, double* out_ms);

/* ---- serving ----------------------------------------------------------
 * A request loop over resident graphs (continuous batching).  pm_serve
 * replays a request trace in real time: request i becomes visible at
 * arrival_s seconds after the call starts, and is planned then (morph plan
 * and compiled plans, which give its estimated kernel work by the cost
 * model of §4.1).  Pending requests are admitted cheapest first into up to
 * max_slots slots, each with its own HIP stream: the pending request of
 * least estimated work and the requests pending on the same graph whose
 * estimate is at most four times its own (up to max_batch) form one batch
 * whose patterns are matched in a single multi-pattern launch; a batch is
 * admitted only while the arena bytes of all in-flight batches stay within
 * budget_bytes.  Batches run concurrently on the device, and a finished
 * slot is refilled at once.  With a deadline, once batches whose costliest
 * requests share a graph and largest pattern size have timed out twice,
 * pending requests of that class estimated at the least of those requests'
 * work or more end at once with PM_E_TIMEOUT (stats.shed) instead of
 * occupying a slot until the deadline -- unless a request of that class
 * estimated at their work or more has completed in time (a timeout of a
 * request no costlier than one that completed teaches nothing: the device
 * was busy); one in 16 of the requests so ended is admitted instead.
 * Each slot's launches take a 1/max_slots share of the grids (the general
 * kernel's and those sized by the CU count), so a cheap batch is not held
 * behind persistent workgroups of heavy ones.
 * Each slot holds its own edge-support counters (a u32 per adjacency entry
 * of the largest graph served) for the closed forms of "edge_support"; with
 * no arena room for them the slots plan without those forms.
 * Latency of a request = completion time - scheduled arrival (queueing
 * included).  Not to be called concurrently with other calls on the same
 * context.  Results are identical to pm_submit/pm_wait of the same
 * request alone. */
#define PM_SERVE_MAX_PATTERNS 8
typedef struct {
    double arrival_s;       /* scheduled arrival, seconds from the start  */
    uint32_t graph_id;
    uint32_t npat;          /* 1 .. PM_SERVE_MAX_PATTERNS                 */
    int32_t morph;          /* PM_MORPH_*                                 */
    pm_pattern pats[PM_SERVE_MAX_PATTERNS];
} pm_serve_request;

typedef struct {
    double latency_s;       /* completion - scheduled arrival             */
    double queue_s;         /* admission - scheduled arrival              */
    int32_t status;         /* PM_OK or the error of this request         */
    uint32_t batch_size;    /* requests in the batch it ran in            */
    int64_t values[PM_SERVE_MAX_PATTERNS];
    double setup_s;         /* host time to plan its batch and build the
                               launch set, before the batch was enqueued  */
    double service_s;       /* completion - admission (the batch on the GPU) */
} pm_serve_result;

typedef struct {
    uint32_t max_slots;     /* batches in flight (>= 1)                   */
    uint32_t max_batch;     /* requests merged into one batch (>= 1)      */
    uint64_t budget_bytes;  /* arena bytes for in-flight batches          */
    double deadline_s;      /* > 0: a batch still running this long after
                               admission is cancelled and its requests end
                               with PM_E_TIMEOUT; 0 = no deadline          */
    uint32_t progress_every; /* > 0: a line on stderr each time this many
                               more requests have finished; 0 = silent     */
} pm_serve_config;

typedef struct {
    double p50_s, p99_s, mean_s, max_s;  /* latency, nearest rank        */
    double makespan_s;                   /* first arrival to last done    */
    double matches_per_s;                /* sum of all values / makespan  */
    double mean_inflight;                /* batches in flight at admissions */
    uint64_t batches, completed, failed, timeouts;
    double mean_setup_s, mean_service_s; /* per completed request          */
    double sustained_qps;                /* completed / makespan          */
    uint64_t shed;                       /* of the timeouts: refused at admission
                                            (a request of the same graph and
                                            pattern size, estimated no
                                            cheaper, timed out)            */
} pm_serve_stats;

pm_status pm_serve(pm_ctx* ctx, const pm_serve_request* reqs, uint32_t nreq,
                   const pm_serve_config* cfg, pm_serve_result* out_results,
                   pm_serve_stats* out_stats);

/* Allocation-free counting, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments and results as pm_submit + pm_wait with
 * PM_AGG_COUNT (counts in `out_values`, host, npat int64), but synchronous
 * on the context's stream, and no device memory is allocated: not from the
 * arena, not by the HIP runtime.  Everything the launch needs beyond the
 * resident graph (plans, counters, queue head, work items, per-wavefront
 * level buffers) lives in one static device array of 64 MiB per GPU, held
 * until the process ends; every plan runs in the general matching kernel.
 * Calls on one GPU share that array: calls from this process are
 * serialised, calls from several processes that overlap on one GPU race.
 * Errors: as pm_submit / pm_wait, and PM_E_NOMEM when the query (at most 64
 * plans) or the graph's level buffers (5 x (max degree + 64) words per
 * wavefront, 4 wavefronts at least) do not fit the 64 MiB. */
pm_status pm_count_noalloc(pm_ctx* ctx, uint32_t graph_id, const pm_pattern* pats,
                           uint32_t npat, int32_t morph, int64_t* out_values);

/* Writes a NUL-terminated description of the matching plan the engine
 * compiles for `pat` on graph `graph_id` (core order, per-level set
 * operations and bounds, tail terms) into `buf` (capacity `cap`). */
pm_status pm_plan_describe(pm_ctx* ctx, uint32_t graph_id, const pm_pattern* pat,
                           char* buf, uint64_t cap);

const char* pm_last_error(void);
const char* pm_status_str(pm_status s);

#ifdef __cplusplus
}
#endif
#endif /* PM_H */
