/*
 * bfscut.h -- C ABI of the MI355X (gfx950) top-k closeness engine.
 *
 * The engine returns the k nodes of largest generalised closeness
 *     c(v) = (r(v) - 1)^2 / ((n - 1) f(v))          (Section 1)
 * where r(v) = |R(v)| counts the nodes reachable from v (v included) and
 * f(v) = sum of d(v, w) over w in R(v) (Table 1), computed with the pruned
 * BFS of Borassi, Crescenzi and Marino (Algorithm 1 and the BFSCut function
 * of Section 2.5, bounds of Lemma 1 / Corollary 1 / Lemma 2, reach bounds of
 * Section 2.3-2.4).  All ranking decisions are exact integer arithmetic:
 *
 *   A(v) = (r(v)-1)^2, F(v) = f(v)     ((A, F) = (0, 1) when r(v) = 1, c = 0)
 *   key(v) > key(w)  iff  A(v) F(w) > A(w) F(v) (unsigned 128-bit), or the
 *                         products are equal and v < w.
 *
 * Results are sorted by decreasing key.  Closeness itself is not returned; a
 * caller computes it for display as (r-1)^2 / ((n-1) f), and 0 when r = 1.
 *
 * Conventions:
 *  - every function returns bc_status and never throws; on failure
 *    bc_last_error() returns a message (thread-local, valid until the next
 *    call on the same thread);
 *  - "host" pointers are ordinary CPU memory; "device" pointers are HIP
 *    device memory of the current device;
 *  - all calls are blocking unless stated otherwise and take an optional
 *    hipStream_t (passed as void*; NULL = the legacy default stream).
 */
#ifndef BFSCUT_H
#define BFSCUT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    BC_OK = 0,
    BC_EINVAL = -1,     /* bad argument (NULL pointer, k <= 0, bad option)      */
    BC_EGRAPH = -2,     /* malformed CSR (see bc_graph_create)                  */
    BC_ENOMEM = -3,     /* device or host allocation failed / over budget       */
    BC_EDEVICE = -4,    /* HIP runtime error                                    */
    BC_EAGAIN = -5,     /* asynchronous query not finished yet                  */
    BC_ECANCELED = -6   /* asynchronous query was cancelled                     */
} bc_status;

typedef struct bc_graph bc_graph;

/* bc_graph_create flags */
#define BC_DIRECTED    0x1u  /* arcs are directed (else every edge must appear in both rows) */
#define BC_VALIDATE    0x2u  /* undirected only: reject a CSR that is not symmetric           */
#define BC_DEVICE_PTRS 0x4u  /* row_ptr / col are device pointers (read, never kept)          */
#define BC_KEEP_IDS    0x10u /* undirected only: keep the caller's numbering on the device.  By
                                default an undirected graph of 100,000 nodes or more is renumbered
                                on upload in breadth-first order (from an approximate centre; other
                                components by degree), so
                                that the node records of neighbours, which a batch reaches together,
                                sit together in memory.  The renumbering is invisible: every result,
                                per-node output and input (orders, scores, warm-start lists) uses the
                                caller's ids, and ties are broken by the caller's ids            */
#define BC_BIG_SCC     0x8u  /* directed only: reach bounds with the largest-SCC refinement at the
                                end of Section 2.4: the largest SCC (largest size; among equals the
                                one holding the smallest node id) gets its exact reach from one
                                breadth-first search, and every component that reaches it also gets
                                the upper bound |R(largest)| + the recurrence over the components
                                outside R(largest).  Tighter bounds, same results               */

/* Source processing order (Algorithm 1 processes nodes in decreasing degree). */
#define BC_ORDER_DEGREE 0    /* decreasing out-degree, ties by increasing id (the paper's order) */
#define BC_ORDER_GIVEN  1    /* opts.perm: a permutation of [0, n) (host pointer)                */
#define BC_ORDER_SCORES 2    /* opts.scores: decreasing score, ties by out-degree then id        */
#define BC_ORDER_GROUPED 3   /* decreasing out-degree; equal degrees grouped by their highest-degree
                                neighbour (then id), so that a batch shares neighbourhoods; ids
                                of the graph's own numbering (see BC_KEEP_IDS)                  */
#define BC_ORDER_LEARNED 4   /* opts.mlp: decreasing score of the order perceptron over the features
                                of bc_graph_features (ties by out-degree, then id)               */
#define BC_ORDER_LEARNED_GROUPED 5 /* opts.mlp: the k best-scored sources (at most as many as the
                                seed batches hold: ceil(k/W) batches unless opts.seed_batches says
                                otherwise) by decreasing score, then all others in BC_ORDER_GROUPED
                                order, so that the seed batches also hold the highest-degree
                                nodes.  On a directed graph it is
                                BC_ORDER_GROUPED: the shipped perceptron is trained on undirected
                                families only, and the degree order is its fallback (its scores
                                picked seed sources that made directed R-MAT 15x slower)          */
#define BC_ORDER_LOCALITY 6  /* compact balls of `width` sources: from a breadth-first order
                                rooted at an approximate centre (middle of a double-sweep
                                path; other components follow in degree order), each batch
                                takes the first unplaced node and grows a breadth-first ball
                                of unplaced nodes around it.  A batch's sources lie within a
                                few hops of each other, so they share most levels (suits
                                graphs without hubs: geometric, grid-like).  Ties and neighbour
                                order follow the graph's own numbering (see BC_KEEP_IDS)        */
#define BC_ORDER_LEARNED_LOCALITY 7 /* opts.mlp: the k best-scored sources (at most as many as the
                                seed batches hold), then all others in BC_ORDER_LOCALITY order (for
                                graphs without hubs); BC_ORDER_LOCALITY on a directed graph      */
#define BC_ORDER_AUTO   -1   /* BC_ORDER_GROUPED in batched mode, BC_ORDER_DEGREE in plain mode   */

/* Parameters of the order perceptron 3 -> 64 -> 64 -> 1 (ReLU, fp32), one flat vector:
 * W1[64][3] @0, b1[64] @192, W2[64][64] @256, b2[64] @4352, w3[64] @4416, b3 @4480. */
#define BC_MLP_PARAMS 4481

/* bc_opts.bounds: optional tighter bounds (each leaves the result unchanged and
 * can only cut a source earlier). */
#define BC_BOUND_FOOTNOTE 0x1u  /* undirected graphs: for d >= 1, ~gamma_{d+1} sums (degree - 1) over
                                   Gamma_d, since one edge of each of its nodes leads back to
                                   Gamma_{d-1} (the footnote of Section 2.3); ignored on directed
                                   graphs                                                        */
#define BC_BOUND_NO_TRIAL 0x2u  /* batched mode, W = 64: skip the over-counted bound test that runs
                                   before a level's exact count (counts taken per arc without
                                   deduplication are at least gamma and ~gamma, so the bound they
                                   give is weaker than Lemma 1 / Lemma 2's and still valid; a source
                                   it cuts skips the exact count).  For measurement and tests     */

/* Execution mode.  Neither changes the result, only the speed. */
#define BC_MODE_PLAIN   0    /* one batch of W sources at a time, level-synchronous
                                kernels launched by a host loop                       */
#define BC_MODE_BATCHED 1    /* seed batches level-synchronously, then one persistent
                                launch in which every workgroup runs whole batches    */

typedef struct bc_opts {
    uint32_t size;          /* sizeof(bc_opts): versioning                               */
    int32_t mode;           /* BC_MODE_*                                                 */
    int32_t order;          /* BC_ORDER_* (default BC_ORDER_AUTO)                        */
    int32_t width;          /* W: sources per bit-parallel batch, 64, 128 or 256         */
    const int32_t* perm;    /* BC_ORDER_GIVEN: host, n entries                           */
    const float* scores;    /* BC_ORDER_SCORES: host, n entries                          */
    float pull_alpha;       /* push -> pull when frontier arcs > m / pull_alpha (0 = never pull) */
    float pull_beta;        /* pull -> push when frontier nodes < n / pull_beta          */
    int32_t slots;          /* BC_MODE_BATCHED: concurrent workgroup batches (0 = auto)  */
    int32_t seed_batches;   /* BC_MODE_BATCHED: level-synchronous batches first (-1 = auto) */
    int32_t chunk;          /* BC_MODE_BATCHED: consecutive batches a workgroup claims at
                               a time (0 = 1)                                            */
    int32_t defer_arcs;     /* BC_MODE_BATCHED: a source whose next level scans more arcs
                               than this leaves its workgroup batch and is re-run by the
                               level-synchronous kernels afterwards (0 = 65536, -1 = never) */
    int32_t lds_tables;     /* BC_MODE_BATCHED, W = 64: keep small batch states in LDS
                               hash tables (0 = yes, -1 = always use the node records,
                               1 = move every batch to the records after its first level,
                               a testing aid for the record path)                       */
    int32_t defer_width;    /* BC_MODE_BATCHED: sources per batch of the re-run of deferred
                               sources, 64, 128 or 256 (0: the narrowest of them that
                               holds every deferred source in one batch, else 256)       */
    const float* mlp;       /* BC_ORDER_LEARNED: host, BC_MLP_PARAMS floats              */
    int32_t graph_levels;   /* level-synchronous batches: 0 (the default) makes one host
                               round trip per level; 1..64 captures that many level steps
                               in a HIP graph and replays it, checking for live sources
                               once per replay; -1 runs every level of every batch of a
                               phase in one cooperative launch, grid barriers between the
                               level steps (BC_EINVAL where the device cannot launch it
                               cooperatively). The default measures fastest on gfx950.  */
    int32_t seed_width;     /* BC_MODE_BATCHED: sources per seed batch, a multiple of width
                               up to 256 (0 = width, or 256 when k > width);
                               seed_batches counts these batches                         */
    uint32_t bounds;        /* BC_BOUND_* flags (default 0: the bounds of Table 1)        */
    const int32_t* first;   /* host, nfirst distinct node ids taken before all others, in
                               this order; the rest follow in the order chosen above (a warm
                               start, e.g. the previous top-k of a graph that has grown;
                               Algorithm 1 gives the same answer for any order)          */
    int32_t nfirst;         /* entries of first, 0 <= nfirst <= n (0: none)              */
} bc_opts;

typedef struct bc_stats {
    uint32_t size;          /* sizeof(bc_stats)                                          */
    uint32_t batches;       /* source batches processed                                  */
    uint64_t m_vis;         /* arcs a sequential BFSCut of each source would scan,
                               summed over sources (the paper's visited arcs)            */
    uint64_t node_arcs;     /* arcs the level kernels scanned (each frontier node once
                               per level, shared by all its live sources)                */
    uint64_t levels;        /* level steps executed                                      */
    uint64_t pull_levels;   /* of which bottom-up                                        */
    uint64_t n_cut, n_done, n_trivial;  /* per-source outcomes                            */
    double preprocess_ms;   /* bc_graph_create time (canonical CSR and reach data)       */
    double query_ms;        /* bc_topk time, call to return                              */
    double seed_ms;         /* level-synchronous part (all of it in plain mode), HIP events */
    double persistent_ms;   /* persistent batched kernel, HIP events on its stream       */
    uint64_t frontier_entries; /* frontier nodes expanded (each once per level)          */
    uint64_t discovered;    /* nodes appended to a new level (each once per level)       */
    uint64_t persistent_arcs;    /* node_arcs of the persistent kernel alone             */
    uint64_t persistent_entries; /* frontier_entries of the persistent kernel alone      */
    uint64_t persistent_discovered; /* discovered of the persistent kernel alone         */
    double defer_ms;        /* level-synchronous re-run of deferred sources, HIP events  */
    uint64_t n_deferred;    /* sources deferred out of the persistent kernel             */
    double phase_ms[5];     /* persistent kernel, summed over its workgroups: batch set-up,
                               level counting, cut step, level build, mark reset         */
    uint64_t lds_levels;    /* persistent W = 64 levels run on the LDS tables            */
    uint64_t record_levels; /* persistent levels run on the global node records          */
    uint64_t spills;        /* batches moved from the LDS tables to the node records     */
    double record_ms;       /* persistent W = 64 levels on the node records, summed over
                               workgroups (part of phase_ms)                             */
    uint64_t record_arcs;   /* arcs those levels scanned                                  */
} bc_stats;

/* Fill *opts with the defaults (plain mode, automatic order, W = 64, bottom-up
 * steps when the frontier holds more than m/3 arcs). */
void bc_opts_default(bc_opts* opts);

/* Message of the last failure on this thread ("" if none). */
const char* bc_last_error(void);

/* Library version string. */
const char* bc_version(void);

/*
 * bc_graph_create -- upload a CSR graph and run the pre-processing step.
 *
 *   n        node count, 0 <= n < 2^31
 *   row_ptr  n + 1 int32 offsets, row_ptr[0] = 0, non-decreasing, row_ptr[n] = m
 *   col      m int32 targets in [0, n)
 *   flags    BC_DIRECTED | BC_VALIDATE | BC_DEVICE_PTRS | BC_BIG_SCC
 *   stream   hipStream_t used by this graph's work (NULL = default stream)
 *   out      receives the handle; release it with bc_graph_destroy
 *
 * The arrays are copied: the caller may free or reuse them on return (host
 * or device).  Rows may be unsorted and may hold self-loops and repeated
 * arcs; these are removed on the device (they change no distance).  The
 * pre-processing follows Section 2.3 (undirected: r(v) = size of the
 * connected component) and Section 2.4 (directed: alpha(v) <= r(v) <=
 * omega(v) from the weighted DAG of strongly connected components, with
 * BC_BIG_SCC also the largest-SCC refinement of the same section).
 *
 * Errors: BC_EINVAL (n < 0, NULL pointer), BC_EGRAPH (row_ptr[0] != 0,
 * decreasing row_ptr, row_ptr[n] != m, col outside [0, n), or with
 * BC_VALIDATE an undirected CSR that is not symmetric), BC_ENOMEM, BC_EDEVICE.
 */
bc_status bc_graph_create(int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col,
                          uint32_t flags, void* stream, bc_graph** out);

/* Release a graph and all its device memory.  NULL is accepted. */
bc_status bc_graph_destroy(bc_graph* g);

/*
 * bc_graph_info -- sizes after canonicalisation (host pointers, any may be NULL).
 */
bc_status bc_graph_info(const bc_graph* g, int32_t* n, int64_t* m, int32_t* directed,
                        double* preprocess_ms);

/*
 * bc_graph_reach -- copy the per-node reach data (host pointers, n entries each):
 * undirected: lo = hi = r(v); directed: lo = alpha(v), hi = omega(v).
 */
bc_status bc_graph_reach(const bc_graph* g, uint32_t* lo, uint32_t* hi);

/*
 * bc_graph_csr -- copy the canonical CSR (host pointers: row_ptr n + 1 entries,
 * col m entries as reported by bc_graph_info).
 */
bc_status bc_graph_csr(const bc_graph* g, int32_t* row_ptr, int32_t* col);

/*
 * bc_topk -- the k nodes of largest closeness (Algorithm 1).
 *
 *   k        number of nodes wanted, k >= 1; count = min(k, n) results
 *   opts     NULL for the defaults (bc_opts_default)
 *   ids      host, capacity k: node ids, decreasing key
 *   farness  host, capacity k: exact f(v)
 *   reach    host, capacity k: exact r(v)
 *   count    host: number of results written
 *   stats    host, optional (NULL): counters and timings of this call
 *
 * The caller owns every output array.  Blocking.  Several calls may run on
 * one graph at the same time from different threads (each call allocates its
 * own working memory).  Errors: BC_EINVAL (k <= 0, NULL outputs, bad opts),
 * BC_ENOMEM, BC_EDEVICE.  With the environment variable BC_CHECK_LISTS=1
 * (a debugging aid), the host-driven level loop also copies the frontier
 * and reset lists after every level and fails with BC_EDEVICE if an entry
 * is not a node id.
 */
bc_status bc_topk(bc_graph* g, int32_t k, const bc_opts* opts, int32_t* ids, uint64_t* farness,
                  uint32_t* reach, int32_t* count, bc_stats* stats);

/*
 * Many queries, one launch.  Algorithm 1 runs its sources in any order and
 * the sources of one query share only the k-th best value (Section 2.1), so
 * the source batches of several queries, on graphs of different sizes, can
 * run side by side in one persistent kernel: every workgroup claims the next
 * batch of a single global sequence, whichever query it belongs to, and each
 * query keeps its own top-k list and threshold records.  The seed batches of
 * every query (ceil(k / W) batches, the first of its order) come first in the
 * sequence; the other batches of a query wait, for a bounded time, until its
 * seed batches have finished, so that they start with a k-th best value to
 * cut against.  Results are those of bc_topk on each graph alone.
 *
 * bc_multi_create -- prepare a launch over `count` queries.
 *   graphs   host array of count graph handles on the current device (a graph
 *            may appear several times; every graph must outlive the launch)
 *   ks       host, count entries: k of each query (>= 1)
 *   opts     NULL for the defaults; width (64, 128 or 256, shared by all
 *            queries), order (a rule applied to each graph: BC_ORDER_DEGREE,
 *            BC_ORDER_GROUPED (the default), BC_ORDER_LOCALITY or a learned
 *            order with opts.mlp), slots (workgroups, 0 = one per compute unit)
 *            and bounds (BC_BOUND_FOOTNOTE) apply; mode, seed_*, defer_*,
 *            lds_tables and graph_levels are ignored (every batch runs in the
 *            launch); BC_ORDER_GIVEN / BC_ORDER_SCORES and opts.first are
 *            rejected (BC_EINVAL)
 *   capture  nonzero: record the launch (a fill kernel that clears the
 *            per-query state, then the persistent kernel) as a HIP graph once,
 *            and replay it on every bc_multi_run
 *   stream   hipStream_t of the runs (NULL = the legacy default stream)
 *   out      receives the handle; release it with bc_multi_destroy
 * The launch owns its device memory: the source orders, per-query lists,
 * threshold records and statistics, and node-record slots sized for the
 * largest graph.  Errors: BC_EINVAL, BC_ENOMEM, BC_EDEVICE.
 *
 * bc_multi_run -- run the prepared launch (blocking; any number of times,
 * never two at once on one handle).
 *   ids, farness, reach  host, sum of ks entries: query i writes its results,
 *            sorted by decreasing key, from offset ks[0] + ... + ks[i-1]
 *   counts   host, count entries: min(k_i, n_i) results per query
 *   stats    host, optional (NULL): count bc_stats, each with its size set
 *            (persistent_ms and query_ms are those of the whole launch)
 *
 * bc_topk_multi -- bc_multi_create (no capture, on the first graph's stream),
 * one bc_multi_run, bc_multi_destroy.
 */
typedef struct bc_multi bc_multi;

bc_status bc_multi_create(bc_graph* const* graphs, int32_t count, const int32_t* ks, const bc_opts* opts,
                          int32_t capture, void* stream, bc_multi** out);
bc_status bc_multi_run(bc_multi* p, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* counts,
                       bc_stats* stats);
bc_status bc_multi_destroy(bc_multi* p);
bc_status bc_topk_multi(bc_graph* const* graphs, int32_t count, const int32_t* ks, const bc_opts* opts,
                        int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* counts, bc_stats* stats);

/*
 * bc_topk_static -- bc_topk in plain mode (W = 64) that allocates nothing:
 * for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc).
 *
 *   g, k, ids, farness, reach, count   as for bc_topk (host outputs of
 *            capacity k; count = min(k, n) results in decreasing key order)
 *
 * Every buffer of the query (control block, top-k list and threshold
 * records, statistics, source order, node records and lists) lives in one
 * static device array of 64 MiB per device, which the library holds from the
 * first call on that device until the process ends; it calls no hipMalloc,
 * hipFree or allocating library routine.  The array needs about 72 n + 32 k
 * bytes plus 20 KiB, so graphs of up to about 900,000 nodes fit; larger
 * ones are rejected with BC_EINVAL and a message.  Sources are taken in the
 * graph's degree order when it holds one (any earlier plain-mode or degree-
 * order query builds it), else in node-id order; the answer is the same.
 * Calls on one device share the array: calls from threads of one process are
 * serialised by the library, and each call clears the state it needs (the
 * array keeps the last call's contents).  Blocking, on the graph's stream.
 * Errors: BC_EINVAL (k <= 0, NULL outputs, graph too large for the array),
 * BC_EDEVICE.
 */
bc_status bc_topk_static(bc_graph* g, int32_t k, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* count);

/*
 * bc_farness_all -- exact farness and reach of every node (the textbook
 * computation of Section 1: one breadth-first search per node, here in
 * bit-parallel batches, with no bound and no cut).
 *
 *   opts     NULL for the defaults; mode, width, order and batching knobs
 *            apply as in bc_topk (they change the speed only)
 *   farness  host, n entries: f(v) of node v
 *   reach    host, n entries: r(v) of node v
 *   stats    host, optional
 *
 * Blocking.  Used to label training data of the order perceptron and as the
 * baseline the pruned search is compared with.  Errors as bc_topk.
 */
bc_status bc_farness_all(bc_graph* g, const bc_opts* opts, uint64_t* farness, uint32_t* reach, bc_stats* stats);

/*
 * bc_source_order -- the order in which bc_topk with the same k and opts
 * takes its sources (Algorithm 1 visits the nodes in any fixed order and
 * returns the same answer; the order only decides how soon the k-th best
 * value is known, Section 2.1).
 *
 *   k        as for bc_topk (the learned grouped order depends on it)
 *   opts     NULL for the defaults; order, perm, scores, mlp, mode, width,
 *            seed_batches and seed_width are read
 *   order    host, n entries: a permutation of 0 .. n-1
 *
 * Blocking.  For inspection and tests.  Errors: BC_EINVAL (k <= 0, NULL
 * order, bad opts), BC_ENOMEM, BC_EDEVICE.
 */
bc_status bc_source_order(bc_graph* g, int32_t k, const bc_opts* opts, int32_t* order);

/*
 * bc_autotune -- pick the batched-mode execution knobs for one graph and k.
 *
 * None of the knobs changes the answer, only the time.  Starting from
 * `base` (NULL: defaults) in BC_MODE_BATCHED, the tuner runs the query over
 * a grid of width (64, 128, 256) x defer_arcs (16384, 65536, 262144, never),
 * then tries one knob at a time around the best setting so far:
 * defer_width (64, 256), pull_alpha (never, 3, 14), slots (128, 256, 512)
 * and order (grouped, degree, locality).  Each setting is timed as the best of
 * `repeats` runs after one
 * warm-up.  Every run must return exactly the first run's top-k, else
 * BC_EDEVICE.  *best receives the fastest setting; report (may be NULL) the
 * trial count and the times of the base and best settings.
 */
typedef struct bc_tune_report {
    uint32_t size;
    int32_t trials;
    double default_ms, best_ms;
} bc_tune_report;

bc_status bc_autotune(bc_graph* g, int32_t k, const bc_opts* base, int32_t repeats, bc_opts* best,
                      bc_tune_report* report);

/*
 * Serving: a queue of top-k requests over many graphs on one GPU.
 *
 * Graphs are registered once (host arrays, copied) and made resident on
 * demand; resident graphs that no running request uses are evicted, least
 * recently used first, when the memory budget needs room.  Requests start
 * in submission order as soon as their footprint fits the free budget, on
 * one of `lanes` concurrent HIP streams, so several requests share the GPU;
 * each batched request's persistent kernel uses at most `slots` workgroups.
 * A request's result is the same as that of bc_topk on the same graph with
 * the same k (Algorithm 1 is exact for every order and threshold history).
 */
typedef struct bc_server bc_server;

typedef struct bc_server_opts {
    uint32_t size;          /* sizeof(bc_server_opts)                                    */
    int32_t lanes;          /* concurrent requests (streams), 1..16 (default 4)          */
    int32_t slots;          /* workgroups of one batched request's persistent kernel
                               (default 64); opts.slots of a request overrides it       */
    int32_t device;         /* HIP device (-1: the current one)                          */
    uint64_t budget_bytes;  /* device memory for resident graphs and running requests
                               (0: 45 % of the free memory at creation)                 */
    int32_t queue;          /* 1: continuous batching through a device-visible queue:
                               lanes only prepare requests (upload, order, lists) and
                               append them to a queue in pinned host memory that one
                               persistent kernel drains while it runs, its workgroups
                               taking the next source batch of whichever request waits,
                               so requests that arrive while others run start as soon as
                               a workgroup is free and run beside them.  Batched requests
                               with k <= 256 on graphs no larger than the largest one
                               registered before the first request use it; others run as
                               whole-request launches on the lanes.  When a lane's own
                               device work has waited 2 ms behind the running kernel, the
                               kernel finishes its current batches, ends, and is launched
                               again after that work.  0 (default): lanes only           */
    int32_t queue_width;    /* W of the queue kernel (64, 128 or 256; default 64): every
                               queued request uses it (the width changes the speed only) */
    int32_t queue_slots;    /* workgroups of the queue kernel (0: one per compute unit);
                               their node records, sized for the largest registered graph,
                               are reserved in the budget while the server lives          */
} bc_server_opts;

typedef struct bc_request_info {
    uint32_t size;          /* sizeof(bc_request_info)                                   */
    int32_t lane;           /* lane the request ran on (-1: never started)               */
    int32_t uploaded;       /* 1 if it had to make its graph resident first              */
    int32_t reserved;
    double submit_ms, start_ms, finish_ms;  /* since server creation (host clock)       */
    uint64_t footprint_bytes;  /* working memory reserved for it                          */
} bc_request_info;

typedef struct bc_server_stats {
    uint32_t size;
    uint32_t graphs, resident_graphs, queued, running, reserved;
    uint64_t budget_bytes, used_bytes, peak_bytes;
    uint64_t uploads, evictions, completed, failed, canceled;
    uint64_t queue_inflight;  /* requests in the device queue now                           */
    uint64_t queue_launches;  /* launches of the queue's persistent kernel so far           */
    uint64_t queue_batches;   /* source batches published to the queue so far               */
} bc_server_stats;

void bc_server_opts_default(bc_server_opts* opts);

/* Start a server (its lane threads and streams).  Errors: BC_EINVAL, BC_EDEVICE. */
bc_status bc_server_create(const bc_server_opts* opts, bc_server** out);

/* Cancel queued requests, wait for running ones (requests in the device queue
 * get a minute; then they fail with BC_EDEVICE and the queue's kernel stops
 * claiming batches), free every graph and stream. */
bc_status bc_server_destroy(bc_server* s);

/* Register a graph (host arrays as for bc_graph_create, copied; not resident
 * until a request needs it).  graph_id receives its index. */
bc_status bc_server_add_graph(bc_server* s, int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col,
                              uint32_t flags, int32_t* graph_id);

/* Queue a top-k request (opts as for bc_topk; the arrays it points at are
 * copied).  Returns at once with a ticket. */
bc_status bc_submit(bc_server* s, int32_t graph_id, int32_t k, const bc_opts* opts, uint64_t* ticket);

/* Block until the request has finished (or timeout_ms passes: BC_EAGAIN;
 * a negative timeout waits for ever). */
bc_status bc_wait(bc_server* s, uint64_t ticket, int32_t timeout_ms);

/* BC_EAGAIN while queued or running.  Once finished: writes the results
 * (host arrays of capacity k, as bc_topk), stats and info (both may be
 * NULL), releases the ticket and returns BC_OK, the request's error (e.g.
 * BC_ENOMEM when its footprint exceeds the whole budget), or BC_ECANCELED. */
bc_status bc_poll(bc_server* s, uint64_t ticket, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* count,
                  bc_stats* stats, bc_request_info* info);

/* Progress of a request in the device queue: source batches finished and
 * batches in all (both 0 for a request that is not in the queue, or not yet
 * in it).  Read from a counter the kernel raises in pinned host memory; no
 * device call.  BC_EINVAL for an unknown ticket. */
bc_status bc_progress(bc_server* s, uint64_t ticket, uint64_t* done_batches, uint64_t* total_batches);

/* Cancel: a queued request is dropped at once; a running one completes and
 * its result is discarded.  BC_EINVAL if it has already finished. */
bc_status bc_cancel(bc_server* s, uint64_t ticket);

bc_status bc_server_info(bc_server* s, bc_server_stats* out);

/* The admission estimate for a graph of n nodes and m arcs and one request
 * (pure arithmetic, no device call): bytes the graph holds while resident,
 * transient bytes of its upload, working memory of the request. */
bc_status bc_footprint(int32_t n, int64_t m, uint32_t flags, int32_t k, const bc_opts* opts, int32_t slots,
                       uint64_t* graph_bytes, uint64_t* upload_bytes, uint64_t* query_bytes);

/*
 * Learned source order.  Algorithm 1 returns the same top-k whatever order
 * the sources are processed in; the order only decides how soon the k-th
 * best value is known (Section 2.1).  The paper processes by decreasing
 * degree; BC_ORDER_LEARNED processes by decreasing score of a perceptron
 * trained to predict log closeness from three per-node features.  These
 * calls expose the features and the perceptron so that it can be trained
 * on the device.
 */

/*
 * bc_graph_features -- per-node features of the order perceptron.
 *
 *   x     device, n * 3 floats, row v = (x0, x1, x2) of node v, each column
 *         standardised over the nodes ((x - mean) / population std; 0 when
 *         the column's integers are all equal):
 *           x0 = log(1 + outdeg(v))
 *           x1 = log(1 + sum of outdeg(u) over the out-arcs v -> u)
 *           x2 = log(1 + core(v))
 *   core  device, n uint32 (may be NULL): core(v), the largest c such that v
 *         lies in a subgraph in which every node has >= c out-neighbours
 *         (the k-core number of an undirected graph)
 *
 * Computed once per graph and cached; the call copies into the caller's
 * arrays and returns when they are written.  Errors: BC_EINVAL, BC_EDEVICE.
 */
bc_status bc_graph_features(bc_graph* g, float* x, uint32_t* core);

/* y[i] = perceptron(x[3i .. 3i+2]) for i < count (device pointers; params
 * holds BC_MLP_PARAMS floats).  Asynchronous on `stream`. */
bc_status bc_mlp_forward(const float* params, const float* x, int64_t count, float* y, void* stream);

/*
 * bc_mlp_loss_grad -- loss and gradient of the order perceptron.
 *
 *   loss = sum_i w[v_i] (y(x[v_i]) - t[v_i])^2 / sum_i w[v_i],  v_i = idx[i]
 *   (or i when idx is NULL), i < count
 *
 *   params  device, BC_MLP_PARAMS floats
 *   x, t, w device, rows * 3, rows, rows floats (w may be NULL: all 1)
 *   idx     device, count int32 in [0, rows), or NULL (then count <= rows)
 *   grad    device, BC_MLP_PARAMS floats, written
 *   loss    host, may be NULL
 *
 * Blocking (synchronises `stream`).  Deterministic: tiles of 128 samples
 * summed in a fixed order.  Errors: BC_EINVAL (an idx entry outside
 * [0, rows), count > rows without idx), BC_ENOMEM, BC_EDEVICE.
 */
bc_status bc_mlp_loss_grad(const float* params, const float* x, const float* t, const float* w, int64_t rows,
                           const int32_t* idx, int64_t count, float* grad, double* loss, void* stream);

/* One Adam step (Kingma and Ba, 2015) on BC_MLP_PARAMS floats (device):
 * m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
 * params -= lr (m / (1-b1^step)) / (sqrt(v / (1-b2^step)) + eps); step >= 1.
 * Asynchronous on `stream`. */
bc_status bc_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                      float beta2, float eps, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* BFSCUT_H */
