// Internal declarations of the gfx950 top-k closeness library.
//
// Device-side layout of one graph (all int32 unless noted):
//   rp[n+1], col[m]        canonical out-CSR (rows sorted, no self-loops or repeats)
//   irp[n+1], icol[m]      in-CSR (directed graphs; aliases the out-CSR otherwise)
//   deg[n]   (u32)         out-degree
//   adj[m]   (int2)        (col[e], deg[col[e]]): each arc with its target's
//                          out-degree, so a level step that counts ~gamma reads
//                          the degree in the same coalesced stream as the target
//   x0[n], x1[n] (u32)     reach data: undirected x0 = x1 = r(v) (component size);
//                          directed x0 = alpha(v), x1 = omega(v)
//   orig[n]                the caller's id of each node, or null when the graph
//                          keeps the caller's numbering.  Undirected graphs are
//                          renumbered on upload in breadth-first order, so that
//                          the nodes a batch reaches together sit together in
//                          the node records; every result and per-node output is
//                          given back in the caller's numbering, and ties are
//                          broken by the caller's ids
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "bfscut.h"

namespace bc {

void set_error(const char* fmt, ...);

#define BC_HIP(expr)                                                                    \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::bc::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),      \
                            __FILE__, __LINE__);                                        \
            return BC_EDEVICE;                                                          \
        }                                                                               \
    } while (0)

#define BC_TRY(expr)                      \
    do {                                  \
        bc_status s_ = (expr);            \
        if (s_ != BC_OK) return s_;       \
    } while (0)

struct DevGraph {
    int32_t n;
    int64_t m;
    int32_t directed;
    const int32_t* rp;
    const int32_t* col;
    const int32_t* irp;
    const int32_t* icol;
    const uint32_t* deg;
    const int2* adj;
    const uint32_t* x0;
    const uint32_t* x1;
    const int32_t* orig;
};

// Raise the release threshold of the device's default memory pool once per
// device, so that stream-ordered frees keep their memory in the pool.
void prepare_pool();

// Device allocation owned by a graph or a query; freed in the destructor.
// alloc() is a plain hipMalloc (graph lifetime); alloc_on(stream) is
// stream-ordered (hipMallocAsync / hipFreeAsync on that stream), so that
// query-lifetime buffers never wait for the whole device when released
// while other streams are running.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    bool ordered = false;
    hipStream_t stream = nullptr;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            if (ordered) (void)hipFreeAsync(p, stream);
            else (void)hipFree(p);
        }
        p = nullptr;
        bytes = 0;
        ordered = false;
    }
    bc_status alloc(size_t nbytes) {
        release();
        if (nbytes == 0) nbytes = 8;
        if (hipMalloc(&p, nbytes) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            set_error("hipMalloc of %zu bytes failed", nbytes);
            return BC_ENOMEM;
        }
        bytes = nbytes;
        return BC_OK;
    }
    bc_status alloc_on(size_t nbytes, hipStream_t s) {
        release();
        prepare_pool();
        if (nbytes == 0) nbytes = 8;
        if (hipMallocAsync(&p, nbytes, s) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            set_error("hipMallocAsync of %zu bytes failed", nbytes);
            return BC_ENOMEM;
        }
        bytes = nbytes;
        ordered = true;
        stream = s;
        return BC_OK;
    }
    template <class T>
    T* as() const { return reinterpret_cast<T*>(p); }
    void swap(DevBuf& o) {
        std::swap(p, o.p);
        std::swap(bytes, o.bytes);
        std::swap(ordered, o.ordered);
        std::swap(stream, o.stream);
    }
};

}  // namespace bc

namespace bc {

// Working memory of top-k queries on one graph, kept between queries.  Every
// query leaves seen/nxt/cur all zero (each batch resets the nodes it
// reached), so a cached workspace is reused without clearing.
struct Workspace {
    int ww = 0;        // mask words per node the buffers were sized for
    int slots = 0;     // batched slots allocated
    DevBuf seen, qa, qb, clr;     // level-synchronous slot: node records and lists
    DevBuf bseen, bqa, bqb, bclr;  // persistent slots
    DevBuf srcs, ctl, nextb, slot_stamp, defer;
    bool plain_ready = false;
    hipStream_t stream = nullptr;  // stream its buffers are ordered on
    uint32_t* hctl = nullptr;      // pinned copy of the level-synchronous control block
    hipStream_t cap = nullptr;     // private stream that captures level-step graphs
    Workspace() = default;
    explicit Workspace(hipStream_t s) : stream(s) {}
    Workspace(const Workspace&) = delete;
    Workspace& operator=(const Workspace&) = delete;
    ~Workspace() {
        if (hctl) (void)hipHostFree(hctl);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

}  // namespace bc

struct bc_graph {
    bc::DevGraph dg{};
    bc::DevBuf rp, col, irp, icol, deg, adj, x0, x1;
    bc::DevBuf order_deg;  // cached degree order (int32 n), built on first use
    bool have_order_deg = false;
    bc::DevBuf order_grp;  // cached grouped degree order
    bool have_order_grp = false;
    bc::DevBuf order_loc_seed;  // cached breadth-first order from a centre
    bool have_order_loc_seed = false;
    bc::DevBuf order_loc[3];  // cached locality orders for batches of 64, 128, 256
    bool have_order_loc[3] = {false, false, false};
    bc::DevBuf feat, core;  // learned-order features (n x 3 float) and core numbers, built on first use
    bool have_feat = false;
    bc::DevBuf order_lrn;                 // cached order by decreasing perceptron score, for lrn_params
    std::vector<float> lrn_params;        // the parameters it was scored with (the first set asked for)
    bool have_order_lrn = false;
    static constexpr int kLrnHeads = 4;   // learned head + grouped tail orders kept, per head length
    bc::DevBuf order_lrn_head[kLrnHeads];
    int32_t lrn_head[kLrnHeads] = {0, 0, 0, 0};
    int n_lrn_heads = 0;
    int core_sweeps = 0;
    hipStream_t stream = nullptr;
    double preprocess_ms = 0.0;
    int device = 0;
    std::mutex ws_mu;                       // guards ws_busy
    bool ws_busy = false;
    std::unique_ptr<bc::Workspace> ws;      // cached workspace (one query at a time)
    std::mutex cache_mu;                    // guards building the cached orders and features
    bool ordered = false;                   // graph buffers are stream-ordered allocations (server graphs)
    bool big_scc = false;                   // directed reach bounds with the largest-SCC refinement
    bc::DevBuf orig, inv;                   // renumbering: our id -> caller's id, caller's id -> ours
    bool relabeled = false;
};

namespace bc {
// A graph-lifetime buffer: stream-ordered on s for server graphs (their
// lane streams outlive them), a plain allocation otherwise.
inline bc_status galloc(bc_graph* g, DevBuf& b, size_t bytes, hipStream_t s) {
    return g->ordered ? b.alloc_on(bytes, s) : b.alloc(bytes);
}
}  // namespace bc

namespace bc {

// Pre-processing (preprocess.hip): validation, canonical CSR, degrees,
// transpose and reach data.  rp/col are host or device pointers per flags.
bc_status graph_build(bc_graph* g, int32_t n, int64_t m, const int32_t* rp, const int32_t* col,
                      uint32_t flags);
// Renumber a built undirected graph in breadth-first order (the locality
// seed order): *out receives the renumbered graph (built on the same stream,
// with orig/inv), g is left as it was for the caller to release.
bc_status graph_relabel(bc_graph* g, uint32_t flags, bool ordered, bc_graph** out);
// Id maps of a renumbered graph, on the device: ids[i] = inv[ids[i]] (caller's
// ids to ours) or orig[ids[i]] (ours to the caller's); no-ops otherwise.
bc_status ids_to_internal(bc_graph* g, int32_t* d_ids, int64_t count, hipStream_t s);
bc_status ids_to_caller(bc_graph* g, int32_t* d_ids, int64_t count, hipStream_t s);
// Gather per-node rows from our numbering into the caller's: dst[v] = src[inv[v]]
// (rows of `width` 4-byte words); a plain copy when the graph is not renumbered.
bc_status rows_to_caller(bc_graph* g, const void* d_src, void* d_dst, int width, hipStream_t s);
// bc_graph_create on stream s; ordered = stream-ordered graph buffers.
bc_status graph_create(int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col, uint32_t flags,
                       hipStream_t s, bool ordered, bc_graph** out);

// Source orders (preprocess.hip): decreasing out-degree (ties by id), or a
// given permutation, or decreasing score (ties by degree, then id).
// Every order call runs on stream s and returns with d_order written.
bc_status order_by_degree(bc_graph* g, int32_t* d_order, hipStream_t s);
bc_status order_grouped(bc_graph* g, int32_t* d_order, hipStream_t s);
bc_status order_by_scores(bc_graph* g, const float* scores, bool scores_on_device, int32_t* d_order, hipStream_t s);
bc_status order_given(bc_graph* g, const int32_t* h_perm, int32_t* d_order, hipStream_t s);
// Move the nf distinct node ids h_first (host) to the front of the order
// d_order (a permutation of [0, n)), keeping the relative order of the rest.
// (caller_ids: h_first holds the caller's ids, else ids of the graph's own numbering)
bc_status order_front(bc_graph* g, const int32_t* h_first, int32_t nf, int32_t* d_order, hipStream_t s,
                      bool caller_ids = true);
// The sources by decreasing perceptron score (ties by degree, then id) for
// the host parameters h_params; cached per graph for the first parameter set.
bc_status order_learned(bc_graph* g, const float* h_params, int32_t* d_order, hipStream_t s);
// The first `head` entries of the device order d_by_score, then every other
// source in the grouped degree order.
bc_status order_head_grouped(bc_graph* g, const int32_t* d_by_score, int32_t head, int32_t* d_order, hipStream_t s);
// The `head` best-scored sources for h_params, then the grouped order; kept
// per graph for the kept parameter set and up to kLrnHeads head lengths.
bc_status order_learned_grouped(bc_graph* g, const float* h_params, int32_t head, int32_t* d_order, hipStream_t s);
bc_status order_locality(bc_graph* g, int32_t B, int32_t* d_order, hipStream_t s);

// Learned order (learned.hip): features cached in g->feat / g->core; the
// perceptron's forward pass, loss gradient and Adam step.
bc_status graph_features(bc_graph* g, hipStream_t s);
bc_status mlp_forward(const float* params, const float* x, int64_t count, float* y, hipStream_t s);
bc_status mlp_loss_grad(const float* params, const float* x, const float* t, const float* w, int64_t rows,
                        const int32_t* idx, int64_t count, float* grad, double* loss, hipStream_t s);
bc_status mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                   float beta2, float eps, hipStream_t s);

// Admission estimate of the server (serve.hip).
void footprint(int32_t n, int64_t m, bool directed, int32_t k, const bc_opts& o, int32_t slots, uint64_t* graph_bytes,
               uint64_t* upload_bytes, uint64_t* query_bytes);

// Top-k drivers (topk.hip).
// Queries run on stream s (the graph's stream for the blocking API, a lane
// stream of the server); with private_ws the query never uses the graph's
// cached workspace (its working memory is allocated and released with it).
bc_status run_topk(bc_graph* g, int32_t k, const bc_opts& o, int32_t* ids, uint64_t* farness,
                   uint32_t* reach, int32_t* count, bc_stats* st, hipStream_t s, bool private_ws = false);
bc_status build_order(bc_graph* g, const bc_opts& o, int32_t kk, int32_t* d_order, hipStream_t s);
bc_status run_farness_all(bc_graph* g, const bc_opts& o, uint64_t* farness, uint32_t* reach, bc_stats* st,
                          hipStream_t s);

// Plain-mode top-k with every buffer in one static device array (topk.hip):
// allocates nothing.
bc_status run_topk_static(bc_graph* g, int32_t k, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* count);

// Many queries (graph, k) in one persistent launch (topk.hip): prepare the
// launch (orders, per-query state, descriptors, shared slots; with capture,
// a HIP graph of it), run it (any number of times), release it.
bc_status multi_create(bc_graph* const* graphs, int32_t count, const int32_t* ks, const bc_opts& o, hipStream_t s,
                       bool capture, bc_multi** out);
bc_status multi_run(bc_multi* p, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* counts,
                    bc_stats* stats);
void multi_destroy(bc_multi* p);

// Serving queue drained by a running persistent job kernel (topk.hip).
// devq_create: ring, result areas and flags in pinned host memory, node-record
// slots for graphs of up to ncap nodes (*device_bytes: their size).
// devq_submit: build the request's order on `prep`, write its descriptor and
// publish it (blocks while every ring slot is in flight); the kernel is
// launched when none is running.  devq_done polls the request's flag;
// devq_collect copies its results; devq_release frees its slot and memory;
// devq_pump relaunches the kernel when work waits and it has ended.
struct DevQueue;
struct QueueJob;
constexpr int kQueueMaxK = 256;  // largest k a queued request may ask for
bc_status devq_create(int W, int32_t ncap, int slots, DevQueue** out, uint64_t* device_bytes);
void devq_destroy(DevQueue* q);
int devq_width(const DevQueue* q);
int32_t devq_ncap(const DevQueue* q);
bc_status devq_submit(DevQueue* q, bc_graph* g, int32_t k, const bc_opts& o, hipStream_t prep, QueueJob** out);
bool devq_done(DevQueue* q, const QueueJob* j);
bc_status devq_collect(DevQueue* q, QueueJob* j, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* count,
                       bc_stats* st, double query_ms);
void devq_release(DevQueue* q, QueueJob* j);
void devq_free(QueueJob* j);  // memory of an entry whose queue is gone
bc_status devq_pump(DevQueue* q);
// A lane brackets device work of its own with these while a queue exists:
// the pump then lets a long-running launch end so that this work, which may
// share a hardware queue with it, can run.
void devq_wait_begin(DevQueue* q);
void devq_wait_end(DevQueue* q);
// Scope form of the pair (also ends the wait when the work throws).
struct DevqWait {
    DevQueue* q;
    explicit DevqWait(DevQueue* q_) : q(q_) { devq_wait_begin(q); }
    ~DevqWait() { devq_wait_end(q); }
    DevqWait(const DevqWait&) = delete;
    DevqWait& operator=(const DevqWait&) = delete;
};
// Publish the rest of a request once its seed batches have finished (true
// when it did); launch and published-batch counts for the server's report.
bool devq_advance(DevQueue* q, QueueJob* j);
void devq_progress(DevQueue* q, const QueueJob* j, uint64_t* done, uint64_t* total);
unsigned long long devq_launches(DevQueue* q);
unsigned long long devq_published(DevQueue* q);

}  // namespace bc
