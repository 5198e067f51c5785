// Serving: many top-k requests over many graphs on one GPU.
//
// Graphs are registered with a host copy of their CSR and made resident on
// demand; a resident graph that no running request uses is evicted, least
// recently used first, when the memory budget needs room.  Requests wait in
// one FIFO queue.  The head request starts as soon as its footprint (the
// graph if it is not resident, plus the request's own working memory) fits
// the free budget; it then runs on one of L lanes, each a worker thread with
// its own non-blocking HIP stream, so the persistent kernels of up to L
// requests share the GPU and a finished request's lane takes the next one at
// once.  Each request's persistent kernel is limited to `slots` workgroups,
// so that L requests fit side by side on the compute units.
//
// With the device queue (bc_server_opts.queue = 1) a lane only prepares a
// request (upload, source order, its list and threshold records) and hands
// it to a device-visible queue that one persistent kernel drains while it
// runs: the kernel's workgroups claim the next source batch of whichever
// queued request it belongs to, so requests that arrive while others are on
// the GPU are admitted as slots free up and their batches run beside the
// others' (continuous batching).  A reaper thread collects finished requests
// from their flags in pinned host memory and relaunches the kernel when it
// has ended with work waiting.
//
// The top-k of a request is the same whatever runs beside it: every query
// keeps its own list, threshold records and working memory (a stale or
// private threshold never changes the result, Section 2.1).
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bc_internal.h"

namespace bc {

// Bytes a graph holds while resident, the transient bytes of its upload,
// and the working memory of one query (an upper estimate: every buffer the
// query path allocates, at its largest).
void footprint(int32_t n, int64_t m, bool directed, int32_t k, const bc_opts& o, int32_t slots,
               uint64_t* graph_bytes, uint64_t* upload_bytes, uint64_t* query_bytes) {
    const uint64_t N = (uint64_t)(n > 0 ? n : 0), M = (uint64_t)(m > 0 ? m : 0);
    // out-CSR, arcs packed with target degrees, degree, reach pair, cached
    // orders (degree, grouped, learned, up to four learned heads + grouped
    // tail), features and core numbers
    uint64_t gb = 4 * (N + 1) + 4 * M + 8 * M + 4 * N + 8 * N + 28 * N + 16 * N;
    if (directed) gb += 4 * (N + 1) + 4 * M;  // in-CSR
    else if (N >= 100000) gb += 8 * N;         // renumbering maps
    // upload: raw copy, sort buffers and component / SCC scratch; an
    // undirected graph is built twice (the second time renumbered), so the
    // first build is held until the second one exists
    uint64_t ub = 12 * M + 40 * N + (1u << 20);
    if (!directed && N >= 100000) ub += gb + 16 * N + 4 * M;
    const int W = o.width == 128 || o.width == 256 ? o.width : 64;
    const uint64_t SW = W == 64 ? 4 : (W == 128 ? 8 : 16);
    const uint64_t per_slot = N * (8 * SW + 12);
    const uint64_t nb = (N + (uint64_t)W - 1) / (uint64_t)W;
    uint64_t sl = slots > 0 ? (uint64_t)slots : 1;
    if (o.slots > 0) sl = (uint64_t)o.slots;
    if (sl > nb) sl = nb > 0 ? nb : 1;
    const uint64_t kk = (uint64_t)(k > 0 ? k : 1);
    uint64_t qb = 4 * N                     // order
                  + 24 * (N + 1)            // threshold records
                  + 64 + 32 * kk            // top-k list
                  + 4096                    // statistics, control blocks
                  + per_slot + 32 * 256     // level-synchronous slot
                  + 4 * N + 64              // deferred sources
                  + 24 * N;                 // order sort temporaries
    if (o.mode == BC_MODE_BATCHED) qb += sl * per_slot + 4 * sl;
    if (o.order == BC_ORDER_LEARNED || o.order == BC_ORDER_LEARNED_GROUPED) qb += 8 * N + 4 * BC_MLP_PARAMS + 16 * N;
    *graph_bytes = gb;
    *upload_bytes = ub;
    *query_bytes = qb;
}

namespace {

enum : int { RQ_QUEUED = 0, RQ_RUNNING = 1, RQ_DONE = 2, RQ_FAILED = 3, RQ_CANCELED = 4 };

struct SrvGraph {
    int32_t n = 0;
    int64_t m = 0;
    uint32_t flags = 0;
    std::vector<int32_t> rp, col;  // host copy
    bc_graph* g = nullptr;         // resident copy, or null
    bool loading = false;
    int refs = 0;                  // requests running on it
    uint64_t last_use = 0;
    uint64_t resident_bytes = 0;   // reserved while resident
};

struct SrvReq {
    uint64_t id = 0;
    int32_t gid = 0;
    int32_t k = 0;
    bc_opts o{};
    std::vector<int32_t> perm, first;
    std::vector<float> scores, mlp;
    int state = RQ_QUEUED;
    bool cancel = false;
    bc_status status = BC_OK;
    std::string err;
    std::vector<int32_t> ids;
    std::vector<uint64_t> far;
    std::vector<uint32_t> reach;
    int32_t count = 0;
    bc_stats st{};
    double t_submit = 0, t_start = 0, t_finish = 0;
    uint64_t query_bytes = 0, upload_bytes = 0;
    uint64_t lane_bytes = 0, queue_bytes = 0;  // working memory as a whole-request launch / in the queue
    bool to_queue = false;                     // admitted for the device queue
    int lane = -1;
    bool uploaded = false;
    QueueJob* qjob = nullptr;  // in the device queue (finished by the reaper)
};

// Working memory of a request in the device queue: its order, threshold
// records, list and statistics, the order's sort temporaries and (learned
// orders) the features and scores.  The node-record slots belong to the queue.
uint64_t queue_request_bytes(int32_t n, int32_t k, const bc_opts& o) {
    const uint64_t N = (uint64_t)(n > 0 ? n : 0), kk = (uint64_t)(k > 0 ? k : 1);
    uint64_t b = 4 * N + 24 * (N + 1) + 512 + 32 * kk + 24 * N;
    if (o.order == BC_ORDER_LEARNED || o.order == BC_ORDER_LEARNED_GROUPED || o.order == BC_ORDER_LEARNED_LOCALITY)
        b += 8 * N + 4 * BC_MLP_PARAMS + 16 * N;
    return b;
}

}  // namespace
}  // namespace bc

struct bc_server {
    int device = 0;
    uint64_t budget = 0;
    int lanes = 4;
    int slots = 64;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<uint64_t> queue;
    std::unordered_map<uint64_t, std::unique_ptr<bc::SrvReq>> reqs;
    std::vector<std::unique_ptr<bc::SrvGraph>> graphs;
    uint64_t used = 0, peak = 0, next_id = 1, clock = 0;
    uint64_t uploads = 0, evictions = 0, completed = 0, failed = 0, canceled = 0;
    int running = 0;
    bool stop = false;
    std::vector<hipStream_t> streams;
    std::vector<std::thread> workers;
    std::chrono::steady_clock::time_point t0;
    // device queue mode
    bool queue_mode = false;
    int queue_width = 64;
    int queue_slots = 0;
    bc::DevQueue* q = nullptr;
    bool q_failed = false;
    uint64_t q_bytes = 0;
    std::vector<bc::SrvReq*> inflight;  // requests in the device queue
    std::vector<bc::QueueJob*> orphans; // queue entries given up at shutdown, freed after the kernel ends
    bool reaper_stop = false;
    std::thread reaper;

    double now_ms() const {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
};

namespace bc {
namespace {

void reserve(bc_server* S, uint64_t b) {
    S->used += b;
    if (S->used > S->peak) S->peak = S->used;
}

// Evict idle resident graphs (least recently used first, never `keep`)
// until `need` more bytes fit.  Caller holds the lock.
void evict_for(bc_server* S, uint64_t need, const SrvGraph* keep) {
    while (S->used + need > S->budget) {
        SrvGraph* victim = nullptr;
        for (auto& G : S->graphs)
            if (G->g && !G->loading && G->refs == 0 && G.get() != keep && (!victim || G->last_use < victim->last_use))
                victim = G.get();
        if (!victim) return;
        (void)bc_graph_destroy(victim->g);
        victim->g = nullptr;
        S->used -= victim->resident_bytes;
        ++S->evictions;
    }
}

// Decide on the head of the queue (caller holds the lock).  Returns the
// request to start, or null.  A head that cannot fit even with every lane
// idle and every other graph evicted fails with BC_ENOMEM.
bool queue_eligible(bc_server* S, const SrvReq* r, const SrvGraph* G);

SrvReq* admit_head(bc_server* S) {
    while (!S->queue.empty()) {
        SrvReq* r = S->reqs.at(S->queue.front()).get();
        SrvGraph* G = S->graphs[(size_t)r->gid].get();
        if (G->loading) return nullptr;  // another lane is uploading it
        r->to_queue = queue_eligible(S, r, G);
        r->query_bytes = r->to_queue ? r->queue_bytes : r->lane_bytes;
        const uint64_t gneed = G->g ? 0 : G->resident_bytes + r->upload_bytes;
        const uint64_t need = r->query_bytes + gneed;
        if (S->used + need > S->budget) evict_for(S, need, G);
        if (S->used + need <= S->budget) return r;
        if (S->running == 0) {
            // nothing will free memory: this request can never start
            S->queue.pop_front();
            r->state = RQ_FAILED;
            r->status = BC_ENOMEM;
            r->err = "request footprint exceeds the server memory budget";
            r->t_start = r->t_finish = S->now_ms();
            ++S->failed;
            S->cv.notify_all();
            continue;
        }
        return nullptr;
    }
    return nullptr;
}

void finish_request(bc_server* S, SrvReq* r, SrvGraph* G, bc_status rs, const std::string& err);
bool queue_eligible(bc_server* S, const SrvReq* r, const SrvGraph* G);
bc_status ensure_queue(bc_server* S);

// The server's device queue, or null before its first queued request (it
// is made once and destroyed only after the lanes have ended).
DevQueue* queue_of(bc_server* S) {
    std::lock_guard<std::mutex> lk(S->mu);
    return S->q;
}

void lane_main(bc_server* S, int lane) {
    (void)hipSetDevice(S->device);
    hipStream_t st = S->streams[(size_t)lane];
    std::unique_lock<std::mutex> lk(S->mu);
    for (;;) {
        SrvReq* r = nullptr;
        S->cv.wait(lk, [&] { return S->stop || (r = admit_head(S)) != nullptr; });
        if (!r) {
            if (S->stop) return;
            continue;
        }
        S->queue.pop_front();
        SrvGraph* G = S->graphs[(size_t)r->gid].get();
        const bool upload = G->g == nullptr;
        reserve(S, r->query_bytes + (upload ? G->resident_bytes + r->upload_bytes : 0));
        if (upload) G->loading = true;
        G->refs += 1;
        r->state = RQ_RUNNING;
        r->lane = lane;
        r->uploaded = upload;
        r->t_start = S->now_ms();
        ++S->running;
        const bool to_queue = r->to_queue;
        lk.unlock();

        bc_status rs = BC_OK;
        std::string err;
        if (upload) {
            bc_graph* g = nullptr;
            try {
                // device work of this lane may wait behind a running queue launch
                DevqWait wait(queue_of(S));
                rs = graph_create(G->n, G->m, G->rp.data(), G->m ? G->col.data() : nullptr, G->flags, st, true, &g);
            } catch (...) {
                set_error("internal error");
                rs = BC_EDEVICE;
            }
            if (rs != BC_OK) err = bc_last_error();
            lk.lock();
            G->loading = false;
            S->used -= r->upload_bytes;  // the upload's scratch is gone
            if (rs == BC_OK) {
                G->g = g;
                ++S->uploads;
            } else {
                S->used -= G->resident_bytes;
            }
            S->cv.notify_all();
            lk.unlock();
        }
        if (rs == BC_OK) {
            if (r->o.order == BC_ORDER_GIVEN) r->o.perm = r->perm.data();
            if (r->o.order == BC_ORDER_SCORES) r->o.scores = r->scores.data();
            if (!r->mlp.empty()) r->o.mlp = r->mlp.data();
            if (r->o.nfirst > 0) r->o.first = r->first.data();
            r->ids.assign((size_t)std::max(r->k, 1), 0);
            r->far.assign((size_t)std::max(r->k, 1), 0);
            r->reach.assign((size_t)std::max(r->k, 1), 0);
            std::memset(&r->st, 0, sizeof(r->st));
            r->st.size = sizeof(bc_stats);
            if (to_queue) {
                QueueJob* j = nullptr;
                try {
                    rs = ensure_queue(S);
                    if (rs == BC_OK) rs = devq_submit(S->q, G->g, r->k, r->o, st, &j);
                } catch (...) {
                    set_error("internal error");
                    rs = BC_EDEVICE;
                }
                if (rs == BC_OK) {
                    // the reaper finishes it when the kernel raises its flag
                    lk.lock();
                    r->qjob = j;
                    S->inflight.push_back(r);
                    S->cv.notify_all();
                    continue;
                }
                err = bc_last_error();
            } else {
                try {
                    DevqWait wait(queue_of(S));
                    rs = run_topk(G->g, r->k, r->o, r->ids.data(), r->far.data(), r->reach.data(), &r->count, &r->st,
                                  st, true);
                } catch (...) {
                    set_error("internal error");
                    rs = BC_EDEVICE;
                }
                if (rs != BC_OK) err = bc_last_error();
            }
        }

        lk.lock();
        finish_request(S, r, G, rs, err);
    }
}

// Bookkeeping of a request that has ended (caller holds the lock).
void finish_request(bc_server* S, SrvReq* r, SrvGraph* G, bc_status rs, const std::string& err) {
    --S->running;
    G->refs -= 1;
    G->last_use = ++S->clock;
    S->used -= r->query_bytes;
    r->t_finish = S->now_ms();
    r->status = rs;
    r->err = err;
    if (r->cancel) {
        r->state = RQ_CANCELED;
        ++S->canceled;
    } else if (rs == BC_OK) {
        r->state = RQ_DONE;
        ++S->completed;
    } else {
        r->state = RQ_FAILED;
        ++S->failed;
    }
    S->cv.notify_all();
}

// Whether a request goes to the device queue (caller holds the lock): batched
// requests whose k and graph fit the queue's result areas and slots.
bool queue_eligible(bc_server* S, const SrvReq* r, const SrvGraph* G) {
    if (!S->queue_mode || S->q_failed || r->o.mode != BC_MODE_BATCHED || r->k > kQueueMaxK || G->n <= 0) return false;
    if (S->q) return G->n <= devq_ncap(S->q);
    return true;  // the queue is sized for the largest registered graph when it is made
}

// Make the device queue on first use: slots sized for the largest graph
// registered so far.  Its memory is reserved in the budget for the server's
// lifetime.
bc_status ensure_queue(bc_server* S) {
    static std::mutex make_mu;
    std::lock_guard<std::mutex> mk(make_mu);
    int32_t ncap = 0;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        if (S->q) return BC_OK;
        for (auto& G : S->graphs) ncap = std::max(ncap, G->n);
    }
    // at most half the budget for the queue's node records
    const uint64_t SW = S->queue_width == 64 ? 4 : (S->queue_width == 128 ? 8 : 16);
    const uint64_t per_slot = (uint64_t)std::max(ncap, 1) * (8 * SW + 12) + 4;
    int slots = S->queue_slots;
    if (slots <= 0) {
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
        slots = cus;
    }
    slots = (int)std::max<uint64_t>(1, std::min<uint64_t>((uint64_t)slots, S->budget / 2 / per_slot));
    DevQueue* q = nullptr;
    uint64_t bytes = 0;
    const bc_status rs = devq_create(S->queue_width, ncap, slots, &q, &bytes);
    std::lock_guard<std::mutex> lk(S->mu);
    if (rs != BC_OK) {
        S->q_failed = true;
        return rs;
    }
    S->q = q;
    S->q_bytes = bytes;
    reserve(S, bytes);
    return BC_OK;
}

// Reaper: finishes queued requests whose flag the kernel has raised, and
// relaunches the kernel when it has ended with requests still waiting.
void reaper_main(bc_server* S) {
    (void)hipSetDevice(S->device);
    std::unique_lock<std::mutex> lk(S->mu);
    double stop_ms = -1.0;
    for (;;) {
        if (S->inflight.empty()) {
            if (S->reaper_stop) return;
            S->cv.wait_for(lk, std::chrono::milliseconds(20));
            continue;
        }
        if (S->reaper_stop) {
            // shutting down: give the queued requests a minute to finish, then
            // fail them; their memory is freed only after the kernel has ended
            if (stop_ms < 0) stop_ms = S->now_ms();
            if (S->now_ms() - stop_ms > 60000.0) {
                for (SrvReq* r : S->inflight) {
                    S->orphans.push_back(r->qjob);
                    r->qjob = nullptr;
                    finish_request(S, r, S->graphs[(size_t)r->gid].get(), BC_EDEVICE,
                                   "queued request did not finish before the server was destroyed");
                }
                S->inflight.clear();
                return;
            }
        }
        for (size_t i = 0; i < S->inflight.size();) {
            SrvReq* r = S->inflight[i];
            if (!devq_done(S->q, r->qjob)) {
                (void)devq_advance(S->q, r->qjob);
                ++i;
                continue;
            }
            SrvGraph* G = S->graphs[(size_t)r->gid].get();
            const double qms = S->now_ms() - r->t_start;
            bc_status rs = devq_collect(S->q, r->qjob, r->ids.data(), r->far.data(), r->reach.data(), &r->count,
                                        &r->st, qms);
            const std::string err = rs == BC_OK ? std::string() : std::string(bc_last_error());
            devq_release(S->q, r->qjob);
            r->qjob = nullptr;
            S->inflight[i] = S->inflight.back();
            S->inflight.pop_back();
            finish_request(S, r, G, rs, err);
        }
        if (!S->inflight.empty()) {
            DevQueue* q = S->q;
            lk.unlock();
            const bc_status ps = devq_pump(q);
            std::this_thread::sleep_for(std::chrono::microseconds(100));
            lk.lock();
            if (ps != BC_OK) {
                // the kernel cannot be launched: fail what waits on it
                const std::string err = bc_last_error();
                for (SrvReq* r : S->inflight) {
                    devq_release(S->q, r->qjob);
                    r->qjob = nullptr;
                    finish_request(S, r, S->graphs[(size_t)r->gid].get(), ps, err);
                }
                S->inflight.clear();
            }
        }
    }
}

}  // namespace
}  // namespace bc

using bc::set_error;

#define SRV_GUARD_BEGIN try {
#define SRV_GUARD_END                                  \
    }                                                  \
    catch (const std::bad_alloc&) {                    \
        set_error("host allocation failed");           \
        return BC_ENOMEM;                              \
    }                                                  \
    catch (...) {                                      \
        set_error("internal error");                   \
        return BC_EDEVICE;                             \
    }

extern "C" {

void bc_server_opts_default(bc_server_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->size = sizeof(bc_server_opts);
    o->lanes = 4;
    o->slots = 64;
    o->budget_bytes = 0;
    o->device = -1;
    o->queue = 0;
    o->queue_width = 64;
    o->queue_slots = 0;
}

bc_status bc_footprint(int32_t n, int64_t m, uint32_t flags, int32_t k, const bc_opts* opts, int32_t slots,
                       uint64_t* graph_bytes, uint64_t* upload_bytes, uint64_t* query_bytes) {
    if (n < 0 || m < 0 || !graph_bytes || !upload_bytes || !query_bytes) {
        set_error("bad argument");
        return BC_EINVAL;
    }
    bc_opts o;
    bc_opts_default(&o);
    if (opts) std::memcpy(&o, opts, std::min<size_t>(opts->size ? opts->size : sizeof(bc_opts), sizeof(bc_opts)));
    bc::footprint(n, m, (flags & BC_DIRECTED) != 0, k, o, slots, graph_bytes, upload_bytes, query_bytes);
    return BC_OK;
}

bc_status bc_server_create(const bc_server_opts* opts, bc_server** out) {
    SRV_GUARD_BEGIN
    if (!out) { set_error("out is NULL"); return BC_EINVAL; }
    *out = nullptr;
    bc_server_opts o;
    bc_server_opts_default(&o);
    if (opts) std::memcpy(&o, opts, std::min<size_t>(opts->size ? opts->size : sizeof(o), sizeof(o)));
    if (o.lanes < 1 || o.lanes > 16) { set_error("lanes must be in [1, 16]"); return BC_EINVAL; }
    if (o.slots < 1) { set_error("slots must be positive"); return BC_EINVAL; }
    std::unique_ptr<bc_server> S(new bc_server());
    if (o.device >= 0) BC_HIP(hipSetDevice(o.device));
    BC_HIP(hipGetDevice(&S->device));
    bc::prepare_pool();
    size_t freeb = 0, totalb = 0;
    BC_HIP(hipMemGetInfo(&freeb, &totalb));
    S->budget = o.budget_bytes > 0 ? o.budget_bytes : (uint64_t)(0.45 * (double)freeb);
    S->lanes = o.lanes;
    S->slots = o.slots;
    S->queue_mode = o.queue != 0;
    S->queue_width = o.queue_width;
    S->queue_slots = o.queue_slots;
    if (S->queue_mode && o.queue_width != 64 && o.queue_width != 128 && o.queue_width != 256) {
        set_error("queue_width must be 64, 128 or 256");
        return BC_EINVAL;
    }
    S->t0 = std::chrono::steady_clock::now();
    for (int i = 0; i < S->lanes; ++i) {
        hipStream_t st = nullptr;
        BC_HIP(hipStreamCreateWithFlags(&st, hipStreamNonBlocking));  // default priority
        S->streams.push_back(st);
    }
    for (int i = 0; i < S->lanes; ++i) S->workers.emplace_back(bc::lane_main, S.get(), i);
    if (S->queue_mode) S->reaper = std::thread(bc::reaper_main, S.get());
    *out = S.release();
    return BC_OK;
    SRV_GUARD_END
}

bc_status bc_server_destroy(bc_server* S) {
    SRV_GUARD_BEGIN
    if (!S) return BC_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
        for (uint64_t id : S->queue) {
            auto& r = S->reqs.at(id);
            r->state = bc::RQ_CANCELED;
            ++S->canceled;
        }
        S->queue.clear();
        S->cv.notify_all();
    }
    for (auto& t : S->workers) t.join();
    if (S->reaper.joinable()) {
        // queued requests on the device finish first
        {
            std::lock_guard<std::mutex> lk(S->mu);
            S->reaper_stop = true;
            S->cv.notify_all();
        }
        S->reaper.join();
    }
    if (S->q) bc::devq_destroy(S->q);  // the kernel has ended when this returns
    S->q = nullptr;
    for (bc::QueueJob* j : S->orphans) bc::devq_free(j);
    S->orphans.clear();
    for (auto& G : S->graphs)
        if (G->g) (void)bc_graph_destroy(G->g);
    for (hipStream_t st : S->streams) {
        (void)hipStreamSynchronize(st);
        (void)hipStreamDestroy(st);
    }
    delete S;
    return BC_OK;
    SRV_GUARD_END
}

bc_status bc_server_add_graph(bc_server* S, int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col,
                              uint32_t flags, int32_t* graph_id) {
    SRV_GUARD_BEGIN
    if (!S || !graph_id || !row_ptr || (m > 0 && !col) || n < 0 || m < 0) { set_error("bad argument"); return BC_EINVAL; }
    if (flags & BC_DEVICE_PTRS) { set_error("server graphs take host arrays"); return BC_EINVAL; }
    if (flags & ~(uint32_t)(BC_DIRECTED | BC_VALIDATE | BC_BIG_SCC | BC_KEEP_IDS)) { set_error("unknown flag bits"); return BC_EINVAL; }
    if (row_ptr[0] != 0 || (int64_t)row_ptr[n] != m) { set_error("row_ptr[0] must be 0 and row_ptr[n] = m"); return BC_EGRAPH; }
    std::unique_ptr<bc::SrvGraph> G(new bc::SrvGraph());
    G->n = n;
    G->m = m;
    G->flags = flags;
    G->rp.assign(row_ptr, row_ptr + (size_t)n + 1);
    G->col.assign(col, col + (size_t)m);
    bc_opts o;
    bc_opts_default(&o);
    uint64_t ub = 0, qb = 0;
    bc::footprint(n, m, (flags & BC_DIRECTED) != 0, 1, o, 1, &G->resident_bytes, &ub, &qb);
    std::lock_guard<std::mutex> lk(S->mu);
    *graph_id = (int32_t)S->graphs.size();
    S->graphs.push_back(std::move(G));
    return BC_OK;
    SRV_GUARD_END
}

bc_status bc_submit(bc_server* S, int32_t graph_id, int32_t k, const bc_opts* opts, uint64_t* ticket) {
    SRV_GUARD_BEGIN
    if (!S || !ticket) { set_error("bad argument"); return BC_EINVAL; }
    if (k <= 0) { set_error("k must be positive (got %d)", k); return BC_EINVAL; }
    std::unique_ptr<bc::SrvReq> r(new bc::SrvReq());
    bc_opts_default(&r->o);
    if (opts) {
        if (opts->size < sizeof(uint32_t) || opts->size > sizeof(bc_opts)) { set_error("opts.size not supported"); return BC_EINVAL; }
        std::memcpy(&r->o, opts, opts->size);
        r->o.size = sizeof(bc_opts);
    }
    std::lock_guard<std::mutex> lk(S->mu);
    if (graph_id < 0 || (size_t)graph_id >= S->graphs.size()) { set_error("unknown graph id %d", graph_id); return BC_EINVAL; }
    bc::SrvGraph* G = S->graphs[(size_t)graph_id].get();
    // deep copies of the host arrays the options point at
    if (r->o.order == BC_ORDER_GIVEN) {
        if (!r->o.perm) { set_error("BC_ORDER_GIVEN needs opts.perm"); return BC_EINVAL; }
        r->perm.assign(r->o.perm, r->o.perm + G->n);
    }
    if (r->o.order == BC_ORDER_SCORES) {
        if (!r->o.scores) { set_error("BC_ORDER_SCORES needs opts.scores"); return BC_EINVAL; }
        r->scores.assign(r->o.scores, r->o.scores + G->n);
    }
    if (r->o.mlp) r->mlp.assign(r->o.mlp, r->o.mlp + BC_MLP_PARAMS);
    if (r->o.nfirst < 0 || r->o.nfirst > G->n) { set_error("opts.nfirst %d outside [0, n]", r->o.nfirst); return BC_EINVAL; }
    if (r->o.nfirst > 0) {
        if (!r->o.first) { set_error("opts.first is NULL with nfirst = %d", r->o.nfirst); return BC_EINVAL; }
        r->first.assign(r->o.first, r->o.first + r->o.nfirst);
    }
    r->o.first = nullptr;
    r->o.perm = nullptr;
    r->o.scores = nullptr;
    r->o.mlp = nullptr;
    r->gid = graph_id;
    r->k = k;
    uint64_t gb = 0, ub = 0, qb = 0;
    bc::footprint(G->n, G->m, (G->flags & BC_DIRECTED) != 0, k, r->o, S->slots, &gb, &ub, &qb);
    if (r->o.mode == BC_MODE_BATCHED && r->o.slots <= 0) r->o.slots = S->slots;
    (void)gb;  // the graph's resident bytes were fixed when it was registered
    r->lane_bytes = qb;
    r->queue_bytes = bc::queue_request_bytes(G->n, k, r->o);
    r->query_bytes = qb;
    r->upload_bytes = ub;
    r->id = S->next_id++;
    r->t_submit = S->now_ms();
    *ticket = r->id;
    S->queue.push_back(r->id);
    S->reqs.emplace(r->id, std::move(r));
    S->cv.notify_all();
    return BC_OK;
    SRV_GUARD_END
}

bc_status bc_wait(bc_server* S, uint64_t ticket, int32_t timeout_ms) {
    SRV_GUARD_BEGIN
    if (!S) { set_error("server is NULL"); return BC_EINVAL; }
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) { set_error("unknown ticket"); return BC_EINVAL; }
    bc::SrvReq* r = it->second.get();
    auto pred = [&] { return r->state >= bc::RQ_DONE; };
    if (timeout_ms < 0) S->cv.wait(lk, pred);
    else if (!S->cv.wait_for(lk, std::chrono::milliseconds(timeout_ms), pred)) return BC_EAGAIN;
    return BC_OK;
    SRV_GUARD_END
}

bc_status bc_poll(bc_server* S, uint64_t ticket, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* count,
                  bc_stats* stats, bc_request_info* info) {
    SRV_GUARD_BEGIN
    if (!S) { set_error("server is NULL"); return BC_EINVAL; }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) { set_error("unknown ticket"); return BC_EINVAL; }
    bc::SrvReq* r = it->second.get();
    if (r->state < bc::RQ_DONE) return BC_EAGAIN;
    if (info) {
        bc_request_info ri;
        std::memset(&ri, 0, sizeof(ri));
        ri.size = sizeof(ri);
        ri.lane = r->lane;
        ri.uploaded = r->uploaded ? 1 : 0;
        ri.submit_ms = r->t_submit;
        ri.start_ms = r->t_start;
        ri.finish_ms = r->t_finish;
        ri.footprint_bytes = r->query_bytes;
        std::memcpy(info, &ri, std::min<size_t>(info->size ? info->size : sizeof(ri), sizeof(ri)));
    }
    bc_status rs;
    if (r->state == bc::RQ_CANCELED) {
        set_error("request was cancelled");
        rs = BC_ECANCELED;
    } else if (r->state == bc::RQ_FAILED) {
        set_error("%s", r->err.c_str());
        rs = r->status;
    } else {
        if (!ids || !farness || !reach || !count) { set_error("NULL output array"); return BC_EINVAL; }
        for (int32_t i = 0; i < r->count; ++i) {
            ids[i] = r->ids[(size_t)i];
            farness[i] = r->far[(size_t)i];
            reach[i] = r->reach[(size_t)i];
        }
        *count = r->count;
        if (stats) {
            const uint32_t sz = stats->size ? stats->size : sizeof(bc_stats);
            std::memcpy(stats, &r->st, std::min<size_t>(sz, sizeof(bc_stats)));
        }
        rs = BC_OK;
    }
    S->reqs.erase(it);
    return rs;
    SRV_GUARD_END
}

bc_status bc_progress(bc_server* S, uint64_t ticket, uint64_t* done_batches, uint64_t* total_batches) {
    SRV_GUARD_BEGIN
    if (!S || !done_batches || !total_batches) { set_error("bad argument"); return BC_EINVAL; }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) { set_error("unknown ticket"); return BC_EINVAL; }
    bc::SrvReq* r = it->second.get();
    *done_batches = 0;
    *total_batches = 0;
    if (r->qjob && S->q) bc::devq_progress(S->q, r->qjob, done_batches, total_batches);
    return BC_OK;
    SRV_GUARD_END
}

bc_status bc_cancel(bc_server* S, uint64_t ticket) {
    SRV_GUARD_BEGIN
    if (!S) { set_error("server is NULL"); return BC_EINVAL; }
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) { set_error("unknown ticket"); return BC_EINVAL; }
    bc::SrvReq* r = it->second.get();
    if (r->state == bc::RQ_QUEUED) {
        for (auto q = S->queue.begin(); q != S->queue.end(); ++q)
            if (*q == ticket) {
                S->queue.erase(q);
                break;
            }
        r->state = bc::RQ_CANCELED;
        r->t_start = r->t_finish = S->now_ms();
        ++S->canceled;
        S->cv.notify_all();
    } else if (r->state == bc::RQ_RUNNING) {
        r->cancel = true;  // runs to its end; the result is dropped
    } else {
        set_error("request already finished");
        return BC_EINVAL;
    }
    return BC_OK;
    SRV_GUARD_END
}

bc_status bc_server_info(bc_server* S, bc_server_stats* out) {
    if (!S || !out) { set_error("bad argument"); return BC_EINVAL; }
    std::lock_guard<std::mutex> lk(S->mu);
    bc_server_stats t;
    std::memset(&t, 0, sizeof(t));
    t.size = sizeof(t);
    t.budget_bytes = S->budget;
    t.used_bytes = S->used;
    t.peak_bytes = S->peak;
    for (auto& G : S->graphs) t.resident_graphs += G->g ? 1 : 0;
    t.graphs = (uint32_t)S->graphs.size();
    t.queued = (uint32_t)S->queue.size();
    t.running = (uint32_t)S->running;
    t.uploads = S->uploads;
    t.evictions = S->evictions;
    t.completed = S->completed;
    t.failed = S->failed;
    t.canceled = S->canceled;
    t.queue_inflight = S->inflight.size();
    if (S->q) {
        t.queue_launches = bc::devq_launches(S->q);
        t.queue_batches = bc::devq_published(S->q);
    }
    std::memcpy(out, &t, std::min<size_t>(out->size ? out->size : sizeof(t), sizeof(t)));
    return BC_OK;
}

}  // extern "C"
