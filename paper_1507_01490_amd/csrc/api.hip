// C ABI of the library (declared in include/bfscut.h).  Every entry point
// returns a bc_status and never lets a C++ exception cross the boundary.
#include <algorithm>
#include <cstdarg>
#include <vector>
#include <cstdio>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>

#include "bc_internal.h"

namespace bc {

static thread_local char g_err[512];

void prepare_pool() {
    static std::mutex mu;
    static bool done[64] = {};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return;
    std::lock_guard<std::mutex> lk(mu);
    if (done[dev]) return;
    done[dev] = true;
    hipMemPool_t pool;
    if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
        uint64_t keep = ~0ull;  // freed blocks stay in the pool for the next query
        (void)hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &keep);
    }
    (void)hipGetLastError();
}

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

constexpr int32_t kRelabelMinNodes = 100000;  // undirected graphs of this many nodes or more are renumbered

bc_status graph_create(int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col, uint32_t flags,
                       hipStream_t stream, bool ordered, bc_graph** out) {
    if (!out) { set_error("out is NULL"); return BC_EINVAL; }
    *out = nullptr;
    if (n < 0 || m < 0) { set_error("negative size"); return BC_EINVAL; }
    if (!row_ptr || (m > 0 && !col)) { set_error("row_ptr/col is NULL"); return BC_EINVAL; }
    if (flags & ~(uint32_t)(BC_DIRECTED | BC_VALIDATE | BC_DEVICE_PTRS | BC_BIG_SCC | BC_KEEP_IDS)) {
        set_error("unknown flag bits");
        return BC_EINVAL;
    }
    std::unique_ptr<bc_graph> g(new bc_graph());
    g->stream = stream;
    g->ordered = ordered;
    (void)hipGetDevice(&g->device);
    bc_status s = graph_build(g.get(), n, m, row_ptr, col, flags & ~(uint32_t)BC_KEEP_IDS);
    if (s != BC_OK) {
        (void)hipStreamSynchronize(g->stream);
        return s;
    }
    // small graphs keep their numbering: their node records stay in the
    // caches anyway, and the second build would dominate their upload
    if (!(flags & (BC_DIRECTED | BC_KEEP_IDS)) && n >= kRelabelMinNodes) {
        bc_graph* h = nullptr;
        s = graph_relabel(g.get(), flags & ~(uint32_t)(BC_DEVICE_PTRS | BC_KEEP_IDS | BC_VALIDATE), ordered, &h);
        (void)hipStreamSynchronize(g->stream);
        if (s != BC_OK) return s;
        g.reset(h);
    }
    *out = g.release();
    return BC_OK;
}

}  // namespace bc

using bc::set_error;

#define BC_GUARD_BEGIN try {
#define BC_GUARD_END                                   \
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

const char* bc_last_error(void) { return bc::g_err; }

const char* bc_version(void) { return "bfscut-gfx950 0.1"; }

void bc_opts_default(bc_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->size = sizeof(bc_opts);
    o->mode = BC_MODE_PLAIN;
    o->order = BC_ORDER_AUTO;
    o->width = 64;
    o->perm = nullptr;
    o->scores = nullptr;
    o->pull_alpha = 3.f;
    o->pull_beta = 24.f;
    o->slots = 0;
    o->seed_batches = -1;
    o->chunk = 0;
    o->defer_arcs = 0;
    o->mlp = nullptr;
    o->graph_levels = 0;
}

bc_status bc_graph_create(int32_t n, int64_t m, const int32_t* row_ptr, const int32_t* col, uint32_t flags,
                          void* stream, bc_graph** out) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    return bc::graph_create(n, m, row_ptr, col, flags, (hipStream_t)stream, false, out);
    BC_GUARD_END
}

bc_status bc_graph_destroy(bc_graph* g) {
    BC_GUARD_BEGIN
    if (!g) return BC_OK;
    (void)hipStreamSynchronize(g->stream);
    delete g;
    return BC_OK;
    BC_GUARD_END
}

bc_status bc_graph_info(const bc_graph* g, int32_t* n, int64_t* m, int32_t* directed, double* preprocess_ms) {
    if (!g) { set_error("graph is NULL"); return BC_EINVAL; }
    if (n) *n = g->dg.n;
    if (m) *m = g->dg.m;
    if (directed) *directed = g->dg.directed;
    if (preprocess_ms) *preprocess_ms = g->preprocess_ms;
    return BC_OK;
}

bc_status bc_graph_reach(const bc_graph* g, uint32_t* lo, uint32_t* hi) {
    BC_GUARD_BEGIN
    if (!g) { set_error("graph is NULL"); return BC_EINVAL; }
    bc_graph* gg = const_cast<bc_graph*>(g);
    size_t bytes = sizeof(uint32_t) * (size_t)g->dg.n;
    if (bytes == 0) return BC_OK;
    // per node in the caller's numbering
    bc::DevBuf t;
    BC_TRY(t.alloc_on(bytes, g->stream));
    if (lo) {
        BC_TRY(bc::rows_to_caller(gg, g->dg.x0, t.p, 1, g->stream));
        BC_HIP(hipMemcpyAsync(lo, t.p, bytes, hipMemcpyDeviceToHost, g->stream));
        BC_HIP(hipStreamSynchronize(g->stream));
    }
    if (hi) {
        BC_TRY(bc::rows_to_caller(gg, g->dg.x1, t.p, 1, g->stream));
        BC_HIP(hipMemcpyAsync(hi, t.p, bytes, hipMemcpyDeviceToHost, g->stream));
        BC_HIP(hipStreamSynchronize(g->stream));
    }
    return BC_OK;
    BC_GUARD_END
}

bc_status bc_graph_csr(const bc_graph* g, int32_t* row_ptr, int32_t* col) {
    BC_GUARD_BEGIN
    if (!g) { set_error("graph is NULL"); return BC_EINVAL; }
    const size_t n = (size_t)g->dg.n, m = (size_t)g->dg.m;
    std::vector<int32_t> rp(n + 1), cl(m > 0 ? m : 1);
    BC_HIP(hipMemcpyAsync(rp.data(), g->dg.rp, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, g->stream));
    if (m > 0) BC_HIP(hipMemcpyAsync(cl.data(), g->dg.col, sizeof(int32_t) * m, hipMemcpyDeviceToHost, g->stream));
    BC_HIP(hipStreamSynchronize(g->stream));
    if (!g->relabeled) {
        if (row_ptr) std::memcpy(row_ptr, rp.data(), sizeof(int32_t) * (n + 1));
        if (col && m > 0) std::memcpy(col, cl.data(), sizeof(int32_t) * m);
        return BC_OK;
    }
    // the canonical CSR in the caller's numbering: row v is our row inv[v]
    // with every target renamed by orig, sorted
    std::vector<int32_t> orig(n), inv(n);
    BC_HIP(hipMemcpyAsync(orig.data(), g->orig.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, g->stream));
    BC_HIP(hipMemcpyAsync(inv.data(), g->inv.p, sizeof(int32_t) * n, hipMemcpyDeviceToHost, g->stream));
    BC_HIP(hipStreamSynchronize(g->stream));
    std::vector<int32_t> orp(n + 1, 0), ocol(m > 0 ? m : 1);
    for (size_t v = 0; v < n; ++v) orp[v + 1] = orp[v] + (rp[(size_t)inv[v] + 1] - rp[(size_t)inv[v]]);
    for (size_t v = 0; v < n; ++v) {
        const int32_t u = inv[v];
        int32_t* dst = ocol.data() + orp[v];
        for (int32_t e = rp[(size_t)u]; e < rp[(size_t)u + 1]; ++e) *dst++ = orig[(size_t)cl[(size_t)e]];
        std::sort(ocol.data() + orp[v], ocol.data() + orp[v + 1]);
    }
    if (row_ptr) std::memcpy(row_ptr, orp.data(), sizeof(int32_t) * (n + 1));
    if (col && m > 0) std::memcpy(col, ocol.data(), sizeof(int32_t) * m);
    return BC_OK;
    BC_GUARD_END
}

static bc_status copy_opts(const bc_opts* opts, bc_opts* o) {
    bc_opts_default(o);
    if (opts) {
        if (opts->size < sizeof(uint32_t) || opts->size > sizeof(bc_opts)) {
            set_error("opts.size %u not supported", opts->size);
            return BC_EINVAL;
        }
        std::memcpy(o, opts, opts->size);
        o->size = sizeof(bc_opts);
        if (o->bounds & ~(uint32_t)(BC_BOUND_FOOTNOTE | BC_BOUND_NO_TRIAL)) {
            set_error("unknown bounds bits 0x%x", o->bounds);
            return BC_EINVAL;
        }
    }
    return BC_OK;
}

bc_status bc_topk(bc_graph* g, int32_t k, const bc_opts* opts, int32_t* ids, uint64_t* farness, uint32_t* reach,
                  int32_t* count, bc_stats* stats) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    if (!g) { set_error("graph is NULL"); return BC_EINVAL; }
    if (k <= 0) { set_error("k must be positive (got %d)", k); return BC_EINVAL; }
    if (!ids || !farness || !reach || !count) { set_error("NULL output array"); return BC_EINVAL; }
    bc_opts o;
    BC_TRY(copy_opts(opts, &o));
    return bc::run_topk(g, k, o, ids, farness, reach, count, stats, g->stream);
    BC_GUARD_END
}

bc_status bc_topk_static(bc_graph* g, int32_t k, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* count) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    if (!g) { set_error("graph is NULL"); return BC_EINVAL; }
    if (k <= 0) { set_error("k must be positive (got %d)", k); return BC_EINVAL; }
    if (!ids || !farness || !reach || !count) { set_error("NULL output array"); return BC_EINVAL; }
    return bc::run_topk_static(g, k, ids, farness, reach, count);
    BC_GUARD_END
}

bc_status bc_farness_all(bc_graph* g, const bc_opts* opts, uint64_t* farness, uint32_t* reach, bc_stats* stats) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    if (!g) { set_error("graph is NULL"); return BC_EINVAL; }
    if (g->dg.n > 0 && (!farness || !reach)) { set_error("NULL output array"); return BC_EINVAL; }
    bc_opts o;
    BC_TRY(copy_opts(opts, &o));
    return bc::run_farness_all(g, o, farness, reach, stats, g->stream);
    BC_GUARD_END
}

bc_status bc_source_order(bc_graph* g, int32_t k, const bc_opts* opts, int32_t* order) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    if (!g) { set_error("graph is NULL"); return BC_EINVAL; }
    if (k <= 0) { set_error("k must be positive (got %d)", k); return BC_EINVAL; }
    const int32_t n = g->dg.n;
    if (n > 0 && !order) { set_error("order is NULL"); return BC_EINVAL; }
    bc_opts o;
    BC_TRY(copy_opts(opts, &o));
    if (o.width != 64 && o.width != 128 && o.width != 256) {
        set_error("width must be 64, 128 or 256 (got %d)", o.width);
        return BC_EINVAL;
    }
    if (n == 0) return BC_OK;
    bc::DevBuf d;
    BC_TRY(d.alloc_on(sizeof(int32_t) * (size_t)n, g->stream));
    BC_TRY(bc::build_order(g, o, std::min(k, n), d.as<int32_t>(), g->stream));
    BC_TRY(bc::ids_to_caller(g, d.as<int32_t>(), n, g->stream));
    BC_HIP(hipMemcpyAsync(order, d.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost, g->stream));
    BC_HIP(hipStreamSynchronize(g->stream));
    return BC_OK;
    BC_GUARD_END
}

static bc_status check_multi(bc_graph* const* graphs, int32_t count, const int32_t* ks, const bc_opts* opts,
                             bc_opts* o) {
    if (count < 1) { set_error("count must be positive (got %d)", count); return BC_EINVAL; }
    if (!graphs || !ks) { set_error("graphs/ks is NULL"); return BC_EINVAL; }
    BC_TRY(copy_opts(opts, o));
    if (o->nfirst != 0) { set_error("opts.first is not supported by job launches"); return BC_EINVAL; }
    if (o->order == BC_ORDER_GIVEN || o->order == BC_ORDER_SCORES) {
        set_error("per-graph orders are not supported by job launches (order %d)", o->order);
        return BC_EINVAL;
    }
    return BC_OK;
}

bc_status bc_multi_create(bc_graph* const* graphs, int32_t count, const int32_t* ks, const bc_opts* opts,
                          int32_t capture, void* stream, bc_multi** out) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    if (!out) { set_error("out is NULL"); return BC_EINVAL; }
    *out = nullptr;
    bc_opts o;
    BC_TRY(check_multi(graphs, count, ks, opts, &o));
    return bc::multi_create(graphs, count, ks, o, (hipStream_t)stream, capture != 0, out);
    BC_GUARD_END
}

bc_status bc_multi_run(bc_multi* p, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* counts,
                       bc_stats* stats) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    if (!p) { set_error("launch is NULL"); return BC_EINVAL; }
    if (!ids || !farness || !reach || !counts) { set_error("NULL output array"); return BC_EINVAL; }
    return bc::multi_run(p, ids, farness, reach, counts, stats);
    BC_GUARD_END
}

bc_status bc_multi_destroy(bc_multi* p) {
    BC_GUARD_BEGIN
    if (p) bc::multi_destroy(p);
    return BC_OK;
    BC_GUARD_END
}

bc_status bc_topk_multi(bc_graph* const* graphs, int32_t count, const int32_t* ks, const bc_opts* opts,
                        int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* counts, bc_stats* stats) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    bc_opts o;
    BC_TRY(check_multi(graphs, count, ks, opts, &o));
    if (!ids || !farness || !reach || !counts) { set_error("NULL output array"); return BC_EINVAL; }
    for (int32_t i = 0; i < count; ++i)
        if (!graphs[i]) { set_error("graph %d is NULL", i); return BC_EINVAL; }
    bc_multi* p = nullptr;
    BC_TRY(bc::multi_create(graphs, count, ks, o, graphs[0]->stream, false, &p));
    const bc_status rs = bc::multi_run(p, ids, farness, reach, counts, stats);
    bc::multi_destroy(p);
    return rs;
    BC_GUARD_END
}

bc_status bc_graph_features(bc_graph* g, float* x, uint32_t* core) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    if (!g) { set_error("graph is NULL"); return BC_EINVAL; }
    if (!x) { set_error("x is NULL"); return BC_EINVAL; }
    BC_TRY(bc::graph_features(g, g->stream));
    const size_t n = (size_t)g->dg.n;
    if (n == 0) return BC_OK;
    // rows in the caller's numbering
    bc::DevBuf t;
    BC_TRY(t.alloc_on(sizeof(float) * 3 * n, g->stream));
    BC_TRY(bc::rows_to_caller(g, g->feat.p, t.p, 3, g->stream));
    BC_HIP(hipMemcpyAsync(x, t.p, sizeof(float) * 3 * n, hipMemcpyDefault, g->stream));
    if (core) {
        BC_HIP(hipStreamSynchronize(g->stream));
        BC_TRY(bc::rows_to_caller(g, g->core.p, t.p, 1, g->stream));
        BC_HIP(hipMemcpyAsync(core, t.p, sizeof(uint32_t) * n, hipMemcpyDefault, g->stream));
    }
    BC_HIP(hipStreamSynchronize(g->stream));
    return BC_OK;
    BC_GUARD_END
}

bc_status bc_mlp_forward(const float* params, const float* x, int64_t count, float* y, void* stream) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    if (count < 0) { set_error("negative count"); return BC_EINVAL; }
    if (count > 0 && (!params || !x || !y)) { set_error("NULL pointer"); return BC_EINVAL; }
    return bc::mlp_forward(params, x, count, y, (hipStream_t)stream);
    BC_GUARD_END
}

bc_status bc_mlp_loss_grad(const float* params, const float* x, const float* t, const float* w, int64_t rows,
                           const int32_t* idx, int64_t count, float* grad, double* loss, void* stream) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    if (count < 0 || rows < 0) { set_error("negative size"); return BC_EINVAL; }
    if (!params || !grad || (count > 0 && (!x || !t))) { set_error("NULL pointer"); return BC_EINVAL; }
    return bc::mlp_loss_grad(params, x, t, w, rows, idx, count, grad, loss, (hipStream_t)stream);
    BC_GUARD_END
}

bc_status bc_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                      float beta2, float eps, void* stream) {
    BC_GUARD_BEGIN
    bc::g_err[0] = 0;
    if (!params || !grad || !m || !v) { set_error("NULL pointer"); return BC_EINVAL; }
    if (step < 1) { set_error("step must be >= 1"); return BC_EINVAL; }
    if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f)) { set_error("betas outside [0, 1)"); return BC_EINVAL; }
    return bc::mlp_adam(params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
    BC_GUARD_END
}

}  // extern "C"
