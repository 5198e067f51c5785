// Pre-processing step of the method (linear time, done once per graph):
//   * CSR validation and canonical form (rows sorted, self-loops and repeated
//     arcs removed; neither changes a distance),
//   * out-degrees, and the in-CSR of a directed graph,
//   * reach data: for an undirected graph r(v) is the size of v's connected
//     component (Section 2.3); for a directed graph alpha(v) <= r(v) <=
//     omega(v) come from the weighted DAG of strongly connected components
//     (Section 2.4), see scc.hip.
//   * source orders for Algorithm 1 (decreasing degree, given, or scored).
#include <hipcub/hipcub.hpp>

#include <algorithm>
#include <cstring>
#include <chrono>

#include "bc_internal.h"

namespace bc {

bc_status directed_reach(bc_graph* g);  // scc.hip

namespace {

constexpr int kBlk = 256;

inline unsigned grid_for(int64_t work, int64_t cap = 8192) {
    int64_t b = (work + kBlk - 1) / kBlk;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

__device__ inline int32_t ld_relaxed(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st_relaxed(int32_t* p, int32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// err bits: 1 bad row_ptr, 2 col out of range, 4 not canonical, 8 not symmetric
__global__ void k_validate(int32_t n, int64_t m, const int32_t* __restrict__ rp,
                           const int32_t* __restrict__ col, uint32_t* err) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n; u += stride) {
        int32_t b = rp[u];
        if (u == 0 && b != 0) atomicOr(err, 1u);
        if (u == n) {
            if ((int64_t)b != m) atomicOr(err, 1u);
            continue;
        }
        int32_t e = rp[u + 1];
        if (e < b || b < 0 || (int64_t)e > m) {
            atomicOr(err, 1u);
            continue;
        }
        uint32_t bits = 0;
        int32_t prev = -1;
        for (int32_t i = b; i < e; ++i) {
            int32_t w = col[i];
            if (w < 0 || w >= n) { bits |= 2u; break; }
            if (w == (int32_t)u || w <= prev) bits |= 4u;
            prev = w;
        }
        if (bits) atomicOr(err, bits);
    }
}

// keep[i] = 1 for the first copy of each non-loop arc of a sorted row
__global__ void k_mark_keep(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            int32_t* __restrict__ cnt) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        int32_t c = 0, prev = -1;
        for (int32_t i = rp[u]; i < rp[u + 1]; ++i) {
            int32_t w = col[i];
            if (w != (int32_t)u && w != prev) ++c;
            prev = w;
        }
        cnt[u] = c;
    }
}

__global__ void k_compact_rows(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                               const int32_t* __restrict__ nrp, int32_t* __restrict__ ncol) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        int32_t o = nrp[u], prev = -1;
        for (int32_t i = rp[u]; i < rp[u + 1]; ++i) {
            int32_t w = col[i];
            if (w != (int32_t)u && w != prev) ncol[o++] = w;
            prev = w;
        }
    }
}

__global__ void k_set_last(int32_t* nrp, int32_t n, const int32_t* cnt) {
    // nrp holds the exclusive sum of cnt in [0, n); close it with the total
    if (blockIdx.x == 0 && threadIdx.x == 0) nrp[n] = (n > 0 ? nrp[n - 1] + cnt[n - 1] : 0);
}

__global__ void k_degree(int32_t n, const int32_t* __restrict__ rp, uint32_t* __restrict__ deg) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
        deg[u] = (uint32_t)(rp[u + 1] - rp[u]);
}

// undirected symmetry: every arc u->w has its reverse w->u (rows are sorted)
__global__ void k_symmetric(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            uint32_t* err) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        for (int32_t i = rp[u]; i < rp[u + 1]; ++i) {
            int32_t w = col[i];
            int32_t lo = rp[w], hi = rp[w + 1];
            while (lo < hi) {
                int32_t mid = (lo + hi) >> 1;
                if (col[mid] < (int32_t)u) lo = mid + 1; else hi = mid;
            }
            if (lo >= rp[w + 1] || col[lo] != (int32_t)u) { atomicOr(err, 8u); break; }
        }
    }
}

// ---- connected components: lock-free union-find (hook larger root under smaller)

__device__ int32_t uf_find(int32_t* P, int32_t v) {
    for (;;) {
        int32_t p = ld_relaxed(&P[v]);
        if (p == v) return v;
        int32_t gp = ld_relaxed(&P[p]);
        if (gp != p) st_relaxed(&P[v], gp);  // path halving: gp is an ancestor of v
        v = gp;
    }
}

__global__ void k_uf_init(int32_t n, int32_t* P) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) P[u] = (int32_t)u;
}

__global__ void k_uf_union(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           int32_t* P) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        for (int32_t i = rp[u]; i < rp[u + 1]; ++i) {
            int32_t w = col[i];
            if (w < (int32_t)u) continue;  // each undirected edge once
            int32_t a = (int32_t)u, b = w;
            for (;;) {
                a = uf_find(P, a);
                b = uf_find(P, b);
                if (a == b) break;
                if (a < b) { int32_t t = a; a = b; b = t; }
                if (atomicCAS(&P[a], a, b) == a) break;
            }
        }
    }
}

__global__ void k_uf_count(int32_t n, int32_t* P, uint32_t* __restrict__ size, int32_t* __restrict__ label) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        int32_t r = uf_find(P, (int32_t)u);
        label[u] = r;
        atomicAdd(&size[r], 1u);
    }
}

__global__ void k_uf_reach(int32_t n, const int32_t* __restrict__ label, const uint32_t* __restrict__ size,
                           uint32_t* __restrict__ x0, uint32_t* __restrict__ x1) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        uint32_t s = size[label[u]];
        x0[u] = s;
        x1[u] = s;
    }
}

// ---- orders

// adj[e] = (col[e], deg[col[e]])
__global__ void k_pack_adj(int64_t m, const int32_t* __restrict__ col, const uint32_t* __restrict__ deg,
                           int2* __restrict__ adj) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        const int32_t w = col[e];
        adj[e] = make_int2(w, (int32_t)deg[w]);
    }
}

// (decreasing degree, increasing id): the id is the caller's (orig[u]) on a
// renumbered graph, so that the degree order is the same with or without it
__global__ void k_degree_keys(int32_t n, const uint32_t* __restrict__ deg, const int32_t* __restrict__ orig,
                              uint64_t* __restrict__ key) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
        key[u] = ((uint64_t)(0xFFFFFFFFu - deg[u]) << 32) | (uint32_t)(orig ? orig[u] : (int32_t)u);
}

__global__ void k_low32(int32_t n, const uint64_t* __restrict__ key, int32_t* __restrict__ out) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride)
        out[u] = (int32_t)(key[u] & 0xFFFFFFFFu);
}

// hub(v): the out-neighbour of largest out-degree (ties by smaller id), n when
// v has no out-neighbour; key = hub << 32 | v
__global__ void k_hub_keys(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const uint32_t* __restrict__ deg, uint64_t* __restrict__ key) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        int32_t best = n;
        uint32_t bd = 0;
        for (int32_t i = rp[u]; i < rp[u + 1]; ++i) {
            const int32_t w = col[i];
            const uint32_t d = deg[w];
            if (best == n || d > bd || (d == bd && w < best)) {
                best = w;
                bd = d;
            }
        }
        key[u] = ((uint64_t)(uint32_t)best << 32) | (uint32_t)u;
    }
}

__global__ void k_degkey_of(int32_t n, const int32_t* __restrict__ perm, const uint32_t* __restrict__ deg,
                            uint32_t* __restrict__ key) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        key[i] = 0xFFFFFFFFu - deg[perm[i]];
}

// score -> unsigned key whose ascending order is decreasing score
__global__ void k_score_keys(int32_t n, const float* __restrict__ s, const int32_t* __restrict__ order,
                             uint32_t* __restrict__ key) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        uint32_t b = __float_as_uint(s[order[i]]);
        if (b == 0x80000000u) b = 0u;  // -0 ranks with +0
        uint32_t asc = (b & 0x80000000u) ? ~b : (b | 0x80000000u);  // monotone in the float
        key[i] = ~asc;
    }
}

// mark[v] = 1 for the first `head` sources of `order`
__global__ void k_mark_head(int32_t head, const int32_t* __restrict__ order, uint8_t* __restrict__ mark) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < head; i += stride) mark[order[i]] = 1;
}

// keep[i] = the i-th source of `order` is not marked
__global__ void k_keep_unmarked(int32_t n, const int32_t* __restrict__ order, const uint8_t* __restrict__ mark,
                                uint8_t* __restrict__ keep) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) keep[i] = !mark[order[i]];
}

// ---------------------------------------------------------- locality order
//
// Breadth-first discovery order from an approximate centre: consecutive
// sources are neighbours, so a batch of them shares its search, and the
// centre (high closeness) comes first.  Deterministic: each level is sorted
// by (position of the node's earliest parent in the order, id).

// dist[v] = -1, parent position = max
__global__ void k_loc_init(int32_t n, int32_t* __restrict__ dist, uint32_t* __restrict__ ppos) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        dist[v] = -1;
        if (ppos) ppos[v] = 0xFFFFFFFFu;
    }
}

// One level: the out-arcs of F[0, flen) (at distance d, order positions
// base + i) discover level d + 1 into N; with ppos, every parent offers its
// position and the smallest is kept.
__global__ void k_loc_expand(const int32_t* __restrict__ rp, const int32_t* __restrict__ col, const int32_t* F,
                             uint32_t flen, int32_t d, uint32_t base, int32_t* dist, uint32_t* ppos, int32_t* N,
                             uint32_t* ncount) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < flen; i += stride) {
        const int32_t u = F[i];
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            const int32_t w = col[e];
            const int32_t old = atomicCAS(&dist[w], -1, d + 1);
            if (old == -1) N[atomicAdd(ncount, 1u)] = w;
            if (ppos && (old == -1 || old == d + 1)) atomicMin(&ppos[w], base + (uint32_t)i);
        }
    }
}

// keys of a discovered level: (earliest parent position, id)
__global__ void k_loc_keys(uint32_t cnt, const int32_t* __restrict__ N, const uint32_t* __restrict__ ppos,
                           uint64_t* __restrict__ key) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < cnt; j += stride)
        key[j] = ((uint64_t)ppos[N[j]] << 32) | (uint32_t)N[j];
}

// farthest reached node: max (dist, -id) packed; and on-path test for the centre
__global__ void k_loc_far(int32_t n, const int32_t* __restrict__ dist, unsigned long long* best) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        if (dist[v] >= 0)
            atomicMax(best, ((unsigned long long)(uint32_t)dist[v] << 32) | (0xFFFFFFFFu - (uint32_t)v));
}

// centre: on a shortest a-b path (da + db = D), nearest to the middle, smallest id
__global__ void k_loc_centre(int32_t n, const int32_t* __restrict__ da, const int32_t* __restrict__ db, int32_t D,
                             unsigned long long* best) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        if (da[v] < 0 || db[v] < 0 || da[v] + db[v] != D) continue;
        const uint32_t off = (uint32_t)abs(2 * da[v] - D);
        atomicMin(best, ((unsigned long long)off << 32) | (uint32_t)v);
    }
}

__global__ void k_loc_unreached(int32_t n, const int32_t* __restrict__ order_deg, const int32_t* __restrict__ dist,
                                uint8_t* __restrict__ flag) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        flag[i] = dist[order_deg[i]] < 0;
}

// Cuts the breadth-first seed order into compact balls, one batch of B
// positions at a time: take the first seed not yet placed, place it, then its
// unplaced neighbours in queue order (frontier position, then arc order)
// level by level until the batch is full; if its component runs dry, the
// next unplaced seed continues the same batch.  A batch of sources that lie
// within a few hops of each other reaches most nodes at the same or
// neighbouring levels, so the bit-parallel search expands each node for many
// sources at once.  Inherently sequential over batches: one workgroup of
// kCarveThreads walks them; each level's arcs are read in chunks of
// kCarveThreads ordinals, a node's first ordinal (an LDS hash) decides who
// places it.
constexpr int kCarveThreads = 1024;
constexpr int kCarveHash = 2048;  // > kCarveThreads: open addressing never fills

__device__ __forceinline__ uint32_t carve_slot(int32_t w) { return ((uint32_t)w * 2654435761u) >> 21; }

__global__ __launch_bounds__(kCarveThreads) void k_carve(int32_t n, const int32_t* __restrict__ rp,
                                                         const int32_t* __restrict__ col,
                                                         const int32_t* __restrict__ seed, int32_t B,
                                                         uint8_t* taken, int32_t* out, int32_t* err) {
    __shared__ int32_t cur[256], nxt[256];
    __shared__ int64_t pre[257];
    __shared__ int32_t hkey[kCarveHash], hval[kCarveHash];
    __shared__ int32_t wsum[kCarveThreads / 64];
    __shared__ int32_t s_first;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    for (int i = tid; i < kCarveHash; i += kCarveThreads) {
        hkey[i] = -1;
        hval[i] = INT32_MAX;
    }
    __syncthreads();
    int32_t pos = 0;
    int64_t ptr = 0;  // uniform across the workgroup
    while (pos < n) {
        const int32_t bend = (int32_t)min((int64_t)pos + B, (int64_t)n);
        while (pos < bend) {
            // first seed at or after ptr not yet placed (every seed before ptr is)
            for (;;) {
                if (ptr >= n) {  // unreachable while pos < n: the seed order is a permutation
                    if (tid == 0) *err = 1;
                    return;
                }
                if (tid == 0) s_first = INT32_MAX;
                __syncthreads();
                const int64_t idx = (int64_t)ptr + tid;
                if (idx < n && !taken[seed[idx]]) atomicMin(&s_first, (int32_t)idx);
                __syncthreads();
                const int32_t f = s_first;
                __syncthreads();
                if (f != INT32_MAX) {
                    ptr = f;
                    break;
                }
                ptr += kCarveThreads;
            }
            if (tid == 0) {
                const int32_t s0 = seed[ptr];
                taken[s0] = 1;
                out[pos] = s0;
                cur[0] = s0;
            }
            pos += 1;
            int32_t clen = 1;
            __syncthreads();
            while (clen > 0 && pos < bend) {
                // pre[i] = out-arcs of cur[0, i)
                if (wv == 0) {
                    int64_t v[4], sum = 0;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int i = 4 * lane + j;
                        if (i < clen) sum += rp[cur[i] + 1] - rp[cur[i]];
                        v[j] = sum;
                    }
                    int64_t x = sum;
                    for (int o = 1; o < 64; o <<= 1) {
                        const int64_t y = __shfl_up(x, o);
                        if (lane >= o) x += y;
                    }
                    const int64_t excl = x - sum;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        const int i = 4 * lane + j;
                        if (i < clen) pre[i + 1] = excl + v[j];
                    }
                    if (lane == 0) pre[0] = 0;
                }
                __syncthreads();
                const int64_t total = pre[clen];
                int32_t nlen = 0;
                for (int64_t base = 0; base < total && pos < bend; base += kCarveThreads) {
                    const int64_t o = base + tid;
                    int32_t w = -1;
                    uint32_t slot = 0;
                    if (o < total) {
                        int lo = 0, hi = clen - 1;
                        while (lo < hi) {
                            const int mid = (lo + hi + 1) >> 1;
                            if (pre[mid] <= o) lo = mid;
                            else hi = mid - 1;
                        }
                        w = col[rp[cur[lo]] + (o - pre[lo])];
                        if (taken[w]) {
                            w = -1;
                        } else {
                            slot = carve_slot(w);
                            for (;;) {
                                const int32_t k = atomicCAS(&hkey[slot], -1, w);
                                if (k == -1 || k == w) break;
                                slot = (slot + 1) & (kCarveHash - 1);
                            }
                            atomicMin(&hval[slot], tid);
                        }
                    }
                    __syncthreads();
                    const bool owner = w >= 0 && hval[slot] == tid;
                    const unsigned long long bal = __ballot(owner);
                    if (lane == 0) wsum[wv] = __popcll(bal);
                    __syncthreads();
                    int32_t rank = __popcll(bal & ((1ull << lane) - 1ull)), cnt = 0;
                    for (int j = 0; j < kCarveThreads / 64; ++j) {
                        if (j < wv) rank += wsum[j];
                        cnt += wsum[j];
                    }
                    const int32_t room = bend - pos;
                    if (owner && rank < room) {
                        out[pos + rank] = w;
                        taken[w] = 1;
                        nxt[nlen + rank] = w;
                    }
                    __syncthreads();
                    if (w >= 0) {
                        hkey[slot] = -1;
                        hval[slot] = INT32_MAX;
                    }
                    const int32_t em = min(cnt, room);
                    pos += em;
                    nlen += em;
                    __syncthreads();
                }
                if (tid < nlen) cur[tid] = nxt[tid];
                clen = nlen;
                __syncthreads();
            }
        }
    }
}

__global__ void k_perm_check(int32_t n, const int32_t* __restrict__ perm, uint32_t* __restrict__ seen,
                             uint32_t* err) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int32_t v = perm[i];
        if (v < 0 || v >= n) { atomicOr(err, 1u); continue; }
        if (atomicAdd(&seen[v], 1u) != 0) atomicOr(err, 1u);
    }
}

// The front list first[0, nf): every id in [0, n) and none repeated (err set
// otherwise); mark[v] = 1 for its nodes.
__global__ void k_front_check(int32_t nf, int32_t n, const int32_t* __restrict__ first, uint32_t* __restrict__ mark,
                              uint32_t* err) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += stride) {
        const int32_t v = first[i];
        if (v < 0 || v >= n) { atomicOr(err, 1u); continue; }
        if (atomicAdd(&mark[v], 1u) != 0) atomicOr(err, 1u);
    }
}

// flag[i] = 1 when order[i] is not one of the front nodes (mark[v] != 0)
__global__ void k_front_flags(int32_t n, const int32_t* __restrict__ order, const uint32_t* __restrict__ mark,
                              int32_t* __restrict__ flag) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        flag[i] = mark[order[i]] ? 0 : 1;
}

// out[nf + pos[i]] = order[i] for the flagged entries (stable)
__global__ void k_front_scatter(int32_t n, int32_t nf, const int32_t* __restrict__ order,
                                const int32_t* __restrict__ flag, const int32_t* __restrict__ pos,
                                int32_t* __restrict__ out) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        if (flag[i]) out[nf + pos[i]] = order[i];
}

// inv[orig[u]] = u
__global__ void k_inverse(int32_t n, const int32_t* __restrict__ orig, int32_t* __restrict__ inv) {
    for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) inv[orig[u]] = u;
}

// row lengths of the renumbered graph: len[u] = outdeg(orig[u])
__global__ void k_relabel_len(int32_t n, const int32_t* __restrict__ orig, const uint32_t* __restrict__ deg,
                              int32_t* __restrict__ len) {
    for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x)
        len[u] = (int32_t)deg[orig[u]];
}

// rows of the renumbered graph: row u is row orig[u] with every target
// renamed by inv (one wave per row)
__global__ void k_relabel_rows(int32_t n, const int32_t* __restrict__ orig, const int32_t* __restrict__ inv,
                               const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                               const int32_t* __restrict__ nrp, int32_t* __restrict__ ncol) {
    const int lane = threadIdx.x & 63;
    const int32_t waves = (int32_t)(gridDim.x * (blockDim.x / 64));
    for (int32_t u = (int32_t)(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64); u < n; u += waves) {
        const int32_t o = orig[u];
        const int32_t b = rp[o], len = rp[o + 1] - b, dst = nrp[u];
        for (int32_t j = lane; j < len; j += 64) ncol[dst + j] = inv[col[b + j]];
    }
}

__global__ void k_map_ids(int64_t count, const int32_t* __restrict__ map, int32_t* __restrict__ ids) {
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
        ids[i] = map[ids[i]];
}

// dst[v] = src[inv[v]], rows of `width` 4-byte words
__global__ void k_gather_rows(int32_t n, int width, const int32_t* __restrict__ inv, const uint32_t* __restrict__ src,
                              uint32_t* __restrict__ dst) {
    const int64_t total = (int64_t)n * width;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
        const int64_t v = i / width, w = i % width;
        dst[i] = src[(int64_t)inv[v] * width + w];
    }
}

// dst[u] = src[orig[u]] (caller's per-node floats into our numbering)
__global__ void k_gather_f32(int32_t n, const int32_t* __restrict__ orig, const float* __restrict__ src,
                             float* __restrict__ dst) {
    for (int32_t u = blockIdx.x * blockDim.x + threadIdx.x; u < n; u += gridDim.x * blockDim.x) dst[u] = src[orig[u]];
}

template <class F>
bc_status cub_call(F&& f, hipStream_t s, DevBuf& tmp) {
    size_t bytes = 0;
    BC_HIP(f((void*)nullptr, bytes));
    if (tmp.bytes < bytes) BC_TRY(tmp.alloc_on(bytes, s));
    BC_HIP(f(tmp.p, bytes));
    (void)s;
    return BC_OK;
}

}  // namespace

bc_status graph_build(bc_graph* g, int32_t n, int64_t m, const int32_t* rp_in, const int32_t* col_in,
                      uint32_t flags) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = g->stream;
    const bool dev = (flags & BC_DEVICE_PTRS) != 0;
    const bool directed = (flags & BC_DIRECTED) != 0;
    if (m >= (int64_t)INT32_MAX) {
        set_error("m = %lld arcs does not fit int32 offsets", (long long)m);
        return BC_EGRAPH;
    }
    DevBuf rp0, col0, errb, tmp;
    BC_TRY(rp0.alloc_on(sizeof(int32_t) * ((size_t)n + 1), s));
    BC_TRY(col0.alloc_on(sizeof(int32_t) * (size_t)(m > 0 ? m : 1), s));
    BC_TRY(errb.alloc_on(sizeof(uint32_t), s));
    hipMemcpyKind kind = dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    BC_HIP(hipMemcpyAsync(rp0.p, rp_in, sizeof(int32_t) * ((size_t)n + 1), kind, s));
    if (m > 0) BC_HIP(hipMemcpyAsync(col0.p, col_in, sizeof(int32_t) * (size_t)m, kind, s));
    BC_HIP(hipMemsetAsync(errb.p, 0, sizeof(uint32_t), s));
    k_validate<<<grid_for((int64_t)n + 1), kBlk, 0, s>>>(n, m, rp0.as<int32_t>(), col0.as<int32_t>(),
                                                        errb.as<uint32_t>());
    uint32_t err = 0;
    BC_HIP(hipMemcpyAsync(&err, errb.p, sizeof(err), hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    if (err & 1u) { set_error("malformed row_ptr (row_ptr[0] != 0, decreasing, or row_ptr[n] != m)"); return BC_EGRAPH; }
    if (err & 2u) { set_error("col entry outside [0, n)"); return BC_EGRAPH; }

    int64_t mc = m;
    if (err & 4u) {
        // canonical form: sort every row, then drop self-loops and repeats
        DevBuf sorted, cnt, nrp;
        BC_TRY(sorted.alloc_on(sizeof(int32_t) * (size_t)(m > 0 ? m : 1), s));
        BC_TRY(cnt.alloc_on(sizeof(int32_t) * (size_t)(n > 0 ? n : 1), s));
        BC_TRY(nrp.alloc_on(sizeof(int32_t) * ((size_t)n + 1), s));
        const int32_t* rpp = rp0.as<int32_t>();
        BC_TRY(cub_call([&](void* t, size_t& b) {
            return hipcub::DeviceSegmentedRadixSort::SortKeys(t, b, col0.as<int32_t>(), sorted.as<int32_t>(),
                                                              (int)m, n, rpp, rpp + 1, 0, 32, s);
        }, s, tmp));
        k_mark_keep<<<grid_for(n), kBlk, 0, s>>>(n, rpp, sorted.as<int32_t>(), cnt.as<int32_t>());
        BC_TRY(cub_call([&](void* t, size_t& b) {
            return hipcub::DeviceScan::ExclusiveSum(t, b, cnt.as<int32_t>(), nrp.as<int32_t>(), n, s);
        }, s, tmp));
        k_set_last<<<1, 1, 0, s>>>(nrp.as<int32_t>(), n, cnt.as<int32_t>());
        int32_t newm = 0;
        BC_HIP(hipMemcpyAsync(&newm, nrp.as<int32_t>() + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        mc = newm;
        BC_TRY(galloc(g, g->rp, sizeof(int32_t) * ((size_t)n + 1), s));
        BC_TRY(galloc(g, g->col, sizeof(int32_t) * (size_t)(mc > 0 ? mc : 1), s));
        BC_HIP(hipMemcpyAsync(g->rp.p, nrp.p, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s));
        k_compact_rows<<<grid_for(n), kBlk, 0, s>>>(n, rpp, sorted.as<int32_t>(), g->rp.as<int32_t>(),
                                                    g->col.as<int32_t>());
        BC_HIP(hipStreamSynchronize(s));
    } else {
        if (g->ordered) {
            g->rp.swap(rp0);
            g->col.swap(col0);
        } else {
            BC_TRY(g->rp.alloc(sizeof(int32_t) * ((size_t)n + 1)));
            BC_TRY(g->col.alloc(sizeof(int32_t) * (size_t)(m > 0 ? m : 1)));
            BC_HIP(hipMemcpyAsync(g->rp.p, rp0.p, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyDeviceToDevice, s));
            if (m > 0)
                BC_HIP(hipMemcpyAsync(g->col.p, col0.p, sizeof(int32_t) * (size_t)m, hipMemcpyDeviceToDevice, s));
        }
    }

    g->dg.n = n;
    g->dg.m = mc;
    g->dg.directed = directed ? 1 : 0;
    g->dg.rp = g->rp.as<int32_t>();
    g->dg.col = g->col.as<int32_t>();
    BC_TRY(galloc(g, g->deg, sizeof(uint32_t) * (size_t)(n > 0 ? n : 1), s));
    k_degree<<<grid_for(n), kBlk, 0, s>>>(n, g->dg.rp, g->deg.as<uint32_t>());
    g->dg.deg = g->deg.as<uint32_t>();
    BC_TRY(galloc(g, g->adj, sizeof(int2) * (size_t)(mc > 0 ? mc : 1), s));
    if (mc > 0) k_pack_adj<<<grid_for(mc), kBlk, 0, s>>>(mc, g->dg.col, g->dg.deg, g->adj.as<int2>());
    g->dg.adj = g->adj.as<int2>();
    BC_TRY(galloc(g, g->x0, sizeof(uint32_t) * (size_t)(n > 0 ? n : 1), s));
    BC_TRY(galloc(g, g->x1, sizeof(uint32_t) * (size_t)(n > 0 ? n : 1), s));
    g->dg.x0 = g->x0.as<uint32_t>();
    g->dg.x1 = g->x1.as<uint32_t>();

    if (!directed) {
        if (flags & BC_VALIDATE) {
            BC_HIP(hipMemsetAsync(errb.p, 0, sizeof(uint32_t), s));
            k_symmetric<<<grid_for(n), kBlk, 0, s>>>(n, g->dg.rp, g->dg.col, errb.as<uint32_t>());
            BC_HIP(hipMemcpyAsync(&err, errb.p, sizeof(err), hipMemcpyDeviceToHost, s));
            BC_HIP(hipStreamSynchronize(s));
            if (err & 8u) { set_error("undirected CSR is not symmetric"); return BC_EGRAPH; }
        }
        g->dg.irp = g->dg.rp;
        g->dg.icol = g->dg.col;
        DevBuf P, size, label;
        BC_TRY(P.alloc_on(sizeof(int32_t) * (size_t)(n > 0 ? n : 1), s));
        BC_TRY(size.alloc_on(sizeof(uint32_t) * (size_t)(n > 0 ? n : 1), s));
        BC_TRY(label.alloc_on(sizeof(int32_t) * (size_t)(n > 0 ? n : 1), s));
        BC_HIP(hipMemsetAsync(size.p, 0, sizeof(uint32_t) * (size_t)(n > 0 ? n : 1), s));
        if (n > 0) {
            k_uf_init<<<grid_for(n), kBlk, 0, s>>>(n, P.as<int32_t>());
            k_uf_union<<<grid_for(n), kBlk, 0, s>>>(n, g->dg.rp, g->dg.col, P.as<int32_t>());
            k_uf_count<<<grid_for(n), kBlk, 0, s>>>(n, P.as<int32_t>(), size.as<uint32_t>(), label.as<int32_t>());
            k_uf_reach<<<grid_for(n), kBlk, 0, s>>>(n, label.as<int32_t>(), size.as<uint32_t>(),
                                                    g->x0.as<uint32_t>(), g->x1.as<uint32_t>());
        }
        BC_HIP(hipStreamSynchronize(s));
    } else {
        g->big_scc = (flags & BC_BIG_SCC) != 0;
        BC_TRY(directed_reach(g));
    }
    BC_HIP(hipGetLastError());
    auto t1 = std::chrono::steady_clock::now();
    g->preprocess_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
    return BC_OK;
}

bc_status order_by_degree(bc_graph* g, int32_t* d_order, hipStream_t s) {
    int32_t n = g->dg.n;
    if (n == 0) return BC_OK;
    std::unique_lock<std::mutex> lk(g->cache_mu);
    if (!g->have_order_deg) {
        DevBuf k0, k1, tmp;
        BC_TRY(k0.alloc_on(sizeof(uint64_t) * (size_t)n, s));
        BC_TRY(k1.alloc_on(sizeof(uint64_t) * (size_t)n, s));
        BC_TRY(galloc(g, g->order_deg, sizeof(int32_t) * (size_t)n, s));
        k_degree_keys<<<grid_for(n), kBlk, 0, s>>>(n, g->dg.deg, g->dg.orig, k0.as<uint64_t>());
        BC_TRY(cub_call([&](void* t, size_t& b) {
            return hipcub::DeviceRadixSort::SortKeys(t, b, k0.as<uint64_t>(), k1.as<uint64_t>(), n, 0, 64, s);
        }, s, tmp));
        k_low32<<<grid_for(n), kBlk, 0, s>>>(n, k1.as<uint64_t>(), g->order_deg.as<int32_t>());
        BC_TRY(ids_to_internal(g, g->order_deg.as<int32_t>(), n, s));
        BC_HIP(hipStreamSynchronize(s));
        g->have_order_deg = true;
    }
    lk.unlock();
    BC_HIP(hipMemcpyAsync(d_order, g->order_deg.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    return BC_OK;
}

// Decreasing out-degree; among equal degrees, sources sharing their
// highest-degree neighbour are adjacent (then by id), so a batch of
// consecutive sources expands common neighbourhoods once.
bc_status order_grouped(bc_graph* g, int32_t* d_order, hipStream_t s) {
    int32_t n = g->dg.n;
    if (n == 0) return BC_OK;
    std::unique_lock<std::mutex> lk(g->cache_mu);
    if (!g->have_order_grp) {
        DevBuf k0, k1, perm, dk0, dk1, tmp;
        BC_TRY(k0.alloc_on(sizeof(uint64_t) * (size_t)n, s));
        BC_TRY(k1.alloc_on(sizeof(uint64_t) * (size_t)n, s));
        BC_TRY(perm.alloc_on(sizeof(int32_t) * (size_t)n, s));
        BC_TRY(dk0.alloc_on(sizeof(uint32_t) * (size_t)n, s));
        BC_TRY(dk1.alloc_on(sizeof(uint32_t) * (size_t)n, s));
        BC_TRY(galloc(g, g->order_grp, sizeof(int32_t) * (size_t)n, s));
        k_hub_keys<<<grid_for(n), kBlk, 0, s>>>(n, g->dg.rp, g->dg.col, g->dg.deg, k0.as<uint64_t>());
        BC_TRY(cub_call([&](void* t, size_t& b) {
            return hipcub::DeviceRadixSort::SortKeys(t, b, k0.as<uint64_t>(), k1.as<uint64_t>(), n, 0, 64, s);
        }, s, tmp));
        k_low32<<<grid_for(n), kBlk, 0, s>>>(n, k1.as<uint64_t>(), perm.as<int32_t>());
        k_degkey_of<<<grid_for(n), kBlk, 0, s>>>(n, perm.as<int32_t>(), g->dg.deg, dk0.as<uint32_t>());
        // stable: equal degrees keep the (hub, id) order
        BC_TRY(cub_call([&](void* t, size_t& b) {
            return hipcub::DeviceRadixSort::SortPairs(t, b, dk0.as<uint32_t>(), dk1.as<uint32_t>(), perm.as<int32_t>(),
                                                      g->order_grp.as<int32_t>(), n, 0, 32, s);
        }, s, tmp));
        BC_HIP(hipStreamSynchronize(s));
        g->have_order_grp = true;
    }
    lk.unlock();
    BC_HIP(hipMemcpyAsync(d_order, g->order_grp.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    return BC_OK;
}

bc_status order_by_scores(bc_graph* g, const float* scores, bool scores_on_device, int32_t* d_order,
                          hipStream_t s) {
    int32_t n = g->dg.n;
    if (n == 0) return BC_OK;
    BC_TRY(order_by_degree(g, d_order, s));
    DevBuf sc, key0, key1, val1, tmp;
    BC_TRY(sc.alloc_on(sizeof(float) * (size_t)n, s));
    BC_TRY(key0.alloc_on(sizeof(uint32_t) * (size_t)n, s));
    BC_TRY(key1.alloc_on(sizeof(uint32_t) * (size_t)n, s));
    BC_TRY(val1.alloc_on(sizeof(int32_t) * (size_t)n, s));
    BC_HIP(hipMemcpyAsync(sc.p, scores, sizeof(float) * (size_t)n,
                          scores_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    if (!scores_on_device && g->relabeled) {
        // the caller's scores are indexed by the caller's ids
        DevBuf sc2;
        BC_TRY(sc2.alloc_on(sizeof(float) * (size_t)n, s));
        k_gather_f32<<<grid_for(n), kBlk, 0, s>>>(n, g->orig.as<int32_t>(), sc.as<float>(), sc2.as<float>());
        sc.swap(sc2);
    }
    k_score_keys<<<grid_for(n), kBlk, 0, s>>>(n, sc.as<float>(), d_order, key0.as<uint32_t>());
    // radix sort is stable: equal scores keep the degree order
    BC_TRY(cub_call([&](void* t, size_t& b) {
        return hipcub::DeviceRadixSort::SortPairs(t, b, key0.as<uint32_t>(), key1.as<uint32_t>(), d_order,
                                                  val1.as<int32_t>(), n, 0, 32, s);
    }, s, tmp));
    BC_HIP(hipMemcpyAsync(d_order, val1.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    BC_HIP(hipStreamSynchronize(s));
    return BC_OK;
}

// Score every source with the perceptron (features cached per graph) and
// sort by decreasing score.  The order depends only on the graph and the
// parameters, so the one for the first parameter set a graph is asked for is
// kept, like the degree-based orders; it is never rebuilt, so a copy taken
// from it on another stream cannot meet a rewrite.  Other parameter sets are
// scored on every call.
bc_status order_learned(bc_graph* g, const float* h_params, int32_t* d_order, hipStream_t s) {
    const int32_t n = g->dg.n;
    if (n == 0) return BC_OK;
    BC_TRY(graph_features(g, s));
    bool keep = false;
    {
        std::lock_guard<std::mutex> lk(g->cache_mu);
        if (g->have_order_lrn &&
            std::memcmp(g->lrn_params.data(), h_params, sizeof(float) * BC_MLP_PARAMS) == 0) {
            BC_HIP(hipMemcpyAsync(d_order, g->order_lrn.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice,
                                  s));
            return BC_OK;
        }
        keep = !g->have_order_lrn;
    }
    // scored without the cache lock (the score order takes it for the degree order)
    DevBuf prm, sc, ord;
    BC_TRY(prm.alloc_on(sizeof(float) * BC_MLP_PARAMS, s));
    BC_TRY(sc.alloc_on(sizeof(float) * (size_t)n, s));
    BC_TRY(galloc(g, ord, sizeof(int32_t) * (size_t)n, s));
    BC_HIP(hipMemcpyAsync(prm.p, h_params, sizeof(float) * BC_MLP_PARAMS, hipMemcpyHostToDevice, s));
    BC_TRY(mlp_forward(prm.as<float>(), g->feat.as<float>(), n, sc.as<float>(), s));
    BC_TRY(order_by_scores(g, sc.as<float>(), true, ord.as<int32_t>(), s));  // returns with s drained
    BC_HIP(hipMemcpyAsync(d_order, ord.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    if (keep) {
        std::lock_guard<std::mutex> lk(g->cache_mu);
        if (!g->have_order_lrn) {  // another thread may have kept its own meanwhile
            g->order_lrn.swap(ord);
            g->lrn_params.assign(h_params, h_params + BC_MLP_PARAMS);
            g->have_order_lrn = true;
            return BC_OK;
        }
    }
    BC_HIP(hipStreamSynchronize(s));  // the copy has read ord before it is freed
    return BC_OK;
}

// The learned head + grouped tail.  Like the score order it depends only on
// the graph, the parameters and the head length (one per k), so for the kept
// parameter set the first kLrnHeads head lengths asked for are kept; none is
// ever rebuilt.  Other requests are merged per call.
bc_status order_learned_grouped(bc_graph* g, const float* h_params, int32_t head, int32_t* d_order,
                                hipStream_t s) {
    const int32_t n = g->dg.n;
    if (n == 0) return BC_OK;
    auto kept_params = [&]() {
        return g->have_order_lrn &&
               std::memcmp(g->lrn_params.data(), h_params, sizeof(float) * BC_MLP_PARAMS) == 0;
    };
    {
        std::lock_guard<std::mutex> lk(g->cache_mu);
        if (kept_params()) {
            for (int i = 0; i < g->n_lrn_heads; ++i) {
                if (g->lrn_head[i] == head) {
                    BC_HIP(hipMemcpyAsync(d_order, g->order_lrn_head[i].p, sizeof(int32_t) * (size_t)n,
                                          hipMemcpyDeviceToDevice, s));
                    return BC_OK;
                }
            }
        }
    }
    DevBuf bys, out;
    BC_TRY(bys.alloc_on(sizeof(int32_t) * (size_t)n, s));
    BC_TRY(galloc(g, out, sizeof(int32_t) * (size_t)n, s));
    BC_TRY(order_learned(g, h_params, bys.as<int32_t>(), s));
    BC_TRY(order_head_grouped(g, bys.as<int32_t>(), head, out.as<int32_t>(), s));  // returns with s drained
    BC_HIP(hipMemcpyAsync(d_order, out.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    {
        std::lock_guard<std::mutex> lk(g->cache_mu);
        bool have = false;
        for (int i = 0; i < g->n_lrn_heads; ++i) have = have || g->lrn_head[i] == head;
        if (kept_params() && !have && g->n_lrn_heads < bc_graph::kLrnHeads) {
            g->order_lrn_head[g->n_lrn_heads].swap(out);
            g->lrn_head[g->n_lrn_heads] = head;
            ++g->n_lrn_heads;
            return BC_OK;
        }
    }
    BC_HIP(hipStreamSynchronize(s));  // the copy has read out before it is freed
    return BC_OK;
}

// The first `head` sources of the score order d_by_score, then every other
// source in the grouped degree order (relative order kept).
bc_status order_head_grouped(bc_graph* g, const int32_t* d_by_score, int32_t head, int32_t* d_order,
                             hipStream_t s) {
    int32_t n = g->dg.n;
    if (n == 0) return BC_OK;
    head = std::min(std::max(head, 0), n);
    DevBuf grp, mark, keep, nsel, tmp;
    BC_TRY(grp.alloc_on(sizeof(int32_t) * (size_t)n, s));
    BC_TRY(mark.alloc_on((size_t)n, s));
    BC_TRY(keep.alloc_on((size_t)n, s));
    BC_TRY(nsel.alloc_on(sizeof(int32_t), s));
    BC_TRY(order_grouped(g, grp.as<int32_t>(), s));
    BC_HIP(hipMemsetAsync(mark.p, 0, (size_t)n, s));
    if (head > 0) {
        k_mark_head<<<grid_for(head), kBlk, 0, s>>>(head, d_by_score, mark.as<uint8_t>());
        BC_HIP(hipMemcpyAsync(d_order, d_by_score, sizeof(int32_t) * (size_t)head, hipMemcpyDeviceToDevice, s));
    }
    k_keep_unmarked<<<grid_for(n), kBlk, 0, s>>>(n, grp.as<int32_t>(), mark.as<uint8_t>(), keep.as<uint8_t>());
    BC_TRY(cub_call([&](void* t, size_t& b) {
        return hipcub::DeviceSelect::Flagged(t, b, grp.as<int32_t>(), keep.as<uint8_t>(), d_order + head,
                                             nsel.as<int32_t>(), n, s);
    }, s, tmp));
    int32_t got = 0;
    BC_HIP(hipMemcpyAsync(&got, nsel.p, sizeof(got), hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    if (got != n - head) {
        set_error("internal: head/grouped order holds %d + %d of %d sources", head, got, n);
        return BC_EDEVICE;
    }
    return BC_OK;
}

// Level-synchronous BFS from src over the out-arcs; dist[] (-1 = not
// reached).  With order != nullptr the discovery order (levels sorted by
// earliest parent position, then id) is written to order[0, *reached).
static bc_status loc_bfs(bc_graph* g, int32_t src, int32_t* dist, uint32_t* ppos, int32_t* order, int32_t* reached,
                         DevBuf& la, DevBuf& lb, DevBuf& k0, DevBuf& k1, DevBuf& cnt, DevBuf& tmp, hipStream_t s) {
    const int32_t n = g->dg.n;
    k_loc_init<<<grid_for(n), kBlk, 0, s>>>(n, dist, ppos);
    const int32_t zero = 0;
    BC_HIP(hipMemcpyAsync(dist + src, &zero, sizeof(int32_t), hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(la.p, &src, sizeof(int32_t), hipMemcpyHostToDevice, s));
    if (order) BC_HIP(hipMemcpyAsync(order, &src, sizeof(int32_t), hipMemcpyHostToDevice, s));
    uint32_t flen = 1, base = 0;
    int32_t* F = la.as<int32_t>();
    int32_t* N = lb.as<int32_t>();
    for (int32_t d = 0; flen > 0; ++d) {
        BC_HIP(hipMemsetAsync(cnt.p, 0, sizeof(uint32_t), s));
        k_loc_expand<<<grid_for(flen), kBlk, 0, s>>>(g->dg.rp, g->dg.col, F, flen, d, base, dist, ppos, N,
                                                      cnt.as<uint32_t>());
        uint32_t nc = 0;
        BC_HIP(hipMemcpyAsync(&nc, cnt.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        if (order && nc > 0) {
            k_loc_keys<<<grid_for(nc), kBlk, 0, s>>>(nc, N, ppos, k0.as<uint64_t>());
            BC_TRY(cub_call([&](void* t, size_t& b) {
                return hipcub::DeviceRadixSort::SortKeys(t, b, k0.as<uint64_t>(), k1.as<uint64_t>(), (int)nc, 0, 64, s);
            }, s, tmp));
            k_low32<<<grid_for(nc), kBlk, 0, s>>>((int32_t)nc, k1.as<uint64_t>(), N);
            BC_HIP(hipMemcpyAsync(order + base + flen, N, sizeof(int32_t) * nc, hipMemcpyDeviceToDevice, s));
        }
        base += flen;
        flen = nc;
        std::swap(F, N);
    }
    *reached = (int32_t)base;
    return BC_OK;
}

// Seed order: breadth-first discovery order from an approximate centre (the
// middle of a shortest path between the ends of a double sweep started at
// the highest-degree node); nodes outside its component follow in degree
// order.  Cached in g->order_loc_seed.
static bc_status locality_seed(bc_graph* g, hipStream_t s) {
    const int32_t n = g->dg.n;
    if (n == 0) return BC_OK;
    {
        std::unique_lock<std::mutex> lk(g->cache_mu);
        if (!g->have_order_loc_seed) {
            lk.unlock();
            DevBuf deg_order;
            BC_TRY(deg_order.alloc_on(sizeof(int32_t) * (size_t)n, s));
            BC_TRY(order_by_degree(g, deg_order.as<int32_t>(), s));
            lk.lock();
            if (!g->have_order_loc_seed) {
                DevBuf da, db, ppos, la, lb, k0, k1, cnt, best, flag, nsel, tmp;
                BC_TRY(da.alloc_on(sizeof(int32_t) * (size_t)n, s));
                BC_TRY(db.alloc_on(sizeof(int32_t) * (size_t)n, s));
                BC_TRY(ppos.alloc_on(sizeof(uint32_t) * (size_t)n, s));
                BC_TRY(la.alloc_on(sizeof(int32_t) * (size_t)n, s));
                BC_TRY(lb.alloc_on(sizeof(int32_t) * (size_t)n, s));
                BC_TRY(k0.alloc_on(sizeof(uint64_t) * (size_t)n, s));
                BC_TRY(k1.alloc_on(sizeof(uint64_t) * (size_t)n, s));
                BC_TRY(cnt.alloc_on(sizeof(uint32_t), s));
                BC_TRY(best.alloc_on(sizeof(unsigned long long), s));
                BC_TRY(flag.alloc_on((size_t)n, s));
                BC_TRY(nsel.alloc_on(sizeof(int32_t), s));
                BC_TRY(galloc(g, g->order_loc_seed, sizeof(int32_t) * (size_t)n, s));
                int32_t* ord = g->order_loc_seed.as<int32_t>();
                int32_t u0 = 0, reached = 0;
                BC_HIP(hipMemcpyAsync(&u0, deg_order.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
                BC_HIP(hipStreamSynchronize(s));
                auto farthest = [&](int32_t* dist, int32_t* out) -> bc_status {
                    const unsigned long long z = 0;
                    BC_HIP(hipMemcpyAsync(best.p, &z, sizeof(z), hipMemcpyHostToDevice, s));
                    k_loc_far<<<grid_for(n), kBlk, 0, s>>>(n, dist, best.as<unsigned long long>());
                    unsigned long long b = 0;
                    BC_HIP(hipMemcpyAsync(&b, best.p, sizeof(b), hipMemcpyDeviceToHost, s));
                    BC_HIP(hipStreamSynchronize(s));
                    *out = (int32_t)(0xFFFFFFFFu - (uint32_t)(b & 0xFFFFFFFFu));
                    return BC_OK;
                };
                // double sweep: u0 -> a (farthest), a -> b (farthest); centre on a-b
                int32_t a = 0, b = 0;
                BC_TRY(loc_bfs(g, u0, da.as<int32_t>(), nullptr, nullptr, &reached, la, lb, k0, k1, cnt, tmp, s));
                BC_TRY(farthest(da.as<int32_t>(), &a));
                BC_TRY(loc_bfs(g, a, da.as<int32_t>(), nullptr, nullptr, &reached, la, lb, k0, k1, cnt, tmp, s));
                BC_TRY(farthest(da.as<int32_t>(), &b));
                int32_t D = 0;
                BC_HIP(hipMemcpyAsync(&D, da.as<int32_t>() + b, sizeof(int32_t), hipMemcpyDeviceToHost, s));
                BC_TRY(loc_bfs(g, b, db.as<int32_t>(), nullptr, nullptr, &reached, la, lb, k0, k1, cnt, tmp, s));
                const unsigned long long mx = ~0ull;
                BC_HIP(hipMemcpyAsync(best.p, &mx, sizeof(mx), hipMemcpyHostToDevice, s));
                k_loc_centre<<<grid_for(n), kBlk, 0, s>>>(n, da.as<int32_t>(), db.as<int32_t>(), D,
                                                          best.as<unsigned long long>());
                unsigned long long cb = 0;
                BC_HIP(hipMemcpyAsync(&cb, best.p, sizeof(cb), hipMemcpyDeviceToHost, s));
                BC_HIP(hipStreamSynchronize(s));
                const int32_t c = cb == ~0ull ? u0 : (int32_t)(uint32_t)(cb & 0xFFFFFFFFu);
                // ordered BFS from the centre, then the other components in degree order
                BC_TRY(loc_bfs(g, c, da.as<int32_t>(), ppos.as<uint32_t>(), ord, &reached, la, lb, k0, k1, cnt, tmp,
                               s));
                k_loc_unreached<<<grid_for(n), kBlk, 0, s>>>(n, deg_order.as<int32_t>(), da.as<int32_t>(),
                                                             flag.as<uint8_t>());
                BC_TRY(cub_call([&](void* t, size_t& bb) {
                    return hipcub::DeviceSelect::Flagged(t, bb, deg_order.as<int32_t>(), flag.as<uint8_t>(),
                                                         ord + reached, nsel.as<int32_t>(), n, s);
                }, s, tmp));
                int32_t rest = 0;
                BC_HIP(hipMemcpyAsync(&rest, nsel.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
                BC_HIP(hipStreamSynchronize(s));
                if (reached + rest != n) {
                    set_error("internal: locality order holds %d + %d of %d sources", reached, rest, n);
                    return BC_EDEVICE;
                }
                g->have_order_loc_seed = true;
            }
        }
    }
    return BC_OK;
}

// Locality order for batches of B sources: the seed order cut into compact
// balls of B (k_carve).  Cached per B.
bc_status order_locality(bc_graph* g, int32_t B, int32_t* d_order, hipStream_t s) {
    const int32_t n = g->dg.n;
    if (n == 0) return BC_OK;
    if (B != 64 && B != 128 && B != 256) {
        set_error("locality order: batch width must be 64, 128 or 256 (got %d)", B);
        return BC_EINVAL;
    }
    BC_TRY(locality_seed(g, s));
    const int slot = B == 64 ? 0 : (B == 128 ? 1 : 2);
    std::lock_guard<std::mutex> lk(g->cache_mu);
    if (!g->have_order_loc[slot]) {
        DevBuf taken, err;
        BC_TRY(taken.alloc_on((size_t)n, s));
        BC_TRY(err.alloc_on(sizeof(int32_t), s));
        BC_HIP(hipMemsetAsync(taken.p, 0, (size_t)n, s));
        BC_HIP(hipMemsetAsync(err.p, 0, sizeof(int32_t), s));
        BC_TRY(galloc(g, g->order_loc[slot], sizeof(int32_t) * (size_t)n, s));
        k_carve<<<1, kCarveThreads, 0, s>>>(n, g->dg.rp, g->dg.col, g->order_loc_seed.as<int32_t>(), B,
                                            taken.as<uint8_t>(), g->order_loc[slot].as<int32_t>(), err.as<int32_t>());
        int32_t e = 0;
        BC_HIP(hipMemcpyAsync(&e, err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        if (e) {
            set_error("internal: locality carving ran out of seeds");
            return BC_EDEVICE;
        }
        g->have_order_loc[slot] = true;
    }
    BC_HIP(hipMemcpyAsync(d_order, g->order_loc[slot].p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    return BC_OK;
}

bc_status order_front(bc_graph* g, const int32_t* h_first, int32_t nf, int32_t* d_order, hipStream_t s,
                      bool caller_ids) {
    const int32_t n = g->dg.n;
    if (nf < 0 || nf > n) { set_error("opts.nfirst %d outside [0, n = %d]", nf, n); return BC_EINVAL; }
    if (nf == 0 || n == 0) return BC_OK;
    if (!h_first) { set_error("opts.first is NULL with nfirst = %d", nf); return BC_EINVAL; }
    DevBuf mark, errb, flag, pos, out, tmp;
    BC_TRY(mark.alloc_on(sizeof(uint32_t) * (size_t)n, s));
    BC_TRY(errb.alloc_on(sizeof(uint32_t), s));
    BC_TRY(flag.alloc_on(sizeof(int32_t) * (size_t)n, s));
    BC_TRY(pos.alloc_on(sizeof(int32_t) * (size_t)n, s));
    BC_TRY(out.alloc_on(sizeof(int32_t) * (size_t)n, s));
    BC_HIP(hipMemsetAsync(mark.p, 0, sizeof(uint32_t) * (size_t)n, s));
    BC_HIP(hipMemsetAsync(errb.p, 0, sizeof(uint32_t), s));
    // the front list goes to out[0, nf); the range check and the repeat check
    // mark each of its nodes once
    BC_HIP(hipMemcpyAsync(out.p, h_first, sizeof(int32_t) * (size_t)nf, hipMemcpyHostToDevice, s));
    k_front_check<<<grid_for(nf), kBlk, 0, s>>>(nf, n, out.as<int32_t>(), mark.as<uint32_t>(), errb.as<uint32_t>());
    uint32_t err = 0;
    BC_HIP(hipMemcpyAsync(&err, errb.p, sizeof(err), hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    if (err) { set_error("opts.first holds a node outside [0, n) or a repeated node"); return BC_EINVAL; }
    if (g->relabeled && caller_ids) {
        // the caller's ids into ours, and the marks again by our ids
        BC_TRY(ids_to_internal(g, out.as<int32_t>(), nf, s));
        BC_HIP(hipMemsetAsync(mark.p, 0, sizeof(uint32_t) * (size_t)n, s));
        k_front_check<<<grid_for(nf), kBlk, 0, s>>>(nf, n, out.as<int32_t>(), mark.as<uint32_t>(), errb.as<uint32_t>());
    }
    k_front_flags<<<grid_for(n), kBlk, 0, s>>>(n, d_order, mark.as<uint32_t>(), flag.as<int32_t>());
    BC_TRY(cub_call([&](void* t, size_t& b) {
        return hipcub::DeviceScan::ExclusiveSum(t, b, flag.as<int32_t>(), pos.as<int32_t>(), n, s);
    }, s, tmp));
    k_front_scatter<<<grid_for(n), kBlk, 0, s>>>(n, nf, d_order, flag.as<int32_t>(), pos.as<int32_t>(),
                                                 out.as<int32_t>());
    BC_HIP(hipMemcpyAsync(d_order, out.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    BC_HIP(hipStreamSynchronize(s));
    return BC_OK;
}

bc_status order_given(bc_graph* g, const int32_t* h_perm, int32_t* d_order, hipStream_t s) {
    int32_t n = g->dg.n;
    if (n == 0) return BC_OK;
    DevBuf seen, errb;
    BC_TRY(seen.alloc_on(sizeof(uint32_t) * (size_t)n, s));
    BC_TRY(errb.alloc_on(sizeof(uint32_t), s));
    BC_HIP(hipMemcpyAsync(d_order, h_perm, sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
    BC_HIP(hipMemsetAsync(seen.p, 0, sizeof(uint32_t) * (size_t)n, s));
    BC_HIP(hipMemsetAsync(errb.p, 0, sizeof(uint32_t), s));
    k_perm_check<<<grid_for(n), kBlk, 0, s>>>(n, d_order, seen.as<uint32_t>(), errb.as<uint32_t>());
    uint32_t err = 0;
    BC_HIP(hipMemcpyAsync(&err, errb.p, sizeof(err), hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    if (err) { set_error("opts.perm is not a permutation of [0, n)"); return BC_EINVAL; }
    return ids_to_internal(g, d_order, n, s);  // the caller's ids into ours
}

bc_status ids_to_internal(bc_graph* g, int32_t* d_ids, int64_t count, hipStream_t s) {
    if (!g->relabeled || count <= 0) return BC_OK;
    k_map_ids<<<grid_for(count), kBlk, 0, s>>>(count, g->inv.as<int32_t>(), d_ids);
    BC_HIP(hipGetLastError());
    return BC_OK;
}

bc_status ids_to_caller(bc_graph* g, int32_t* d_ids, int64_t count, hipStream_t s) {
    if (!g->relabeled || count <= 0) return BC_OK;
    k_map_ids<<<grid_for(count), kBlk, 0, s>>>(count, g->orig.as<int32_t>(), d_ids);
    BC_HIP(hipGetLastError());
    return BC_OK;
}

bc_status rows_to_caller(bc_graph* g, const void* d_src, void* d_dst, int width, hipStream_t s) {
    const int32_t n = g->dg.n;
    if (n == 0) return BC_OK;
    if (!g->relabeled) {
        BC_HIP(hipMemcpyAsync(d_dst, d_src, sizeof(uint32_t) * (size_t)n * width, hipMemcpyDeviceToDevice, s));
        return BC_OK;
    }
    k_gather_rows<<<grid_for((int64_t)n * width), kBlk, 0, s>>>(n, width, g->inv.as<int32_t>(),
                                                                 static_cast<const uint32_t*>(d_src),
                                                                 static_cast<uint32_t*>(d_dst));
    BC_HIP(hipGetLastError());
    return BC_OK;
}

// The renumbered graph: nodes in the locality seed order (breadth-first from
// an approximate centre, then the other components by degree), so that a
// node's neighbours, which a batch reaches together, have nearby ids and
// their node records share cache lines and memory pages.  Built by a second
// pass of graph_build over the renamed rows (which sorts them); the result
// is the same graph up to the names of its nodes.
bc_status graph_relabel(bc_graph* g, uint32_t flags, bool ordered, bc_graph** out) {
    *out = nullptr;
    const int32_t n = g->dg.n;
    const int64_t m = g->dg.m;
    hipStream_t s = g->stream;
    BC_TRY(locality_seed(g, s));
    std::unique_ptr<bc_graph> h(new bc_graph());
    h->stream = s;
    h->ordered = ordered;
    h->device = g->device;
    BC_TRY(galloc(h.get(), h->orig, sizeof(int32_t) * (size_t)n, s));
    BC_TRY(galloc(h.get(), h->inv, sizeof(int32_t) * (size_t)n, s));
    BC_HIP(hipMemcpyAsync(h->orig.p, g->order_loc_seed.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    k_inverse<<<grid_for(n), kBlk, 0, s>>>(n, h->orig.as<int32_t>(), h->inv.as<int32_t>());
    DevBuf len, nrp, ncol, tmp;
    BC_TRY(len.alloc_on(sizeof(int32_t) * (size_t)n, s));
    BC_TRY(nrp.alloc_on(sizeof(int32_t) * ((size_t)n + 1), s));
    BC_TRY(ncol.alloc_on(sizeof(int32_t) * (size_t)(m > 0 ? m : 1), s));
    k_relabel_len<<<grid_for(n), kBlk, 0, s>>>(n, h->orig.as<int32_t>(), g->dg.deg, len.as<int32_t>());
    BC_TRY(cub_call([&](void* t, size_t& b) {
        return hipcub::DeviceScan::ExclusiveSum(t, b, len.as<int32_t>(), nrp.as<int32_t>(), n, s);
    }, s, tmp));
    const int32_t mm = (int32_t)m;
    BC_HIP(hipMemcpyAsync(nrp.as<int32_t>() + n, &mm, sizeof(int32_t), hipMemcpyHostToDevice, s));
    k_relabel_rows<<<grid_for((int64_t)n * 64), kBlk, 0, s>>>(n, h->orig.as<int32_t>(), h->inv.as<int32_t>(),
                                                                g->dg.rp, g->dg.col, nrp.as<int32_t>(),
                                                                ncol.as<int32_t>());
    BC_HIP(hipStreamSynchronize(s));
    BC_TRY(graph_build(h.get(), n, m, nrp.as<int32_t>(), ncol.as<int32_t>(), flags | BC_DEVICE_PTRS));
    h->dg.orig = h->orig.as<int32_t>();
    h->relabeled = true;
    h->preprocess_ms += g->preprocess_ms;
    *out = h.release();
    return BC_OK;
}

}  // namespace bc
