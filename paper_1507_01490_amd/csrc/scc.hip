// Directed pre-processing (Section 2.4): the in-CSR, the strongly connected
// components, and the reach bounds alpha(v) <= r(v) <= omega(v) from the
// weighted DAG of SCCs, w(C) = |C|, arcs taken as a set:
//     alpha(C) = w(C) + max over successors D of alpha(D)   (w(C) for a sink)
//     omega(C) = w(C) + sum over successors D of omega(D),  capped at n,
// evaluated in reverse topological order (a component once all of its
// successors are known).
//
// Optional refinement (end of Section 2.4, graph flag BC_BIG_SCC): the
// largest component T (largest w; among equals the one holding the smallest
// node id) takes its exact reach rT = |R(T)| from one breadth-first search
// instead of the recurrence, so alpha(T) = omega(T) = rT and the exact value
// flows into every component that reaches T.  Such a component C also gets
// the upper bound rT + omega'(C), where omega' is the same recurrence over
// the components outside R(T) only (what C reaches outside R(T) is exactly
// what it reaches in the DAG without R(T)); omega(C) is the smaller bound.
//
// SCCs are found on the GPU without recursion:
//   1. trim: a node with no remaining in-arc or no remaining out-arc is a
//      singleton SCC (repeated a few times);
//   2. forward-backward: the SCC of a high-degree pivot is the intersection
//      of its forward and backward reachable sets (finds the giant SCC);
//   3. colouring rounds on what is left: colour(v) = largest id that reaches
//      v (max-propagation along arcs); a node whose colour is its own id is a
//      root, and the SCC of root c is the set of nodes of colour c that reach
//      c through nodes of colour c.  Every round removes at least the SCC of
//      the largest remaining id.
#include <hipcub/hipcub.hpp>

#include "bc_internal.h"

namespace bc {

namespace {

constexpr int kBlk = 256;

inline unsigned grid_for(int64_t work, int64_t cap = 8192) {
    int64_t b = (work + kBlk - 1) / kBlk;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

#define GSTRIDE_LOOP(i, N)                                                      \
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (N);   \
         i += (int64_t)gridDim.x * blockDim.x)

__device__ inline int32_t ld_rel(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_indeg(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                        int32_t* __restrict__ icnt) {
    GSTRIDE_LOOP(u, n) {
        for (int32_t i = rp[u]; i < rp[u + 1]; ++i) atomicAdd(&icnt[col[i]], 1);
    }
}

__global__ void k_close(int32_t* rp, int32_t n, const int32_t* cnt) {
    if (blockIdx.x == 0 && threadIdx.x == 0) rp[n] = n > 0 ? rp[n - 1] + cnt[n - 1] : 0;
}

__global__ void k_fill_in(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                          const int32_t* __restrict__ irp, int32_t* __restrict__ fill, int32_t* __restrict__ icol) {
    GSTRIDE_LOOP(u, n) {
        for (int32_t i = rp[u]; i < rp[u + 1]; ++i) {
            int32_t w = col[i];
            int32_t p = atomicAdd(&fill[w], 1);
            icol[irp[w] + p] = (int32_t)u;
        }
    }
}

__global__ void k_fill_i32(int64_t n, int32_t* p, int32_t v) {
    GSTRIDE_LOOP(i, n) p[i] = v;
}

// trim: active v (comp < 0) without an active out-neighbour or without an
// active in-neighbour becomes its own SCC
__global__ void k_trim(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                       const int32_t* __restrict__ irp, const int32_t* __restrict__ icol, int32_t* comp,
                       int32_t* changed) {
    GSTRIDE_LOOP(v, n) {
        if (ld_rel(&comp[v]) >= 0) continue;
        bool out = false, in = false;
        for (int32_t i = rp[v]; i < rp[v + 1] && !out; ++i) {
            int32_t w = col[i];
            out = (w != (int32_t)v) && ld_rel(&comp[w]) < 0;
        }
        for (int32_t i = irp[v]; i < irp[v + 1] && !in; ++i) {
            int32_t w = icol[i];
            in = (w != (int32_t)v) && ld_rel(&comp[w]) < 0;
        }
        if (!out || !in) {
            __hip_atomic_store(&comp[v], (int32_t)v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *changed = 1;
        }
    }
}

__global__ void k_pivot(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ irp,
                        const int32_t* __restrict__ comp, unsigned long long* best) {
    GSTRIDE_LOOP(v, n) {
        if (comp[v] >= 0) continue;
        uint64_t a = (uint64_t)(rp[v + 1] - rp[v]), b = (uint64_t)(irp[v + 1] - irp[v]);
        uint64_t sc = a * b;
        if (sc > 0x7FFFFFFFull) sc = 0x7FFFFFFFull;
        atomicMax(best, (unsigned long long)((sc << 32) | (uint32_t)v));
    }
}

// one level of a BFS restricted to active nodes; mark bit `bit` in mark[]
__global__ void k_reach_level(const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                              const int32_t* __restrict__ comp, uint32_t* mark, uint32_t bit,
                              const int32_t* __restrict__ fq, int32_t fn, int32_t* nq, int32_t* ncnt) {
    GSTRIDE_LOOP(i, fn) {
        int32_t u = fq[i];
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            int32_t w = col[e];
            if (comp[w] >= 0) continue;
            if (atomicOr(&mark[w], bit) & bit) continue;
            nq[atomicAdd(ncnt, 1)] = w;
        }
    }
}

__global__ void k_fwbw_assign(int32_t n, const uint32_t* __restrict__ mark, int32_t* comp, int32_t pivot) {
    GSTRIDE_LOOP(v, n) {
        if (comp[v] < 0 && mark[v] == 3u) comp[v] = pivot;
    }
}

__global__ void k_color_init(int32_t n, const int32_t* __restrict__ comp, int32_t* color) {
    GSTRIDE_LOOP(v, n) color[v] = comp[v] < 0 ? (int32_t)v : -1;
}

// colour(w) = max colour of active in-neighbours (read as they change)
__global__ void k_color_prop(int32_t n, const int32_t* __restrict__ irp, const int32_t* __restrict__ icol,
                             const int32_t* __restrict__ comp, int32_t* color, int32_t* changed) {
    GSTRIDE_LOOP(w, n) {
        if (comp[w] >= 0) continue;
        int32_t c = ld_rel(&color[w]), c0 = c;
        for (int32_t e = irp[w]; e < irp[w + 1]; ++e) {
            int32_t u = icol[e];
            if (comp[u] >= 0) continue;
            int32_t cu = ld_rel(&color[u]);
            if (cu > c) c = cu;
        }
        if (c > c0) {
            atomicMax(&color[w], c);
            *changed = 1;
        }
    }
}

// roots of the colour classes; in-class reach-to-root marking
__global__ void k_color_roots(int32_t n, const int32_t* __restrict__ color, int32_t* comp_next) {
    GSTRIDE_LOOP(v, n) {
        if (color[v] == (int32_t)v) comp_next[v] = (int32_t)v;
    }
}

__global__ void k_color_back(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                             const int32_t* __restrict__ comp, const int32_t* __restrict__ color,
                             int32_t* comp_next, int32_t* changed) {
    GSTRIDE_LOOP(v, n) {
        if (comp[v] >= 0 || ld_rel(&comp_next[v]) >= 0) continue;
        int32_t c = color[v];
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
            int32_t w = col[e];
            if (comp[w] >= 0 || color[w] != c) continue;
            if (ld_rel(&comp_next[w]) == c) {
                __hip_atomic_store(&comp_next[v], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                *changed = 1;
                break;
            }
        }
    }
}

__global__ void k_color_commit(int32_t n, int32_t* comp, const int32_t* __restrict__ comp_next, int32_t* left) {
    GSTRIDE_LOOP(v, n) {
        if (comp[v] >= 0) continue;
        if (comp_next[v] >= 0) comp[v] = comp_next[v];
        else atomicAdd(left, 1);
    }
}

// dense component ids: is_root scan
__global__ void k_is_root(int32_t n, const int32_t* __restrict__ comp, int32_t* __restrict__ flag) {
    GSTRIDE_LOOP(v, n) flag[v] = comp[v] == (int32_t)v ? 1 : 0;
}

__global__ void k_cid(int32_t n, const int32_t* __restrict__ comp, const int32_t* __restrict__ rootpos,
                      int32_t* __restrict__ cid, uint32_t* __restrict__ wsize) {
    GSTRIDE_LOOP(v, n) {
        int32_t c = rootpos[comp[v]];
        cid[v] = c;
        atomicAdd(&wsize[c], 1u);
    }
}

__global__ void k_dag_arcs(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                           const int32_t* __restrict__ cid, uint64_t* __restrict__ keys, int32_t* cnt) {
    GSTRIDE_LOOP(u, n) {
        int32_t cu = cid[u];
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            int32_t cw = cid[col[e]];
            if (cw == cu) continue;
            keys[atomicAdd(cnt, 1)] = ((uint64_t)(uint32_t)cu << 32) | (uint32_t)cw;
        }
    }
}

// sorted keys -> per-component distinct successor lists (CSR by source)
__global__ void k_dag_count(int32_t na, const uint64_t* __restrict__ keys, int32_t* __restrict__ dcnt) {
    GSTRIDE_LOOP(i, na) {
        if (i > 0 && keys[i] == keys[i - 1]) continue;
        atomicAdd(&dcnt[(int32_t)(keys[i] >> 32)], 1);
    }
}

__global__ void k_dag_fill(int32_t na, const uint64_t* __restrict__ keys, const int32_t* __restrict__ drp,
                           int32_t* __restrict__ dfill, int32_t* __restrict__ dcol) {
    GSTRIDE_LOOP(i, na) {
        if (i > 0 && keys[i] == keys[i - 1]) continue;
        int32_t c = (int32_t)(keys[i] >> 32);
        dcol[drp[c] + atomicAdd(&dfill[c], 1)] = (int32_t)(keys[i] & 0xFFFFFFFFu);
    }
}

// The refinement's inputs (BigScc::c < 0: plain recurrence only).
struct BigScc {
    int32_t c;            // component T
    uint64_t rT;          // |R(T)|
    const int32_t* inRT;  // per component: 1 if reachable from T (T included)
    uint64_t* omega2;     // per component outside R(T): omega' (recurrence outside R(T))
    int32_t* toT;         // per component: 1 if it reaches T (T itself: 0)
};

// one round of the alpha/omega recurrence: every component whose successors
// are all final becomes final
__global__ void k_dag_round(int32_t nc, const int32_t* __restrict__ drp, const int32_t* __restrict__ dcol,
                            const uint32_t* __restrict__ wsize, uint64_t* alpha, uint64_t* omega,
                            int32_t* done, uint64_t ncap, int32_t* left, BigScc B) {
    GSTRIDE_LOOP(c, nc) {
        if (done[c]) continue;
        uint64_t amax = 0, osum = 0, osum2 = 0;
        bool ready = true, reaches = false;
        for (int32_t e = drp[c]; e < drp[c + 1]; ++e) {
            int32_t d = dcol[e];
            if (!__hip_atomic_load(&done[d], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)) { ready = false; break; }
            uint64_t a = __hip_atomic_load(&alpha[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            uint64_t o = __hip_atomic_load(&omega[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (a > amax) amax = a;
            osum += o;
            if (osum > ncap) osum = ncap;
            if (B.c >= 0) {
                if (d == B.c || __hip_atomic_load(&B.toT[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT))
                    reaches = true;
                if (!B.inRT[d]) {
                    osum2 += __hip_atomic_load(&B.omega2[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (osum2 > ncap) osum2 = ncap;
                }
            }
        }
        if (!ready) { atomicAdd(left, 1); continue; }
        uint64_t w = wsize[c];
        uint64_t a = w + amax;
        uint64_t o = w + osum;
        if (o > ncap) o = ncap;
        if (B.c >= 0) {
            uint64_t o2 = w + osum2;
            if (o2 > ncap) o2 = ncap;
            if (c == B.c) {
                a = o = B.rT;  // exact, from the breadth-first search
                o2 = 0;
            } else if (reaches) {
                uint64_t b = B.rT + o2;
                if (b > ncap) b = ncap;
                if (b < o) o = b;
            }
            __hip_atomic_store(&B.omega2[c], o2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&B.toT[c], reaches ? 1 : 0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __hip_atomic_store(&alpha[c], a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&omega[c], o, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&done[c], 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The largest component: max over nodes of (w(cid[v]) << 32 | (2^31 - 1 - v)),
// i.e. the largest size, then the smallest node id.  Wave-reduced, one
// atomic per wave.
__global__ void k_big_pick(int32_t n, const int32_t* __restrict__ cid, const uint32_t* __restrict__ wsize,
                           unsigned long long* best) {
    unsigned long long mx = 0;
    GSTRIDE_LOOP(v, n) {
        unsigned long long key = ((unsigned long long)wsize[cid[v]] << 32) | (uint32_t)(0x7FFFFFFF - (int32_t)v);
        if (key > mx) mx = key;
    }
    for (int off = 32; off > 0; off >>= 1) {
        unsigned long long o = __shfl_xor(mx, off);
        if (o > mx) mx = o;
    }
    if (__lane_id() == 0 && mx) atomicMax(best, mx);
}

// one level of an unrestricted breadth-first search; mark[] = 1 once reached
__global__ void k_bfs_level(const int32_t* __restrict__ rp, const int32_t* __restrict__ col, uint32_t* mark,
                            const int32_t* __restrict__ fq, int32_t fn, int32_t* nq, int32_t* ncnt) {
    GSTRIDE_LOOP(i, fn) {
        int32_t u = fq[i];
        for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
            int32_t w = col[e];
            if (mark[w] || atomicOr(&mark[w], 1u)) continue;
            nq[atomicAdd(ncnt, 1)] = w;
        }
    }
}

// inRT[c] = 1 for every component holding a node the search reached
__global__ void k_mark_comps(int32_t n, const uint32_t* __restrict__ mark, const int32_t* __restrict__ cid,
                             int32_t* inRT) {
    GSTRIDE_LOOP(v, n) {
        if (mark[v]) inRT[cid[v]] = 1;
    }
}

__global__ void k_reach_out(int32_t n, const int32_t* __restrict__ cid, const uint64_t* __restrict__ alpha,
                            const uint64_t* __restrict__ omega, uint32_t* __restrict__ x0, uint32_t* __restrict__ x1) {
    GSTRIDE_LOOP(v, n) {
        x0[v] = (uint32_t)alpha[cid[v]];
        x1[v] = (uint32_t)omega[cid[v]];
    }
}

template <class F>
bc_status cub_call(F&& f, DevBuf& tmp, hipStream_t s) {
    size_t bytes = 0;
    BC_HIP(f((void*)nullptr, bytes));
    if (tmp.bytes < bytes) BC_TRY(tmp.alloc_on(bytes, s));
    BC_HIP(f(tmp.p, bytes));
    return BC_OK;
}

bc_status read_i32(const int32_t* d, int32_t* h, hipStream_t s) {
    BC_HIP(hipMemcpyAsync(h, d, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    return BC_OK;
}

}  // namespace

bc_status directed_reach(bc_graph* g) {
    const int32_t n = g->dg.n;
    const int64_t m = g->dg.m;
    hipStream_t s = g->stream;
    const size_t N = (size_t)(n > 0 ? n : 1);
    DevBuf tmp, icnt, fill, flag;
    // in-CSR
    BC_TRY(galloc(g, g->irp, sizeof(int32_t) * (N + 1), s));
    BC_TRY(galloc(g, g->icol, sizeof(int32_t) * (size_t)(m > 0 ? m : 1), s));
    BC_TRY(icnt.alloc_on(sizeof(int32_t) * N, s));
    BC_TRY(fill.alloc_on(sizeof(int32_t) * N, s));
    BC_TRY(flag.alloc_on(sizeof(int32_t) * 4, s));
    int32_t* fl = flag.as<int32_t>();
    BC_HIP(hipMemsetAsync(icnt.p, 0, sizeof(int32_t) * N, s));
    BC_HIP(hipMemsetAsync(fill.p, 0, sizeof(int32_t) * N, s));
    if (n == 0) {
        BC_HIP(hipMemsetAsync(g->irp.p, 0, sizeof(int32_t), s));
        g->dg.irp = g->irp.as<int32_t>();
        g->dg.icol = g->icol.as<int32_t>();
        BC_HIP(hipStreamSynchronize(s));
        return BC_OK;
    }
    k_indeg<<<grid_for(n), kBlk, 0, s>>>(n, g->dg.rp, g->dg.col, icnt.as<int32_t>());
    BC_TRY(cub_call([&](void* t, size_t& b) {
        return hipcub::DeviceScan::ExclusiveSum(t, b, icnt.as<int32_t>(), g->irp.as<int32_t>(), n, s);
    }, tmp, s));
    k_close<<<1, 1, 0, s>>>(g->irp.as<int32_t>(), n, icnt.as<int32_t>());
    k_fill_in<<<grid_for(n), kBlk, 0, s>>>(n, g->dg.rp, g->dg.col, g->irp.as<int32_t>(), fill.as<int32_t>(),
                                           g->icol.as<int32_t>());
    g->dg.irp = g->irp.as<int32_t>();
    g->dg.icol = g->icol.as<int32_t>();
    const int32_t *rp = g->dg.rp, *col = g->dg.col, *irp = g->dg.irp, *icol = g->dg.icol;

    // ---- SCCs
    DevBuf comp, comp_next, color, mark, q0, q1, best;
    BC_TRY(comp.alloc_on(sizeof(int32_t) * N, s));
    BC_TRY(comp_next.alloc_on(sizeof(int32_t) * N, s));
    BC_TRY(color.alloc_on(sizeof(int32_t) * N, s));
    BC_TRY(mark.alloc_on(sizeof(uint32_t) * N, s));
    BC_TRY(q0.alloc_on(sizeof(int32_t) * N, s));
    BC_TRY(q1.alloc_on(sizeof(int32_t) * N, s));
    BC_TRY(best.alloc_on(sizeof(unsigned long long), s));
    int32_t* cp = comp.as<int32_t>();
    k_fill_i32<<<grid_for(n), kBlk, 0, s>>>(n, cp, -1);
    auto trim = [&](int passes) -> bc_status {
        for (int it = 0; it < passes; ++it) {
            BC_HIP(hipMemsetAsync(fl, 0, sizeof(int32_t), s));
            k_trim<<<grid_for(n), kBlk, 0, s>>>(n, rp, col, irp, icol, cp, fl);
            int32_t ch = 0;
            BC_TRY(read_i32(fl, &ch, s));
            if (!ch) break;
        }
        return BC_OK;
    };
    BC_TRY(trim(4));
    // forward-backward from the pivot of largest in-degree x out-degree
    {
        BC_HIP(hipMemsetAsync(best.p, 0, sizeof(unsigned long long), s));
        k_pivot<<<grid_for(n), kBlk, 0, s>>>(n, rp, irp, cp, best.as<unsigned long long>());
        unsigned long long bk = 0;
        BC_HIP(hipMemcpyAsync(&bk, best.p, sizeof(bk), hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        if ((bk >> 32) > 0) {
            int32_t pivot = (int32_t)(bk & 0xFFFFFFFFu);
            BC_HIP(hipMemsetAsync(mark.p, 0, sizeof(uint32_t) * N, s));
            for (int dir = 0; dir < 2; ++dir) {
                const int32_t* R = dir == 0 ? rp : irp;
                const int32_t* C = dir == 0 ? col : icol;
                uint32_t bit = 1u << dir;
                // seed: the pivot itself
                uint32_t pbits = 0;
                BC_HIP(hipMemcpyAsync(&pbits, mark.as<uint32_t>() + pivot, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
                BC_HIP(hipStreamSynchronize(s));
                pbits |= bit;
                BC_HIP(hipMemcpyAsync(mark.as<uint32_t>() + pivot, &pbits, sizeof(uint32_t), hipMemcpyHostToDevice, s));
                BC_HIP(hipMemcpyAsync(q0.p, &pivot, sizeof(int32_t), hipMemcpyHostToDevice, s));
                int32_t fn = 1;
                int32_t *fq = q0.as<int32_t>(), *nq = q1.as<int32_t>();
                while (fn > 0) {
                    BC_HIP(hipMemsetAsync(fl + 1, 0, sizeof(int32_t), s));
                    k_reach_level<<<grid_for(fn), kBlk, 0, s>>>(R, C, cp, mark.as<uint32_t>(), bit, fq, fn, nq, fl + 1);
                    BC_TRY(read_i32(fl + 1, &fn, s));
                    std::swap(fq, nq);
                }
            }
            k_fwbw_assign<<<grid_for(n), kBlk, 0, s>>>(n, mark.as<uint32_t>(), cp, pivot);
        }
    }
    BC_TRY(trim(4));
    // colouring rounds; every round assigns at least one node
    int32_t prev_left = n + 1;
    for (int round = 0;; ++round) {
        k_color_init<<<grid_for(n), kBlk, 0, s>>>(n, cp, color.as<int32_t>());
        for (;;) {
            BC_HIP(hipMemsetAsync(fl, 0, sizeof(int32_t), s));
            k_color_prop<<<grid_for(n), kBlk, 0, s>>>(n, irp, icol, cp, color.as<int32_t>(), fl);
            int32_t ch = 0;
            BC_TRY(read_i32(fl, &ch, s));
            if (!ch) break;
        }
        k_fill_i32<<<grid_for(n), kBlk, 0, s>>>(n, comp_next.as<int32_t>(), -1);
        k_color_roots<<<grid_for(n), kBlk, 0, s>>>(n, color.as<int32_t>(), comp_next.as<int32_t>());
        for (;;) {
            BC_HIP(hipMemsetAsync(fl, 0, sizeof(int32_t), s));
            k_color_back<<<grid_for(n), kBlk, 0, s>>>(n, rp, col, cp, color.as<int32_t>(), comp_next.as<int32_t>(), fl);
            int32_t ch = 0;
            BC_TRY(read_i32(fl, &ch, s));
            if (!ch) break;
        }
        BC_HIP(hipMemsetAsync(fl + 2, 0, sizeof(int32_t), s));
        k_color_commit<<<grid_for(n), kBlk, 0, s>>>(n, cp, comp_next.as<int32_t>(), fl + 2);
        int32_t left = 0;
        BC_TRY(read_i32(fl + 2, &left, s));
        if (left == 0) break;
        if (left >= prev_left) {
            set_error("SCC colouring made no progress (%d nodes left)", left);
            return BC_EDEVICE;
        }
        prev_left = left;
        BC_TRY(trim(2));
    }

    // ---- condensation DAG and the alpha/omega recurrence
    DevBuf rootpos, cid, wsize, keys, keys2, dcnt, drp, dfill, dcol, alpha, omega, done;
    BC_TRY(rootpos.alloc_on(sizeof(int32_t) * (N + 1), s));
    BC_TRY(cid.alloc_on(sizeof(int32_t) * N, s));
    k_is_root<<<grid_for(n), kBlk, 0, s>>>(n, cp, color.as<int32_t>());
    BC_TRY(cub_call([&](void* t, size_t& b) {
        return hipcub::DeviceScan::ExclusiveSum(t, b, color.as<int32_t>(), rootpos.as<int32_t>(), n, s);
    }, tmp, s));
    k_close<<<1, 1, 0, s>>>(rootpos.as<int32_t>(), n, color.as<int32_t>());
    int32_t nc = 0;
    BC_TRY(read_i32(rootpos.as<int32_t>() + n, &nc, s));
    const size_t NC = (size_t)(nc > 0 ? nc : 1);
    BC_TRY(wsize.alloc_on(sizeof(uint32_t) * NC, s));
    BC_HIP(hipMemsetAsync(wsize.p, 0, sizeof(uint32_t) * NC, s));
    k_cid<<<grid_for(n), kBlk, 0, s>>>(n, cp, rootpos.as<int32_t>(), cid.as<int32_t>(), wsize.as<uint32_t>());
    BC_TRY(keys.alloc_on(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1), s));
    BC_TRY(keys2.alloc_on(sizeof(uint64_t) * (size_t)(m > 0 ? m : 1), s));
    BC_HIP(hipMemsetAsync(fl + 3, 0, sizeof(int32_t), s));
    k_dag_arcs<<<grid_for(n), kBlk, 0, s>>>(n, rp, col, cid.as<int32_t>(), keys.as<uint64_t>(), fl + 3);
    int32_t na = 0;
    BC_TRY(read_i32(fl + 3, &na, s));
    if (na > 0) {
        BC_TRY(cub_call([&](void* t, size_t& b) {
            return hipcub::DeviceRadixSort::SortKeys(t, b, keys.as<uint64_t>(), keys2.as<uint64_t>(), na, 0, 64, s);
        }, tmp, s));
    }
    BC_TRY(dcnt.alloc_on(sizeof(int32_t) * NC, s));
    BC_TRY(drp.alloc_on(sizeof(int32_t) * (NC + 1), s));
    BC_TRY(dfill.alloc_on(sizeof(int32_t) * NC, s));
    BC_TRY(dcol.alloc_on(sizeof(int32_t) * (size_t)(na > 0 ? na : 1), s));
    BC_HIP(hipMemsetAsync(dcnt.p, 0, sizeof(int32_t) * NC, s));
    BC_HIP(hipMemsetAsync(dfill.p, 0, sizeof(int32_t) * NC, s));
    if (na > 0) k_dag_count<<<grid_for(na), kBlk, 0, s>>>(na, keys2.as<uint64_t>(), dcnt.as<int32_t>());
    BC_TRY(cub_call([&](void* t, size_t& b) {
        return hipcub::DeviceScan::ExclusiveSum(t, b, dcnt.as<int32_t>(), drp.as<int32_t>(), nc, s);
    }, tmp, s));
    k_close<<<1, 1, 0, s>>>(drp.as<int32_t>(), nc, dcnt.as<int32_t>());
    if (na > 0)
        k_dag_fill<<<grid_for(na), kBlk, 0, s>>>(na, keys2.as<uint64_t>(), drp.as<int32_t>(), dfill.as<int32_t>(),
                                                 dcol.as<int32_t>());
    BC_TRY(alpha.alloc_on(sizeof(uint64_t) * NC, s));
    BC_TRY(omega.alloc_on(sizeof(uint64_t) * NC, s));
    BC_TRY(done.alloc_on(sizeof(int32_t) * NC, s));
    BC_HIP(hipMemsetAsync(done.p, 0, sizeof(int32_t) * NC, s));
    // largest-SCC refinement: T, its exact reach, the components in R(T)
    BigScc big{-1, 0, nullptr, nullptr, nullptr};
    DevBuf inRT, omega2, toT;
    if (g->big_scc && nc > 0) {
        BC_HIP(hipMemsetAsync(best.p, 0, sizeof(unsigned long long), s));
        k_big_pick<<<grid_for(n), kBlk, 0, s>>>(n, cid.as<int32_t>(), wsize.as<uint32_t>(),
                                                best.as<unsigned long long>());
        unsigned long long bk = 0;
        BC_HIP(hipMemcpyAsync(&bk, best.p, sizeof(bk), hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        const int32_t root = 0x7FFFFFFF - (int32_t)(uint32_t)(bk & 0xFFFFFFFFu);
        if (root < 0 || root >= n) {
            set_error("internal: largest SCC root %d out of range", root);
            return BC_EDEVICE;
        }
        uint32_t* mk = mark.as<uint32_t>();
        BC_HIP(hipMemsetAsync(mk, 0, sizeof(uint32_t) * N, s));
        const uint32_t one = 1;
        BC_HIP(hipMemcpyAsync(mk + root, &one, sizeof(uint32_t), hipMemcpyHostToDevice, s));
        BC_HIP(hipMemcpyAsync(q0.p, &root, sizeof(int32_t), hipMemcpyHostToDevice, s));
        uint64_t reached = 1;
        int32_t fn = 1;
        int32_t *fq = q0.as<int32_t>(), *nq = q1.as<int32_t>();
        while (fn > 0) {
            BC_HIP(hipMemsetAsync(fl + 1, 0, sizeof(int32_t), s));
            k_bfs_level<<<grid_for(fn), kBlk, 0, s>>>(rp, col, mk, fq, fn, nq, fl + 1);
            BC_TRY(read_i32(fl + 1, &fn, s));
            reached += (uint64_t)fn;
            std::swap(fq, nq);
        }
        int32_t c_big = 0;
        BC_TRY(read_i32(cid.as<int32_t>() + root, &c_big, s));
        BC_TRY(inRT.alloc_on(sizeof(int32_t) * NC, s));
        BC_TRY(omega2.alloc_on(sizeof(uint64_t) * NC, s));
        BC_TRY(toT.alloc_on(sizeof(int32_t) * NC, s));
        BC_HIP(hipMemsetAsync(inRT.p, 0, sizeof(int32_t) * NC, s));
        BC_HIP(hipMemsetAsync(toT.p, 0, sizeof(int32_t) * NC, s));
        k_mark_comps<<<grid_for(n), kBlk, 0, s>>>(n, mk, cid.as<int32_t>(), inRT.as<int32_t>());
        big = BigScc{c_big, reached, inRT.as<int32_t>(), omega2.as<uint64_t>(), toT.as<int32_t>()};
    }
    for (int32_t prev = nc + 1;;) {
        BC_HIP(hipMemsetAsync(fl, 0, sizeof(int32_t), s));
        k_dag_round<<<grid_for(nc), kBlk, 0, s>>>(nc, drp.as<int32_t>(), dcol.as<int32_t>(), wsize.as<uint32_t>(),
                                                  alpha.as<uint64_t>(), omega.as<uint64_t>(), done.as<int32_t>(),
                                                  (uint64_t)n, fl, big);
        int32_t left = 0;
        BC_TRY(read_i32(fl, &left, s));
        if (left == 0) break;
        if (left >= prev) {
            set_error("condensation DAG has a cycle (%d components unresolved)", left);
            return BC_EDEVICE;
        }
        prev = left;
    }
    k_reach_out<<<grid_for(n), kBlk, 0, s>>>(n, cid.as<int32_t>(), alpha.as<uint64_t>(), omega.as<uint64_t>(),
                                             g->x0.as<uint32_t>(), g->x1.as<uint32_t>());
    BC_HIP(hipStreamSynchronize(s));
    return BC_OK;
}

}  // namespace bc
