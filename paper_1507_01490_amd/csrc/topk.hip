// Top-k closeness on gfx950: Algorithm 1 with the BFSCut function
// (Section 2.5), run as bit-parallel multi-source BFS.
//
// A batch holds W = 64 * WW sources, one bit each.  Every node has one
// record per batch slot (SW uint64 words, node-major, one 32/64/128-byte
// block so that every per-node access touches one cache line):
//   seen[WW]   sources that have reached the node      (the "visited" marks)
//   nxt[WW]    sources reaching it in the level being built
//   cur[WW]    sources for which it is in the current frontier Gamma_d
//   meta       low 32 bits: first-touch stamp (WW > 1); high 32 bits: out-degree
// plus three node lists of capacity n: the current frontier F (compacted to
// nodes with a live source bit), the nodes reached by the level being built
// N (each once per level), and the reset list (each node once, when its seen
// mask first becomes non-zero) that clears the marks when the batch ends.
//
// Per source (SrcState) the counters of Table 1 are kept exactly:
//   nd = n_d (nodes within distance d), fd = f_d (distance sum over them),
//   tg = ~gamma_{d+1} (sum of out-degrees over Gamma_d), mvis (arcs a
//   sequential search of this source scans).
// One level: expand F (every arc u->w with a live bit of cur[u] not yet in
// seen[w] ORs it into nxt[w]); the thread whose atomic OR newly sets bit b of
// nxt[w] adds 1 to gamma_{d+1}(b) and deg(w) to ~gamma_{d+2}(b), so each
// (node, source) pair is counted once.  A source with gamma = 0 is complete
// (r = nd, f = fd); every other live source is tested against the current
// k-th best record with the bound of Lemma 1 (undirected, x = r(v)) or
// Lemma 2 (directed, x in {alpha(v), omega(v)}), and its bit is retired when
// it cannot enter the top-k.  Only then is the new level materialised
// (seen |= nxt & live, cur = nxt & live), and only for live bits; when no
// source of the batch is left, the pass just resets nxt.
//
// The k-th best record: a device top-k list guarded by a lock, plus an
// append-only ring of immutable threshold records and a monotone sequence
// number.  A reader takes the record at seq-1; any record it can see is <=
// the true k-th best, and a stale one only weakens the cut (the shared value
// of the parallel loop, Section 2.1), so results never change.
#include <chrono>
#include <condition_variable>
#include <cstddef>
#include <cstring>

#include <hip/hip_cooperative_groups.h>

#include "bc_internal.h"

namespace bc {

namespace {

constexpr int kBlk = 256;  // threads per workgroup in every level kernel (and the most sources per batch)
constexpr int kBatchBlk = 1024;  // threads per workgroup of the persistent batched kernel

// words per node record: seen, nxt, cur (WW each) + meta, padded to 32/64/128 B
template <int WW>
struct Layout {
    static constexpr int SW = WW == 1 ? 4 : (WW == 2 ? 8 : 16);
    static constexpr int NXT = WW, CUR = 2 * WW, META = 3 * WW;
};

enum : int32_t { S_EMPTY = 0, S_LIVE = 1, S_CUT = 2, S_DONE = 3, S_TRIVIAL = 4, S_DEFER = 5 };

struct SrcState {
    int32_t id, status;   // id: the node in the graph's own numbering (what the batch traverses)
    uint32_t x0, x1;
    int32_t oid, pad_;    // oid: the caller's id of the node (ties, results, per-node outputs)
    uint64_t nd, fd, tg, mvis;
};

struct Rec {           // one completed source; fields read/written atomically
    uint64_t A, F;     // (r-1)^2 and f, or (0, 1) when r = 1
    uint64_t f;        // exact farness
    uint64_t idr;      // id (low 32 bits) | r (high 32 bits)
};

struct ThRec {         // immutable threshold record
    uint64_t A, F;
    int64_t id;
};

struct QStats {
    unsigned long long m_vis, node_arcs, levels, pull_levels, n_cut, n_done, n_trivial, batches;
    unsigned long long frontier_entries, discovered, n_deferred;
    unsigned long long phase_ticks[5];  // persistent kernel: set-up, expand, cut, build, reset (100 MHz)
    unsigned long long lds_levels, record_levels, spills;  // LDS-table levels, node-record levels, moves
    unsigned long long record_ticks, record_arcs;          // persistent levels on node records: time, arcs
};

// Sources handed from the persistent kernel to the level-synchronous kernels
// (a source whose next level would scan more than the budget of arcs).
struct DeferList {
    int32_t* ids;       // capacity n
    uint32_t* cnt;
    uint64_t budget;    // 0: never defer
};

struct TopKDev {
    int32_t k;
    int32_t* cnt;
    uint32_t* lock;
    uint32_t* seq;
    Rec* list;
    ThRec* ring;
    // every-node mode (no top-k list, no threshold): completed sources write
    // their exact farness and reach here, indexed by node id
    uint64_t* all_f;
    uint32_t* all_r;
    // undirected graph with the footnote bound of Section 2.3: for d >= 1,
    // ~gamma_{d+1} = sum of (deg - 1) over Gamma_d
    int32_t footnote;
};

// Level-synchronous control block (device memory) of the plain slot.
struct Ctl {
    uint32_t d, flen, nlen, clen;  // level, frontier length, reached-list and reset-list counters
    uint32_t live, pull, chunk, done_blocks;
    uint32_t stamp, ran;           // ran: a level kernel ran in this step (captured level steps)
    unsigned long long front_arcs, acc_arcs;
    unsigned long long active[4];
    uint32_t cnt_g[256];
    unsigned long long cnt_t[256];
    uint32_t err;                  // cooperative level loop: a list outgrew n (the loop stopped)
};

struct SlotPtrs {
    uint64_t* ns;   // n * SW node records
    int32_t* qa;    // n, frontier list F
    int32_t* qb;    // n, reached list N
    int32_t* clr;   // n, reset list
};

struct LevelParams {
    float pull_alpha, pull_beta;
    int32_t can_pull;
};

// ------------------------------------------------------------ helpers

__device__ inline uint64_t ld64(const uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void st64(uint64_t* p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline int32_t ld32(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t ldu32(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// A value that every lane of the workgroup holds alike (read from LDS after a
// barrier) moved to a scalar register, so that the branches and counters
// that depend on it stay scalar instead of taking vector registers.
__device__ inline uint32_t uni32(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ inline uint64_t uni64(uint64_t v) {
    return ((uint64_t)uni32((uint32_t)(v >> 32)) << 32) | (uint64_t)uni32((uint32_t)v);
}

// key(x) > key(y): A_x F_y > A_y F_x in 128 bits, ties by the smaller id
__device__ inline bool key_gt(uint64_t Ax, uint64_t Fx, int32_t ix, uint64_t Ay, uint64_t Fy, int32_t iy) {
    unsigned __int128 a = (unsigned __int128)Ax * Fy;
    unsigned __int128 b = (unsigned __int128)Ay * Fx;
    if (a != b) return a > b;
    return ix < iy;
}

// Insert one completed source into the top-k list (caller serialises).  When
// the list is full afterwards, publish its k-th record.
__device__ void topk_insert(const TopKDev& T, uint64_t A, uint64_t F, uint64_t f, int32_t id, uint32_t r) {
    const int32_t k = T.k;
    int32_t c = ld32(T.cnt);
    if (c == k) {
        Rec* last = &T.list[k - 1];
        if (!key_gt(A, F, id, ld64(&last->A), ld64(&last->F), (int32_t)(uint32_t)ld64(&last->idr))) return;
    }
    int32_t i;
    if (c < k) {
        i = c;
        c += 1;
        __hip_atomic_store(T.cnt, c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else {
        i = k - 1;
    }
    while (i > 0) {
        Rec* y = &T.list[i - 1];
        uint64_t yA = ld64(&y->A), yF = ld64(&y->F), yidr = ld64(&y->idr);
        if (!key_gt(A, F, id, yA, yF, (int32_t)(uint32_t)yidr)) break;
        Rec* z = &T.list[i];
        st64(&z->A, yA);
        st64(&z->F, yF);
        st64(&z->f, ld64(&y->f));
        st64(&z->idr, yidr);
        --i;
    }
    Rec* z = &T.list[i];
    st64(&z->A, A);
    st64(&z->F, F);
    st64(&z->f, f);
    st64(&z->idr, ((uint64_t)r << 32) | (uint32_t)id);
    if (c == k) {
        uint32_t s = __hip_atomic_load(T.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        Rec* kth = &T.list[k - 1];
        ThRec* o = &T.ring[s];
        st64(&o->A, ld64(&kth->A));
        st64(&o->F, ld64(&kth->F));
        st64((uint64_t*)&o->id, (uint64_t)(int64_t)(int32_t)(uint32_t)ld64(&kth->idr));
        __hip_atomic_store(T.seq, s + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// The record at seq-1 was written before seq was published with a release
// store at agent scope; the acquire load of seq here pairs with it, so the
// record's three words are visible once seq is (the ring itself is never
// cleared between queries).  A record with F = 0 cannot be a published one
// (F = f >= 1 for r >= 2, and F = 1 for r = 1) and is treated as no threshold,
// which is always safe: it only means no source is cut.
__device__ inline bool load_threshold(const TopKDev& T, ThRec* th) {
    uint32_t s = __hip_atomic_load(T.seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
    if (s == 0) return false;
    ThRec* r = &T.ring[s - 1];
    th->A = ld64(&r->A);
    th->F = ld64(&r->F);
    th->id = (int64_t)ld64((const uint64_t*)&r->id);
    return th->F != 0;
}

__device__ inline void lock_acquire(uint32_t* l) {
    while (atomicCAS(l, 0u, 1u) != 0u) __builtin_amdgcn_s_sleep(2);
    __atomic_thread_fence(__ATOMIC_ACQUIRE);
}
__device__ inline void lock_release(uint32_t* l) {
    __hip_atomic_store(l, 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

// The cut rule at level d for a live source (Lemma 1 / Lemma 2 with the
// current k-th best record th).  For each candidate reach x,
//   L_x = f_d - ~gamma_{d+1} + (d+2)(x - n_d)   (farness lower bound),
// and the source cannot enter the top-k when L_x / (x-1)^2 > F/A for every
// x, or >= for every x with the source id larger than th.id.
__device__ inline bool cut_rule(const SrcState& s, uint32_t d, const ThRec& th) {
    const uint32_t xs[2] = {s.x0, s.x1};
    const int nx = s.x1 != s.x0 ? 2 : 1;
    bool all_gt = true, all_ge = true;
    for (int i = 0; i < nx; ++i) {
        const int64_t x = (int64_t)xs[i];
        const int64_t L = (int64_t)s.fd - (int64_t)s.tg + (int64_t)(d + 2) * (x - (int64_t)s.nd);
        if (L <= 0) return false;
        const unsigned __int128 lhs = (unsigned __int128)(uint64_t)L * th.A;
        const unsigned __int128 rhs = (unsigned __int128)th.F * (uint64_t)((x - 1) * (x - 1));
        all_gt = all_gt && (lhs > rhs);
        all_ge = all_ge && (lhs >= rhs);
    }
    return all_gt || (all_ge && (int64_t)s.oid > th.id);
}

__device__ inline uint32_t lane_id() { return __lane_id(); }

// Seen filter of a batch on the node records: one bit per hashed node id
// (2^17 bits in LDS), set for every node that has a seen bit in the records.
// A clear bit proves the node unseen, so its record need not be read.
constexpr uint32_t kFiltBits = 1u << 17;
__device__ inline uint32_t filter_hash(int32_t w) { return ((uint32_t)w * 0x9E3779B1u) >> 15; }
__device__ inline void filter_set(uint32_t* f, int32_t w) {
    const uint32_t h = filter_hash(w);
    atomicOr(&f[h >> 5], 1u << (h & 31));
}
__device__ inline bool filter_maybe(const uint32_t* f, int32_t w) {
    const uint32_t h = filter_hash(w);
    return (f[h >> 5] >> (h & 31)) & 1u;
}

// Wave-aggregated append of w to list[] when `app` holds.
__device__ inline void append_if(bool app, int32_t w, int32_t* list, uint32_t* ctr) {
    unsigned long long bal = __ballot(app);
    if (bal == 0) return;
    const int lane = (int)lane_id();
    const int leader = __ffsll((long long)bal) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(ctr, (uint32_t)__popcll(bal));
    base = __shfl(base, leader);
    if (app) list[base + __popcll(bal & ((1ull << lane) - 1ull))] = w;
}

// Workgroup-aggregated append of w[u] where app[u] holds, u < N: one atomic
// on the global counter per workgroup and call instead of one per wave (the
// level-synchronous kernels' counters are single words that every wave of
// the grid would otherwise hit).  sh: B / 64 + 1 words of LDS.  Call with
// the whole workgroup.
template <int B, int N>
__device__ inline void block_append(const bool* app, const int32_t* w, int32_t* list, uint32_t* ctr, uint32_t* sh) {
    const int lane = (int)lane_id();
    const int wave = threadIdx.x >> 6;
    unsigned long long bal[N];
    uint32_t wc = 0;
#pragma unroll
    for (int u = 0; u < N; ++u) {
        bal[u] = __ballot(app[u]);
        wc += (uint32_t)__popcll(bal[u]);
    }
    if (lane == 0) sh[wave] = wc;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int i = 0; i < B / 64; ++i) {
            const uint32_t x = sh[i];
            sh[i] = t;
            t += x;
        }
        sh[B / 64] = t ? atomicAdd(ctr, t) : 0u;
    }
    __syncthreads();
    uint32_t pos = sh[B / 64] + sh[wave];
    const unsigned long long lt = (1ull << lane) - 1ull;
#pragma unroll
    for (int u = 0; u < N; ++u) {
        if (app[u]) list[pos + (uint32_t)__popcll(bal[u] & lt)] = w[u];
        pos += (uint32_t)__popcll(bal[u]);
    }
    __syncthreads();  // sh is reused by the next call
}

// gamma(b) += 1 and tgamma(b) += deg for every bit b of `bits` (word j)
__device__ inline void count_new(uint64_t bits, int j, uint32_t deg, uint32_t* cg, unsigned long long* ct) {
    while (bits) {
        const int b = __ffsll((long long)bits) - 1;
        bits &= bits - 1ull;
        atomicAdd(&cg[j * 64 + b], 1u);
        atomicAdd(&ct[j * 64 + b], (unsigned long long)deg);
    }
}

// Transpose of the 64 x 64 bit matrix held one row per lane (row = lane,
// column = bit): afterwards lane b holds column b, bit i = bit b of lane i.
// Six butterfly stages; at stage s a lane keeps the half of its row whose
// column bit s equals its own lane bit s and takes the other half from lane
// lane ^ s.  Wave-uniform call.
__device__ inline uint64_t transpose64(uint64_t x) {
    const uint32_t lane = lane_id();
    constexpr uint64_t kM[6] = {0x00000000FFFFFFFFull, 0x0000FFFF0000FFFFull, 0x00FF00FF00FF00FFull,
                                0x0F0F0F0F0F0F0F0Full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int st = 0; st < 6; ++st) {
        const int sh = 32 >> st;
        const uint64_t m = kM[st];
        const uint64_t y = __shfl_xor(x, sh);
        x = (lane & (uint32_t)sh) ? ((x & ~m) | ((y & ~m) >> sh)) : ((x & m) | ((y & m) << sh));
    }
    return x;
}

// Per-source counts of a wave of newly reached nodes: lane i holds the nxt
// bits nb[j] of its node and the node's out-degree; lane b of the wave adds,
// for source j * 64 + b, the number of nodes with bit b and the sum of their
// degrees (the degree is taken bit plane by bit plane: plane k is a ballot,
// and the sum is the popcounts of the column masked by each plane, shifted).
// Wave-uniform call.
template <int WW>
__device__ inline void wave_count_nodes(const uint64_t* nb, uint32_t deg, uint32_t* cg, unsigned long long* ct) {
    uint64_t col[WW];
    bool any = false;
#pragma unroll
    for (int j = 0; j < WW; ++j) {
        const bool has = __ballot(nb[j] != 0ull) != 0ull;
        col[j] = has ? transpose64(nb[j]) : 0ull;
        any |= has;
    }
    if (!any) return;
    unsigned long long t[WW];
#pragma unroll
    for (int j = 0; j < WW; ++j) t[j] = 0;
    for (int k = 0; k < 32; ++k) {
        if (__ballot((deg >> k) != 0u) == 0ull) break;
        const uint64_t plane = __ballot(((deg >> k) & 1u) != 0u);
#pragma unroll
        for (int j = 0; j < WW; ++j) t[j] += (unsigned long long)__popcll(col[j] & plane) << k;
    }
    const uint32_t lane = lane_id();
#pragma unroll
    for (int j = 0; j < WW; ++j) {
        const uint32_t g = (uint32_t)__popcll(col[j]);
        if (g) {
            atomicAdd(&cg[j * 64 + lane], g);
            atomicAdd(&ct[j * 64 + lane], t[j]);
        }
    }
}

// Counters of the level just reached, from its list N[0, len) of newly
// reached nodes (each once) after the expansion: the nxt masks are read from
// L2 (they were written by atomics this level).  The out-degree comes from
// the record's meta word, or from degs[] when the records are shared by the
// batches of several graphs (their meta words then hold no degree).
template <int WW, int B>
__device__ void count_level(const SlotPtrs& P, const int32_t* N, uint32_t len, uint32_t* cg, unsigned long long* ct,
                            const uint32_t* degs = nullptr) {
    using Lo = Layout<WW>;
    const uint32_t tid = threadIdx.x;
    for (uint32_t rb = 0; rb < len; rb += B) {
        if (rb + (tid & ~63u) >= len) break;  // wave-uniform: nothing left for this wave
        const uint32_t i = rb + tid;
        uint64_t nb[WW];
        uint32_t deg = 0;
#pragma unroll
        for (int j = 0; j < WW; ++j) nb[j] = 0;
        if (i < len) {
            uint64_t* rec = &P.ns[(size_t)N[i] * Lo::SW];
#pragma unroll
            for (int j = 0; j < WW; ++j)
                nb[j] = __hip_atomic_load(&rec[Lo::NXT + j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            deg = degs ? degs[N[i]] : (uint32_t)(rec[Lo::META] >> 32);
        }
        wave_count_nodes<WW>(nb, deg, cg, ct);
    }
}

// Arc u->w for the live source bits m of u: OR the unseen ones into nxt[w]
// (the per-source counters are taken later, once per reached node).  Returns
// whether w is new this level.
template <int WW>
__device__ inline bool visit(uint64_t* rec, const uint64_t* m, uint32_t stamp) {
    using Lo = Layout<WW>;
    uint64_t nb[WW];
    uint64_t any = 0;
    if constexpr (WW == 1) {
        // seen and nxt share one 16-byte load; a stale nxt only costs an extra atomic
        const ulonglong2 sn = *reinterpret_cast<const ulonglong2*>(rec);
        nb[0] = m[0] & ~(sn.x | sn.y);
        any = nb[0];
    } else {
#pragma unroll
        for (int j = 0; j < WW; ++j) {
            nb[j] = m[j] & ~(rec[j] | rec[Lo::NXT + j]);
            any |= nb[j];
        }
    }
    if (!any) return false;
    if constexpr (WW == 1) {
        // one word: the first toucher is the one that finds nxt empty (stamp unused)
        (void)stamp;
        return atomicOr((unsigned long long*)&rec[Lo::NXT], (unsigned long long)nb[0]) == 0ull;
    } else {
#pragma unroll
        for (int j = 0; j < WW; ++j)
            if (nb[j]) atomicOr((unsigned long long*)&rec[Lo::NXT + j], (unsigned long long)nb[j]);
        return atomicMax(reinterpret_cast<uint32_t*>(&rec[Lo::META]), stamp) < stamp;
    }
}

// Block-wide exclusive scan of one uint32 per thread (B threads).
template <int B = kBlk>
__device__ inline uint32_t block_exscan(uint32_t v, uint32_t* tmp /* B/64 + 1 */, uint32_t* total) {
    const int lane = (int)lane_id();
    const int wave = threadIdx.x / 64;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) tmp[wave] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int i = 0; i < B / 64; ++i) {
            uint32_t t = tmp[i];
            tmp[i] = acc;
            acc += t;
        }
        tmp[B / 64] = acc;
    }
    __syncthreads();
    uint32_t r = tmp[wave] + x - v;
    *total = tmp[B / 64];
    __syncthreads();
    return r;
}

template <int WW, int B = kBlk>
struct LdsExpand {
    int32_t beg[B];
    uint32_t off[B + 1];
    uint64_t m[B * WW];
    uint32_t scan[B / 64 + 1];
    uint32_t chunk;
};

// Expand entries [e0, e1) (at most kBlk) of the frontier list F: every arc of
// every entry with a live bit, balanced over the workgroup by a scan of the
// degrees.  Nodes reached for the first time this level go to N once.  Each
// thread takes kArcs arcs per round (a, a + B, ...) and issues all their
// target loads before it visits any target's record: two in the
// level-synchronous kernel, one in the persistent kernels, where the second
// arc's registers cost more than its overlap gains.
template <int WW, int B = kBlk, int kArcs = 2, bool kBlockAppend = false>
__device__ void expand_entries(const DevGraph& G, const SlotPtrs& P, const int32_t* F, uint32_t e0, uint32_t e1,
                               const uint64_t* act, int32_t* N, uint32_t* nctr, uint32_t stamp, LdsExpand<WW, B>& L,
                               unsigned long long* arcs, unsigned long long* entries, uint32_t* bsh = nullptr) {
    using Lo = Layout<WW>;
    const int tid = threadIdx.x;
    const uint32_t e = e0 + tid;
    uint32_t deg = 0;
    int32_t beg = 0;
    uint64_t m[WW];
#pragma unroll
    for (int j = 0; j < WW; ++j) m[j] = 0;
    if (e < e1) {
        const int32_t u = F[e];
        const uint64_t* rec = &P.ns[(size_t)u * Lo::SW];
        uint64_t any = 0;
#pragma unroll
        for (int j = 0; j < WW; ++j) {
            m[j] = rec[Lo::CUR + j] & act[j];
            any |= m[j];
        }
        if (any) {
            beg = G.rp[u];
            deg = (uint32_t)(G.rp[u + 1] - beg);
        }
    }
    const unsigned long long nlive = __ballot(deg != 0);
    if ((tid & 63) == 0 && nlive) atomicAdd(entries, (unsigned long long)__popcll(nlive));
    L.beg[tid] = beg;
#pragma unroll
    for (int j = 0; j < WW; ++j) L.m[tid * WW + j] = m[j];
    uint32_t total;
    const uint32_t off = block_exscan<B>(deg, L.scan, &total);
    L.off[tid] = off;
    __syncthreads();
    if constexpr (kArcs == 1) {
        for (uint32_t a0 = 0; a0 < total; a0 += B) {
            const uint32_t a = a0 + tid;
            bool app = false;
            int32_t w = 0;
            if (a < total) {
                // owner entry: the last i with off[i] <= a (off[0] = 0 <= a)
                uint32_t lo = 0, hi = B;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (L.off[mid] <= a) lo = mid + 1; else hi = mid;
                }
                const uint32_t i = lo - 1;
                w = G.col[L.beg[i] + (int32_t)(a - L.off[i])];
                app = visit<WW>(&P.ns[(size_t)w * Lo::SW], &L.m[i * WW], stamp);
            }
            if constexpr (kBlockAppend) block_append<B, 1>(&app, &w, N, nctr, bsh);
            else append_if(app, w, N, nctr);
        }
    } else {
        for (uint32_t a0 = 0; a0 < total; a0 += kArcs * B) {
            bool app[kArcs];
            int32_t w[kArcs];
            uint32_t own[kArcs];
#pragma unroll
            for (int u = 0; u < kArcs; ++u) {
                app[u] = false;
                w[u] = 0;
                own[u] = 0;
                const uint32_t a = a0 + (uint32_t)u * B + tid;
                if (a < total) {
                    // owner entry: the last i with off[i] <= a (off[0] = 0 <= a)
                    uint32_t lo = 0, hi = B;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (L.off[mid] <= a) lo = mid + 1; else hi = mid;
                    }
                    own[u] = lo - 1;
                    w[u] = G.col[L.beg[own[u]] + (int32_t)(a - L.off[own[u]])];
                    app[u] = true;
                }
            }
#pragma unroll
            for (int u = 0; u < kArcs; ++u)
                if (app[u]) app[u] = visit<WW>(&P.ns[(size_t)w[u] * Lo::SW], &L.m[own[u] * WW], stamp);
            if constexpr (kBlockAppend) {
                block_append<B, kArcs>(app, w, N, nctr, bsh);
            } else {
#pragma unroll
                for (int u = 0; u < kArcs; ++u) append_if(app[u], w[u], N, nctr);
            }
        }
    }
    if (tid == 0) *arcs += total;
    __syncthreads();
}

// Zero the cur masks of the list entries [first, len) (stride).
template <int WW>
__device__ inline void clear_cur(const SlotPtrs& P, const int32_t* F, uint32_t len, uint32_t first, uint32_t stride) {
    using Lo = Layout<WW>;
    for (uint32_t i = first + threadIdx.x; i < len; i += stride) {
        uint64_t* rec = &P.ns[(size_t)F[i] * Lo::SW];
#pragma unroll
        for (int j = 0; j < WW; ++j) rec[Lo::CUR + j] = 0;
    }
}

// Build the new frontier from the reached list N[0, len) once the cut step
// has run: nxt is reset everywhere; the live bits go to seen and cur, nodes
// with a live bit go to the frontier list F, first-seen nodes to the reset
// list.  With no live bit at all only nxt is reset.  Block-uniform loop.
// kFresh: the caller's compute unit holds no copy of the records that
// predates the level's atomic updates (a kernel of its own, or after a grid
// barrier's acquire), so nxt is read with a plain load; otherwise (the
// persistent kernels, whose own plain loads may have cached a record before
// the atomics changed it) it is taken with an exchange.
template <int WW, bool kFresh = false>
__device__ void build_level(const SlotPtrs& P, const int32_t* N, uint32_t len, uint32_t first, uint32_t stride,
                            const uint64_t* act, bool any_live, int32_t* F, uint32_t* fctr, uint32_t* clen,
                            unsigned long long* arcs, uint32_t* seen_filter = nullptr, uint32_t* bsh = nullptr) {
    using Lo = Layout<WW>;
    const int tid = threadIdx.x;
    unsigned long long my_arcs = 0;
    for (uint32_t rb = first; rb < len; rb += stride) {
        const uint32_t i = rb + tid;
        bool keep = false, fresh = false;
        int32_t w = 0;
        if (i < len) {
            w = N[i];
            uint64_t* rec = &P.ns[(size_t)w * Lo::SW];
            if (!any_live) {
#pragma unroll
                for (int j = 0; j < WW; ++j) rec[Lo::NXT + j] = 0;
            } else {
                uint64_t nb[WW];
                uint64_t any = 0;
                if constexpr (kFresh) {
#pragma unroll
                    for (int j = 0; j < WW; ++j) nb[j] = rec[Lo::NXT + j];
#pragma unroll
                    for (int j = 0; j < WW; ++j) {
                        rec[Lo::NXT + j] = 0;
                        nb[j] &= act[j];
                        any |= nb[j];
                    }
                } else {
#pragma unroll
                    for (int j = 0; j < WW; ++j) {
                        nb[j] = atomicExch((unsigned long long*)&rec[Lo::NXT + j], 0ull) & act[j];
                        any |= nb[j];
                    }
                }
                if (any) {
                    uint64_t old_any = 0;
#pragma unroll
                    for (int j = 0; j < WW; ++j) {
                        const uint64_t old = rec[j];
                        old_any |= old;
                        rec[j] = old | nb[j];
                        rec[Lo::CUR + j] = nb[j];
                    }
                    keep = true;
                    fresh = old_any == 0ull;
                    my_arcs += (uint32_t)(rec[Lo::META] >> 32);
                    if (seen_filter) filter_set(seen_filter, w);
                }
            }
        }
        if (any_live) {
            if constexpr (kFresh) {
                // a kernel of its own over the whole grid: one global atomic
                // per workgroup and list (kBlk threads)
                block_append<kBlk, 1>(&keep, &w, F, fctr, bsh);
                block_append<kBlk, 1>(&fresh, &w, P.clr, clen, bsh);
            } else {
                append_if(keep, w, F, fctr);
                append_if(fresh, w, P.clr, clen);
            }
        }
    }
    if (my_arcs) atomicAdd(arcs, my_arcs);
}

// The per-level decision for the W sources of a batch (first W threads of one
// workgroup).  With apply = true, first fold the counters of the level just
// reached (gamma == 0 completes a source).  Then insert completions into the
// top-k, read the threshold, and cut (or defer).  Writes the active masks
// and returns the live count (to every thread).
struct CutLds {
    uint32_t flags[kBlk];
    ThRec th;
    uint32_t have_th, live;
};

template <int WW>
__device__ uint32_t cut_step(const TopKDev& T, SrcState* S, int W, uint32_t d, bool apply, const uint32_t* cg,
                             const unsigned long long* ct, bool global_counts, bool locked, QStats* st,
                             uint64_t* active, CutLds& CL, const DeferList* D = nullptr) {
    uint32_t* s_flags = CL.flags;
    uint32_t* s_live = &CL.live;
    const int tid = threadIdx.x;
    // arcs of Gamma_d that the footnote bound leaves out of ~gamma_{d+1}: one
    // edge per node back to Gamma_{d-1} (still scanned, so still in m_vis)
    uint64_t back = 0;
    if (tid < W) {
        SrcState s = S[tid];
        uint32_t fl = 0;
        if (s.status == S_LIVE && apply) {
            uint32_t g;
            unsigned long long t;
            if (global_counts) {
                g = __hip_atomic_load(&cg[tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                t = __hip_atomic_load(&ct[tid], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            } else {
                g = cg[tid];
                t = ct[tid];
            }
            if (g == 0) {
                s.status = S_DONE;
                fl = 1;
            } else {
                s.nd += g;
                s.fd += (uint64_t)d * g;
                back = T.footnote ? ((uint64_t)g < t ? (uint64_t)g : t) : 0;
                s.tg = t - back;
            }
        } else if (s.status == S_TRIVIAL && !apply) {
            fl = 1;
        }
        S[tid] = s;
        s_flags[tid] = fl;
    }
    if (tid == 0) *s_live = 0;
    const int any = __syncthreads_or(tid < W ? (int)s_flags[tid] : 0);
    if (tid == 0) {
        uint32_t nd = 0, nt = 0;
        unsigned long long mv = 0;
        if (any && T.all_f) {
            for (int j = 0; j < W; ++j) {
                if (!s_flags[j]) continue;
                const SrcState& s = S[j];
                const bool triv = s.status == S_TRIVIAL;
                T.all_f[s.oid] = triv ? 0 : s.fd;
                T.all_r[s.oid] = triv ? 1u : (uint32_t)s.nd;
                if (triv) ++nt;
                else {
                    ++nd;
                    mv += s.mvis;
                }
            }
            if (nd) atomicAdd(&st->n_done, (unsigned long long)nd);
            if (nt) atomicAdd(&st->n_trivial, (unsigned long long)nt);
            if (mv) atomicAdd(&st->m_vis, mv);
        } else if (any) {
            // A completed source whose key is not above a published k-th
            // record can never enter (the k-th best value only grows): drop
            // it without the lock, so that the lock is taken only by sources
            // that may enter (most completions, e.g. trivial sources, never do).
            ThRec th0;
            const bool have0 = load_threshold(T, &th0);
            bool need = false;
            for (int j = 0; j < W; ++j) {
                if (!s_flags[j]) continue;
                const SrcState& s = S[j];
                const bool triv = s.status == S_TRIVIAL;
                const uint64_t r = triv ? 1 : s.nd;
                const uint64_t A = r <= 1 ? 0 : (r - 1) * (r - 1);
                const uint64_t F = r <= 1 ? 1 : s.fd;
                if (triv) ++nt;
                else {
                    ++nd;
                    mv += s.mvis;
                }
                if (have0 && !key_gt(A, F, s.oid, th0.A, th0.F, (int32_t)th0.id)) s_flags[j] = 0;
                else need = true;
            }
            if (need) {
                if (locked) lock_acquire(T.lock);
                for (int j = 0; j < W; ++j) {
                    if (!s_flags[j]) continue;
                    const SrcState& s = S[j];
                    if (s.status == S_TRIVIAL) {
                        topk_insert(T, 0, 1, 0, s.oid, 1);
                    } else {
                        const uint64_t r = s.nd;
                        const uint64_t A = r <= 1 ? 0 : (r - 1) * (r - 1);
                        const uint64_t F = r <= 1 ? 1 : s.fd;
                        topk_insert(T, A, F, s.fd, s.oid, (uint32_t)r);
                    }
                }
                if (locked) lock_release(T.lock);
            }
            if (nd) atomicAdd(&st->n_done, (unsigned long long)nd);
            if (nt) atomicAdd(&st->n_trivial, (unsigned long long)nt);
            if (mv) atomicAdd(&st->m_vis, mv);
        }
        ThRec th;
        CL.have_th = load_threshold(T, &th) ? 1u : 0u;
        CL.th = th;
    }
    __syncthreads();
    const bool have_th = CL.have_th != 0;
    bool live = false;
    if (tid < W) {
        SrcState s = S[tid];
        if (s.status == S_LIVE) {
            if (have_th && cut_rule(s, d, CL.th)) {
                s.status = S_CUT;
                atomicAdd(&st->n_cut, 1ull);
                if (s.mvis) atomicAdd(&st->m_vis, (unsigned long long)s.mvis);
            } else if (D && D->budget && s.tg + back > D->budget) {
                // too deep for one workgroup: restart it on the whole GPU later
                s.status = S_DEFER;
                D->ids[atomicAdd(D->cnt, 1u)] = s.id;
                atomicAdd(&st->n_deferred, 1ull);
                if (s.mvis) atomicAdd(&st->m_vis, (unsigned long long)s.mvis);
            } else {
                s.mvis += s.tg + back;  // this source scans the out-arcs of Gamma_d
                live = true;
            }
            S[tid] = s;
        }
    }
    const unsigned long long bal = __ballot(live);
    if (tid < W && lane_id() == 0) {
        active[tid / 64] = bal;
        if (bal) atomicAdd(s_live, (uint32_t)__popcll(bal));
    }
    __syncthreads();
    const uint32_t nlive = *s_live;
    __syncthreads();
    return nlive;
}

// Bound test of the level just reached (d) with over-counted sizes, before
// the exact count: g(b) and t(b) count every arc from the frontier of source
// b to a node b has not seen (and that node's degree), so g >= gamma_d(b)
// and t >= ~gamma_{d+1}(b), with equality when no node is reached twice.
// Each extra count lowers L_x = f_d - ~gamma_{d+1} + (d+2)(x - n_d) by 2 plus
// the node's degree (by 1 plus the degree with the footnote bound), so L_x
// from these counts is at most the exact one and still bounds f from below
// (Lemma 1, Lemma 2): a source it cuts would be cut by the exact test too.
// Retires such sources (same bookkeeping as cut_step); every other source
// keeps its exact state and is counted exactly afterwards.  A source with
// g = 0 reached nothing new, which the exact count confirms (it completes
// there).  Writes the active masks and returns the live count.
__device__ uint32_t trial_cut(const TopKDev& T, SrcState* S, int W, uint32_t d, const uint32_t* cg,
                              const unsigned long long* ct, QStats* st, uint64_t* active, CutLds& CL) {
    const int tid = threadIdx.x;
    if (tid == 0) {
        ThRec th;
        CL.have_th = load_threshold(T, &th) ? 1u : 0u;
        CL.th = th;
        CL.live = 0;
    }
    __syncthreads();
    bool live = false;
    if (tid < W) {
        SrcState s = S[tid];
        if (s.status == S_LIVE) {
            live = true;
            const uint32_t g = cg[tid];
            if (CL.have_th && g > 0) {
                const unsigned long long t = ct[tid];
                SrcState q = s;
                q.nd += g;
                q.fd += (uint64_t)d * g;
                q.tg = t - (T.footnote ? ((uint64_t)g < t ? (uint64_t)g : t) : 0);
                if (cut_rule(q, d, CL.th)) {
                    s.status = S_CUT;
                    atomicAdd(&st->n_cut, 1ull);
                    if (s.mvis) atomicAdd(&st->m_vis, (unsigned long long)s.mvis);
                    S[tid] = s;
                    live = false;
                }
            }
        }
    }
    const unsigned long long bal = __ballot(live);
    if (tid < W && lane_id() == 0) {
        active[tid / 64] = bal;
        if (bal) atomicAdd(&CL.live, (uint32_t)__popcll(bal));
    }
    __syncthreads();
    const uint32_t nlive = CL.live;
    __syncthreads();
    return nlive;
}

// Initialise the W sources of batch b: the frontier list F and the reset
// list hold the sources themselves, each with its one-hot mask.
template <int WW>
__device__ void init_batch(const DevGraph& G, const int32_t* order, int32_t n, uint32_t b, int W, const SlotPtrs& P,
                           SrcState* S, uint32_t* flen_lds, unsigned long long* arcs_lds) {
    using Lo = Layout<WW>;
    const int tid = threadIdx.x;
    if (tid == 0) {
        *flen_lds = 0;
        *arcs_lds = 0;
    }
    __syncthreads();
    if (tid < W) {
        const int64_t i = (int64_t)b * W + tid;
        SrcState s;
        s.nd = 1;
        s.fd = 0;
        s.mvis = 0;
        if (i < n) {
            const int32_t v = order[i];
            s.id = v;
            s.oid = G.orig ? G.orig[v] : v;
            s.x0 = G.x0[v];
            s.x1 = G.x1[v];
            s.tg = G.deg[v];
            s.status = s.x0 <= 1 ? S_TRIVIAL : S_LIVE;
            if (s.status == S_LIVE) {
                const uint64_t bit = 1ull << (tid & 63);
                uint64_t* rec = &P.ns[(size_t)v * Lo::SW];
#pragma unroll
                for (int j = 0; j < WW; ++j) {
                    const uint64_t x = (j == (tid >> 6)) ? bit : 0ull;
                    rec[j] = x;
                    rec[Lo::CUR + j] = x;
                }
                const uint32_t pos = atomicAdd(flen_lds, 1u);
                P.qa[pos] = v;
                P.clr[pos] = v;
                atomicAdd(arcs_lds, (unsigned long long)s.tg);
            }
        } else {
            s.id = -1;
            s.oid = -1;
            s.x0 = s.x1 = 0;
            s.tg = 0;
            s.status = S_EMPTY;
        }
        S[tid] = s;
    }
    __syncthreads();
}

// Write the out-degree into the meta word of every node record of `slots`
// consecutive slots (the rest of a record is zero at rest).
template <int WW>
__global__ void k_slot_init(const uint32_t* __restrict__ deg, int32_t n, uint64_t* ns, int slots) {
    using Lo = Layout<WW>;
    const size_t total = (size_t)n * slots;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += (size_t)gridDim.x * blockDim.x)
        ns[i * Lo::SW + Lo::META] = (uint64_t)deg[i % (size_t)n] << 32;
}

// ------------------------------------------------------- plain kernels
//
// One batch at a time; per level the host launches
//   expand (or pull; its last workgroup runs the cut step) -> clearcur -> build
// and reads the control block to see whether any source is still live.

template <int WW>
__device__ void plain_init_body(const DevGraph& G, const int32_t* order, int32_t count, uint32_t b, int W,
                                const SlotPtrs& P, SrcState* S, Ctl* C, const TopKDev& T, QStats* st, CutLds& CL,
                                uint32_t& s_flen, unsigned long long& s_arcs, uint64_t* s_act) {
    init_batch<WW>(G, order, count, b, W, P, S, &s_flen, &s_arcs);
    const uint32_t live = cut_step<WW>(T, S, W, 0, false, nullptr, nullptr, false, false, st, s_act, CL);
    if (threadIdx.x == 0) {
        C->stamp = C->stamp + 1;
        C->d = 0;
        C->flen = s_flen;
        C->nlen = 0;
        C->clen = s_flen;
        C->live = live;
        C->pull = 0;
        C->chunk = 0;
        C->done_blocks = 0;
        C->front_arcs = s_arcs;
        C->acc_arcs = 0;
        for (int j = 0; j < 4; ++j) C->active[j] = j < WW ? s_act[j] : 0;
        atomicAdd(&st->batches, 1ull);
    }
}

template <int WW>
__global__ __launch_bounds__(kBlk) void k_plain_init(DevGraph G, const int32_t* order, int32_t count, uint32_t b,
                                                    int W, SlotPtrs P, SrcState* S, Ctl* C, TopKDev T, QStats* st) {
    __shared__ CutLds CL;
    __shared__ uint32_t s_flen;
    __shared__ unsigned long long s_arcs;
    __shared__ uint64_t s_act[4];
    plain_init_body<WW>(G, order, count, b, W, P, S, C, T, st, CL, s_flen, s_arcs, s_act);
}

// Shared epilogue of the plain expand/pull kernels: flush the workgroup's bit
// counters; the last workgroup to finish runs the cut step for the level.
template <int WW>
__device__ void plain_level_epilogue(Ctl* C, SrcState* S, TopKDev T, QStats* st, int W, const uint32_t* cg,
                                     const unsigned long long* ct, CutLds& CL, uint64_t* s_act, uint32_t* s_last) {
    const int tid = threadIdx.x;
    if (tid < W && cg[tid]) {
        atomicAdd(&C->cnt_g[tid], cg[tid]);
        atomicAdd(&C->cnt_t[tid], ct[tid]);
    }
    __threadfence();
    __syncthreads();
    if (tid == 0) *s_last = (atomicAdd(&C->done_blocks, 1u) == gridDim.x - 1) ? 1u : 0u;
    __syncthreads();
    if (!*s_last) return;
    __threadfence();
    const uint32_t d = C->d;
    const uint32_t live = cut_step<WW>(T, S, W, d + 1, true, C->cnt_g, C->cnt_t, true, false, st, s_act, CL);
    if (tid < W) {
        C->cnt_g[tid] = 0;
        C->cnt_t[tid] = 0;
    }
    if (tid == 0) {
        if (C->pull) atomicAdd(&st->pull_levels, 1ull);
        C->d = d + 1;
        C->live = live;
        C->ran = 1;
        C->chunk = 0;
        for (int j = 0; j < 4; ++j) C->active[j] = j < WW ? s_act[j] : 0;
        atomicAdd(&st->levels, 1ull);
        atomicAdd(&st->discovered, (unsigned long long)C->nlen);
        __threadfence();
        C->done_blocks = 0;
    }
}

// gated: a step of a captured level sequence, which runs only while a
// source is live and the step's direction is push (the pull kernel of the
// same step takes the other case).  Every thread reads the same control
// words, written by kernels that finished before this one started.
// Frontier entries per chunk a workgroup claims in a push step: about
// kChunkArcs arcs (the level's arcs spread evenly over its entries), at most
// kBlk.  A level of a few heavy entries, such as the hub sources of level 0
// in degree order, then spreads over many workgroups instead of one.
constexpr unsigned long long kChunkArcs = 4096;
__host__ __device__ inline uint32_t expand_chunk(uint32_t flen, unsigned long long arcs) {
    if (arcs == 0) return kBlk;
    const unsigned long long per = (unsigned long long)flen * kChunkArcs / arcs;
    return per < 1 ? 1u : (per > (unsigned long long)kBlk ? (uint32_t)kBlk : (uint32_t)per);
}

template <int WW>
__device__ void plain_expand_body(const DevGraph& G, const SlotPtrs& P, Ctl* C, QStats* st, LdsExpand<WW>& L,
                                  uint64_t* s_act, unsigned long long& s_arcs, unsigned long long& s_ent,
                                  uint32_t* bsh) {
    const uint32_t flen = C->flen, stamp = C->stamp;
    const uint32_t per = expand_chunk(flen, C->front_arcs);
    const int tid = threadIdx.x;
    if (tid < WW) s_act[tid] = C->active[tid];
    if (tid == 0) {
        s_arcs = 0;
        s_ent = 0;
    }
    __syncthreads();
    for (;;) {
        if (tid == 0) L.chunk = atomicAdd(&C->chunk, 1u);
        __syncthreads();
        const unsigned long long e0 = (unsigned long long)L.chunk * per;
        __syncthreads();
        if (e0 >= flen) break;
        expand_entries<WW, kBlk, 2, true>(G, P, P.qa, (uint32_t)e0, min(flen, (uint32_t)e0 + per), s_act, P.qb,
                                          &C->nlen, stamp, L, &s_arcs, &s_ent, bsh);
    }
    if (tid == 0 && s_arcs) atomicAdd(&st->node_arcs, s_arcs);
    if (tid == 0 && s_ent) atomicAdd(&st->frontier_entries, s_ent);
}

template <int WW>
__global__ __launch_bounds__(kBlk) void k_plain_expand(DevGraph G, SlotPtrs P, Ctl* C, QStats* st, int gated) {
    if (gated && (C->live == 0 || C->pull != 0)) return;
    __shared__ LdsExpand<WW> L;
    __shared__ uint64_t s_act[4];
    __shared__ unsigned long long s_arcs, s_ent;
    __shared__ uint32_t bsh[kBlk / 64 + 1];
    plain_expand_body<WW>(G, P, C, st, L, s_act, s_arcs, s_ent, bsh);
}

// After a push step: the per-source counters of the level from its list of
// newly reached nodes (once per node), then the cut step in the last
// workgroup.  Same gate as the push step.
template <int WW>
__device__ void plain_count_body(const SlotPtrs& P, SrcState* S, Ctl* C, const TopKDev& T, QStats* st, int W,
                                 uint32_t* cg, unsigned long long* ct, CutLds& CL, uint32_t& s_last,
                                 uint64_t* s_act) {
    using Lo = Layout<WW>;
    const uint32_t tid = threadIdx.x;
    cg[tid] = 0;
    ct[tid] = 0;
    __syncthreads();
    const uint32_t len = C->nlen;
    const uint32_t stride = gridDim.x * kBlk;
    for (uint32_t base = blockIdx.x * kBlk; base < len; base += stride) {
        if (base + (tid & ~63u) >= len) break;  // wave-uniform: nothing left for this wave
        const uint32_t i = base + tid;
        uint64_t nb[WW];
        uint32_t deg = 0;
#pragma unroll
        for (int j = 0; j < WW; ++j) nb[j] = 0;
        if (i < len) {
            const uint64_t* rec = &P.ns[(size_t)P.qb[i] * Lo::SW];
#pragma unroll
            for (int j = 0; j < WW; ++j) nb[j] = rec[Lo::NXT + j];
            deg = (uint32_t)(rec[Lo::META] >> 32);
        }
        wave_count_nodes<WW>(nb, deg, cg, ct);
    }
    __syncthreads();
    plain_level_epilogue<WW>(C, S, T, st, W, cg, ct, CL, s_act, &s_last);
}

template <int WW>
__global__ __launch_bounds__(kBlk) void k_plain_count(SlotPtrs P, SrcState* S, Ctl* C, TopKDev T, QStats* st,
                                                     int W, int gated) {
    if (gated && (C->live == 0 || C->pull != 0)) return;
    __shared__ uint32_t cg[kBlk];
    __shared__ unsigned long long ct[kBlk];
    __shared__ CutLds CL;
    __shared__ uint32_t s_last;
    __shared__ uint64_t s_act[4];
    plain_count_body<WW>(P, S, C, T, st, W, cg, ct, CL, s_last, s_act);
}

// Bottom-up step: every node not yet seen by some live source looks for an
// in-neighbour in the frontier of that source (early exit once all of its
// unseen live bits are found).  One thread owns a node, so all bits it finds
// are new and counted here.  A node with more than kPullWave in-arcs is
// scanned by its whole wave, 64 arcs a round, the bits found OR-reduced over
// the wave (on skewed graphs one thread walking a hub's list serially held
// its wave, and the level, for the whole walk).
constexpr int32_t kPullWave = 32;

// OR of x over the 64 lanes of the wave, in every lane.
__device__ inline uint64_t wave_or(uint64_t x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x |= __shfl_xor(x, o);
    return x;
}

template <int WW>
__device__ void plain_pull_body(const DevGraph& G, const SlotPtrs& P, SrcState* S, Ctl* C, const TopKDev& T,
                                QStats* st, int W, uint32_t* cg, unsigned long long* ct, CutLds& CL,
                                uint32_t& s_last, uint64_t* s_act, uint32_t* bsh) {
    using Lo = Layout<WW>;
    const int tid = threadIdx.x;
    const int lane = (int)lane_id();
    uint64_t act[WW];
#pragma unroll
    for (int j = 0; j < WW; ++j) act[j] = C->active[j];
    cg[tid] = 0;
    ct[tid] = 0;
    __syncthreads();
    unsigned long long scanned = 0;
    const uint32_t stride = gridDim.x * kBlk;
    for (uint32_t base = blockIdx.x * kBlk; base < (uint32_t)G.n; base += stride) {
        const int32_t w = (int32_t)(base + tid);
        bool app = false;
        uint64_t pbits[WW], unv[WW], acc[WW];
        uint32_t pdeg = 0;
        uint64_t any = 0;
        int32_t e0 = 0, e1 = 0;
#pragma unroll
        for (int j = 0; j < WW; ++j) {
            pbits[j] = 0;
            unv[j] = 0;
            acc[j] = 0;
        }
        uint64_t* rec = nullptr;
        if (w < G.n) {
            rec = &P.ns[(size_t)w * Lo::SW];
#pragma unroll
            for (int j = 0; j < WW; ++j) {
                unv[j] = act[j] & ~rec[j];
                any |= unv[j];
            }
            if (any) {
                e0 = G.irp[w];
                e1 = G.irp[w + 1];
            }
        }
        const bool heavy = any && e1 - e0 > kPullWave;
        if (any && !heavy) {
            for (int32_t e = e0; e < e1; ++e) {
                const uint64_t* ur = &P.ns[(size_t)G.icol[e] * Lo::SW];
                ++scanned;
                bool full = true;
#pragma unroll
                for (int j = 0; j < WW; ++j) {
                    acc[j] |= ur[Lo::CUR + j] & unv[j];
                    full = full && (acc[j] == unv[j]);
                }
                if (full) break;
            }
        }
        // the wave's heavy nodes, one at a time, each list read by all lanes
        unsigned long long hm = __ballot(heavy);
        while (hm) {
            const int l = __ffsll((long long)hm) - 1;
            hm &= hm - 1;
            const int32_t h0 = __shfl(e0, l), h1 = __shfl(e1, l);
            uint64_t hu[WW], ha[WW];
#pragma unroll
            for (int j = 0; j < WW; ++j) {
                hu[j] = __shfl(unv[j], l);
                ha[j] = 0;
            }
            for (int32_t eb = h0; eb < h1; eb += 64) {
                const int32_t e = eb + lane;
                uint64_t part[WW];
#pragma unroll
                for (int j = 0; j < WW; ++j) part[j] = 0;
                if (e < h1) {
                    const uint64_t* ur = &P.ns[(size_t)G.icol[e] * Lo::SW];
#pragma unroll
                    for (int j = 0; j < WW; ++j) part[j] = ur[Lo::CUR + j] & hu[j];
                }
                if (lane == 0) scanned += (unsigned long long)min(64, h1 - eb);
                bool full = true;
#pragma unroll
                for (int j = 0; j < WW; ++j) {
                    ha[j] |= wave_or(part[j]);
                    full = full && (ha[j] == hu[j]);
                }
                if (full) break;
            }
            if (lane == l) {
#pragma unroll
                for (int j = 0; j < WW; ++j) acc[j] = ha[j];
            }
        }
        if (any) {
            uint64_t got = 0;
#pragma unroll
            for (int j = 0; j < WW; ++j) got |= acc[j];
            if (got) {
                pdeg = (uint32_t)(rec[Lo::META] >> 32);
#pragma unroll
                for (int j = 0; j < WW; ++j) {
                    rec[Lo::NXT + j] = acc[j];
                    pbits[j] = acc[j];
                }
                app = true;
            }
        }
        wave_count_nodes<WW>(pbits, pdeg, cg, ct);
        block_append<kBlk, 1>(&app, &w, P.qb, &C->nlen, bsh);
    }
    if (scanned) atomicAdd(&st->node_arcs, scanned);
    __syncthreads();
    plain_level_epilogue<WW>(C, S, T, st, W, cg, ct, CL, s_act, &s_last);
}

template <int WW>
__global__ __launch_bounds__(kBlk) void k_plain_pull(DevGraph G, SlotPtrs P, SrcState* S, Ctl* C, TopKDev T,
                                                    QStats* st, int W, int gated) {
    if (gated && (C->live == 0 || C->pull == 0)) return;
    __shared__ uint32_t cg[kBlk];
    __shared__ unsigned long long ct[kBlk];
    __shared__ CutLds CL;
    __shared__ uint32_t s_last;
    __shared__ uint64_t s_act[4];
    __shared__ uint32_t bsh[kBlk / 64 + 1];
    plain_pull_body<WW>(G, P, S, C, T, st, W, cg, ct, CL, s_last, s_act, bsh);
}

template <int WW>
__global__ __launch_bounds__(kBlk) void k_plain_clearcur(SlotPtrs P, Ctl* C, int gated) {
    if (gated && C->ran == 0) return;
    clear_cur<WW>(P, P.qa, C->flen, blockIdx.x * kBlk, gridDim.x * kBlk);
}

// Materialise the level (or only reset nxt when nothing is live); the last
// workgroup closes the level: frontier length, next direction.  The chunk
// counter is idle between levels and counts finished workgroups here; the
// done_blocks word counts the new frontier entries.
template <int WW>
__device__ void plain_build_body(const DevGraph& G, const SlotPtrs& P, Ctl* C, const LevelParams& lp,
                                 uint32_t& s_last, unsigned long long& s_arcs, uint32_t* bsh) {
    const int tid = threadIdx.x;
    uint64_t act[WW];
#pragma unroll
    for (int j = 0; j < WW; ++j) act[j] = C->active[j];
    const bool any_live = C->live != 0;
    const uint32_t nlen = C->nlen;
    if (tid == 0) s_arcs = 0;
    __syncthreads();
    build_level<WW, true>(P, P.qb, nlen, blockIdx.x * kBlk, gridDim.x * kBlk, act, any_live, P.qa, &C->done_blocks,
                          &C->clen, &s_arcs, nullptr, bsh);
    __syncthreads();
    if (tid == 0 && s_arcs) atomicAdd(&C->acc_arcs, s_arcs);
    __threadfence();
    __syncthreads();
    if (tid == 0) s_last = (atomicAdd(&C->chunk, 1u) == gridDim.x - 1) ? 1u : 0u;
    __syncthreads();
    if (!s_last || tid != 0) return;
    __threadfence();
    const uint32_t flen =
        any_live ? __hip_atomic_load(&C->done_blocks, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : 0;
    const unsigned long long fa = __hip_atomic_load(&C->acc_arcs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    uint32_t pull = C->pull;
    if (lp.can_pull) {
        if (!pull && lp.pull_alpha > 0.f && (double)fa > (double)G.m / lp.pull_alpha) pull = 1;
        else if (pull && (double)flen < (double)G.n / lp.pull_beta) pull = 0;
    }
    C->pull = pull;
    C->flen = flen;
    C->nlen = 0;
    C->front_arcs = fa;
    C->acc_arcs = 0;
    C->stamp = C->stamp + 1;
    C->chunk = 0;
    C->ran = 0;
    __threadfence();
    C->done_blocks = 0;
}

template <int WW>
__global__ __launch_bounds__(kBlk) void k_plain_build(DevGraph G, SlotPtrs P, Ctl* C, LevelParams lp, int gated) {
    if (gated && C->ran == 0) return;
    __shared__ uint32_t s_last;
    __shared__ unsigned long long s_arcs;
    __shared__ uint32_t bsh[kBlk / 64 + 1];
    plain_build_body<WW>(G, P, C, lp, s_last, s_arcs, bsh);
}

// End of a batch: reset seen and cur of every node the batch reached (nxt
// is already zero; cur is non-zero only for sources of a batch that ended
// at level 0).
template <int WW>
__device__ void plain_clear_body(const SlotPtrs& P, Ctl* C) {
    using Lo = Layout<WW>;
    const uint32_t nc = C->clen;
    for (uint32_t i = blockIdx.x * kBlk + threadIdx.x; i < nc; i += gridDim.x * kBlk) {
        uint64_t* rec = &P.ns[(size_t)P.clr[i] * Lo::SW];
#pragma unroll
        for (int j = 0; j < WW; ++j) {
            rec[j] = 0;
            rec[Lo::CUR + j] = 0;
        }
    }
}

template <int WW>
__global__ __launch_bounds__(kBlk) void k_plain_clear(SlotPtrs P, Ctl* C) {
    plain_clear_body<WW>(P, C);
}

// Every level of `nb` consecutive batches in one cooperative launch: the
// phases the host otherwise launches one by one per level are separated by
// grid barriers, and the decision to go on is read on the device.  Each
// branch after a barrier reads only control words that no phase changes
// before the next barrier (live, pull and the list lengths at the top of a
// level, nlen after the counting phase), so every workgroup takes the same
// branch and reaches the same barriers.  A list longer than n (which would
// mean the level step wrote out of order) stops the loop with C->err set,
// before any kernel indexes the lists with that length.
__device__ inline void grid_barrier(cooperative_groups::grid_group& g) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    g.sync();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

template <int WW>
__global__ __launch_bounds__(kBlk) void k_plain_coop(DevGraph G, const int32_t* order, int32_t count, uint32_t b0,
                                                    uint32_t nb, int W, SlotPtrs P, SrcState* S, Ctl* C, TopKDev T,
                                                    QStats* st, LevelParams lp) {
    cooperative_groups::grid_group grid = cooperative_groups::this_grid();
    __shared__ LdsExpand<WW> L;
    __shared__ uint32_t cg[kBlk];
    __shared__ unsigned long long ct[kBlk];
    __shared__ CutLds CL;
    __shared__ uint32_t s_last, s_flen;
    __shared__ unsigned long long s_arcs, s_ent;
    __shared__ uint64_t s_act[4];
    __shared__ uint32_t bsh[kBlk / 64 + 1];
    const uint32_t n = (uint32_t)G.n;
    for (uint32_t b = b0; b < b0 + nb; ++b) {
        if (blockIdx.x == 0) plain_init_body<WW>(G, order, count, b, W, P, S, C, T, st, CL, s_flen, s_arcs, s_act);
        grid_barrier(grid);
        bool bad = false;
        for (;;) {
            const uint32_t live = ldu32(&C->live), pull = ldu32(&C->pull);
            if (ldu32(&C->flen) > n || ldu32(&C->clen) > n) {
                bad = true;
                break;
            }
            if (!live) break;
            if (pull) {
                plain_pull_body<WW>(G, P, S, C, T, st, W, cg, ct, CL, s_last, s_act, bsh);
                grid_barrier(grid);
            } else {
                plain_expand_body<WW>(G, P, C, st, L, s_act, s_arcs, s_ent, bsh);
                grid_barrier(grid);
                if (ldu32(&C->nlen) > n) {
                    bad = true;
                    break;
                }
                plain_count_body<WW>(P, S, C, T, st, W, cg, ct, CL, s_last, s_act);
                grid_barrier(grid);
            }
            if (ldu32(&C->nlen) > n) {
                bad = true;
                break;
            }
            clear_cur<WW>(P, P.qa, ldu32(&C->flen), blockIdx.x * kBlk, gridDim.x * kBlk);
            grid_barrier(grid);
            plain_build_body<WW>(G, P, C, lp, s_last, s_arcs, bsh);
            grid_barrier(grid);
        }
        if (bad) {
            if (blockIdx.x == 0 && threadIdx.x == 0) __hip_atomic_store(&C->err, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            return;  // every workgroup read the same lengths, so all of them end here
        }
        plain_clear_body<WW>(P, C);
        grid_barrier(grid);
    }
}

// ------------------------------------------------------ batched kernel

// Shared memory of the record-based persistent kernels (one slot per
// workgroup, every level of a batch inside the workgroup).
template <int WW, int B>
struct RecLds {
    LdsExpand<WW, B> LE;
    SrcState S[kBlk];
    uint32_t cg[kBlk];
    unsigned long long ct[kBlk];
    CutLds CL;
    uint32_t flen, nlen, clen;
    uint64_t act[4];
    unsigned long long arcs, narcs, ent;  // narcs, ent: arcs and frontier entries expanded
};

// Per-workgroup counters of a record-based persistent kernel.
struct RecCounters {
    unsigned long long levels = 0, batches = 0, disc = 0;
    unsigned long long ticks[5] = {0, 0, 0, 0, 0};  // set-up, expand, cut, build, reset (100 MHz)
};

// One whole batch b (sources order[b W .. b W + W)) of graph G on the node
// records of slot P: level 0, then per level the expansion over the frontier,
// the counters of the level reached, the cut step and the build of the live
// bits, until no source is live; then the marks of every node the batch
// reached are reset, so the slot is all zero again.  degs: out-degrees from
// the graph (records shared by several graphs) or null (from the records'
// meta words).  Block-uniform call.
template <int WW, int B>
__device__ void record_batch(const DevGraph& G, const int32_t* order, int W, uint32_t b, const SlotPtrs& P,
                             const TopKDev& T, QStats* st, const DeferList* D, const uint32_t* degs,
                             RecLds<WW, B>& R, uint32_t& stamp, RecCounters& K) {
    using Lo = Layout<WW>;
    const int tid = threadIdx.x;
    ++K.batches;
    const uint64_t tb = __builtin_amdgcn_s_memrealtime();
    init_batch<WW>(G, order, G.n, b, W, P, R.S, &R.flen, &R.arcs);
    if (tid == 0) R.clen = R.flen;
    uint32_t live = cut_step<WW>(T, R.S, W, 0, false, nullptr, nullptr, false, true, st, R.act, R.CL, D);
    uint32_t flen = R.flen, d = 0;
    uint64_t tp = __builtin_amdgcn_s_memrealtime();
    K.ticks[0] += tp - tb;
    while (live) {
        ++stamp;
        if (tid < kBlk) {
            R.cg[tid] = 0;
            R.ct[tid] = 0;
        }
        if (tid == 0) R.nlen = 0;
        __syncthreads();
        for (uint32_t e0 = 0; e0 < flen; e0 += B)
            expand_entries<WW, B, 1>(G, P, P.qa, e0, min(flen, e0 + B), R.act, P.qb, &R.nlen, stamp, R.LE, &R.narcs,
                                     &R.ent);
        __syncthreads();
        const uint32_t nlen = R.nlen;
        count_level<WW, B>(P, P.qb, nlen, R.cg, R.ct, degs);
        __syncthreads();
        K.disc += nlen;
        uint64_t tq = __builtin_amdgcn_s_memrealtime();
        K.ticks[1] += tq - tp;
        tp = tq;
        ++d;
        ++K.levels;
        live = cut_step<WW>(T, R.S, W, d, true, R.cg, R.ct, false, true, st, R.act, R.CL, D);
        tq = __builtin_amdgcn_s_memrealtime();
        K.ticks[2] += tq - tp;
        tp = tq;
        clear_cur<WW>(P, P.qa, flen, 0, B);
        if (tid == 0) R.flen = 0;
        __syncthreads();
        build_level<WW>(P, P.qb, nlen, 0, B, R.act, live != 0, P.qa, &R.flen, &R.clen, &R.arcs);
        __syncthreads();
        flen = R.flen;
        tq = __builtin_amdgcn_s_memrealtime();
        K.ticks[3] += tq - tp;
        tp = tq;
    }
    // reset seen and cur of every node this batch reached
    const uint32_t nc = R.clen;
    for (uint32_t i = tid; i < nc; i += B) {
        uint64_t* rec = &P.ns[(size_t)P.clr[i] * Lo::SW];
#pragma unroll
        for (int j = 0; j < WW; ++j) {
            rec[j] = 0;
            rec[Lo::CUR + j] = 0;
        }
    }
    __syncthreads();
    K.ticks[4] += __builtin_amdgcn_s_memrealtime() - tp;
}

// Persistent: every workgroup owns one slot and runs whole batches, pulling
// batch indices from a device counter, with every level inside the workgroup.
// B threads per workgroup (kBatchBlk): a level's arcs are spread over all of
// them, so a CU keeps B / 64 waves of node-record loads and atomics in flight.
template <int WW, int B>
__global__ __launch_bounds__(B) void k_batched(DevGraph G, const int32_t* order, int W, uint32_t nbatches,
                                                 uint32_t* next_batch, uint32_t chunk, SlotPtrs base,
                                                 uint32_t* slot_stamp, TopKDev T, QStats* st, DeferList D) {
    using Lo = Layout<WW>;
    __shared__ RecLds<WW, B> R;
    __shared__ uint32_t s_b, s_next, s_end;
    const int tid = threadIdx.x;
    const size_t slot = blockIdx.x;
    SlotPtrs P;
    P.ns = base.ns + slot * (size_t)G.n * Lo::SW;
    P.qa = base.qa + slot * (size_t)G.n;
    P.qb = base.qb + slot * (size_t)G.n;
    P.clr = base.clr + slot * (size_t)G.n;
    // first-touch stamps keep growing across queries (stamps are never cleared)
    uint32_t stamp = slot_stamp[slot];
    RecCounters K;
    if (tid == 0) {
        R.narcs = 0;
        R.ent = 0;
        s_next = s_end = 0;
    }
    for (;;) {
        // claim `chunk` consecutive batches at a time: neighbouring batches of
        // the grouped order share neighbourhoods, whose records then stay cached
        if (tid == 0) {
            if (s_next >= s_end) {
                s_next = atomicAdd(next_batch, chunk);
                s_end = s_next + chunk;
            }
            s_b = s_next++;
        }
        __syncthreads();
        const uint32_t b = s_b;
        __syncthreads();
        if (b >= nbatches) break;
        record_batch<WW, B>(G, order, W, b, P, T, st, &D, nullptr, R, stamp, K);
    }
    if (tid == 0) {
        atomicAdd(&st->levels, K.levels);
        atomicAdd(&st->batches, K.batches);
        atomicAdd(&st->discovered, K.disc);
        if (R.narcs) atomicAdd(&st->node_arcs, R.narcs);
        if (R.ent) atomicAdd(&st->frontier_entries, R.ent);
        for (int i = 0; i < 5; ++i) atomicAdd(&st->phase_ticks[i], K.ticks[i]);
        slot_stamp[slot] = stamp;
    }
}

// --------------------------------------------------------- job launches
//
// A job is one top-k query (a graph, its source order, k) of a launch that
// runs the batches of many queries, on graphs of different sizes, in one
// persistent kernel: the parallel loop of Algorithm 1 (Section 2.1) over the
// sources of every query at once.  Each query keeps its own top-k list,
// threshold records and statistics, so it returns what it returns alone.
//
// Every batch of every query has a place in one global batch sequence.  A
// descriptor (JobDesc) covers a contiguous range of it: `count` batches of
// one query, its local batches bofs .. bofs + count.  A query may have two
// ranges (its seed batches early in the sequence, the rest later), which
// share its state.  Workgroups claim global batches one at a time with a
// compare-and-swap that never passes the published total, so every claimed
// batch exists and is run; the total only grows (a serving queue appends
// queries while the kernel runs).  Node records are shared by all queries:
// they are sized for the largest graph and all zero at rest, degrees come
// from each graph's own array.

struct JobDesc {
    DevGraph G;
    const int32_t* order;
    TopKDev T;
    QStats* st;
    // the range of global batches, one word so that a reader that races a
    // rewrite of the slot sees the old range, none, or the new one, never a
    // mix: (count << kRangeStartBits) | (first batch mod 2^kRangeStartBits);
    // 0 = no range.  Written last when a descriptor is published.
    unsigned long long range;
    uint32_t bofs;             // local index of its first batch
    uint32_t total;            // batches of the whole query
    uint32_t seed;             // the query's first `seed` batches: the others wait (bounded) for them
    uint32_t pad_;
    uint32_t* ctr;             // device, 2 words: finished batches, finished seed batches
    Rec* out;                  // host-visible copy of the finished list (k records), or null
    unsigned long long* out_st;  // host-visible copy of the QStats words, or null
    uint32_t* done;            // host-visible: count of results + 1 once the query is finished, or null
    uint32_t* seeded;          // host-visible: 1 once the query's seed batches have finished, or null
    uint32_t* progress;        // host-visible: batches of the query finished so far, or null
};
static_assert(sizeof(JobDesc) % 8 == 0, "descriptors are copied in 8-byte words");
static_assert(offsetof(JobDesc, range) % 8 == 0, "the range is read as one 8-byte word");

// A range's count takes the top 26 bits (a query has at most
// ceil((2^31 - 1) / 64) < 2^26 batches) and its first batch the low 38, modulo
// 2^38: the ranges in a table at one time lie within a few queries of each
// other, far less than 2^38 batches apart, so the difference below is exact.
constexpr int kRangeStartBits = 38;
constexpr unsigned long long kRangeStartMask = (1ull << kRangeStartBits) - 1;
__host__ __device__ inline unsigned long long pack_range(unsigned long long start, uint32_t count) {
    return ((unsigned long long)count << kRangeStartBits) | (start & kRangeStartMask);
}
// Position of global batch c in the range packed in w, or a value >= the
// range's count when c is outside it.
__host__ __device__ inline unsigned long long range_offset(unsigned long long w, unsigned long long c) {
    return (c - (w & kRangeStartMask)) & kRangeStartMask;
}
__host__ __device__ inline uint32_t range_count(unsigned long long w) { return (uint32_t)(w >> kRangeStartBits); }
static_assert(sizeof(QStats) % 8 == 0, "statistics are copied in 8-byte words");

struct JobLaunch {
    const JobDesc* jobs;                  // descriptor table (device or pinned host memory)
    uint32_t njobs;                       // entries of the table scanned for a batch
    uint32_t pad_;
    uint64_t idle_ticks;                  // time with nothing claimable, no batch of the launch running
                                          // and none ended, before a workgroup ends (100 MHz ticks; 0:
                                          // at the first look)
    uint64_t idle_cap;                    // time with nothing claimable after which a workgroup ends
                                          // whatever the others do
    const unsigned long long* published;  // batches published (monotone; device or pinned host memory)
    const uint32_t* stop;                 // nonzero: claim nothing more and end (may be null)
    uint32_t* running;                    // device: batches claimed and not yet ended (may be null: the
                                          // idle rule is then the time alone)
    unsigned long long* last_end;         // device: clock reading when a batch last ended (with running)
    unsigned long long* claim;            // device: next global batch to hand out (kept across launches)
    int W;
    int32_t ncap;                         // nodes per slot (the largest graph)
};

constexpr uint64_t kSeedWaitTicks = 20000000;  // bound of the wait for a query's seed batches: 0.2 s (100 MHz)
constexpr int kQueueCap = 256;             // requests in flight in a serving queue (ring slots)

__device__ inline unsigned long long sys_ld64(const unsigned long long* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ inline void sys_st64(unsigned long long* p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
// The current value of a device word that other workgroups change while this
// one polls it: a read-modify-write that adds nothing is performed where the
// atomics of every compute unit meet, so it never returns a copy that this
// compute unit's caches kept from before (a plain or relaxed load may).
__device__ inline unsigned long long poll64(unsigned long long* p) {
    return __hip_atomic_fetch_add(p, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t poll32(uint32_t* p) {
    return __hip_atomic_fetch_or(p, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Sleep between polls, doubling from about 3.4 us up to about 110 us, so that
// many idle workgroups do not crowd the atomic unit that the busy ones need.
__device__ inline void backoff(uint32_t& reps) {
    for (uint32_t i = 0; i < reps; ++i) __builtin_amdgcn_s_sleep(127);
    if (reps < 32) reps *= 2;
}

// Pointer and size fields of a descriptor read from LDS into scalar
// registers (the same in every lane), so that the level loops address the
// graph as they do when it is a kernel argument.
template <class Ptr>
__device__ inline Ptr uni_ptr(Ptr p) {
    return reinterpret_cast<Ptr>(uni64(reinterpret_cast<uint64_t>(p)));
}
__device__ inline DevGraph uni_graph(const DevGraph& g) {
    DevGraph o;
    o.n = (int32_t)uni32((uint32_t)g.n);
    o.m = (int64_t)uni64((uint64_t)g.m);
    o.directed = (int32_t)uni32((uint32_t)g.directed);
    o.rp = uni_ptr(g.rp);
    o.col = uni_ptr(g.col);
    o.irp = uni_ptr(g.irp);
    o.icol = uni_ptr(g.icol);
    o.deg = uni_ptr(g.deg);
    o.adj = uni_ptr(g.adj);
    o.x0 = uni_ptr(g.x0);
    o.x1 = uni_ptr(g.x1);
    o.orig = uni_ptr(g.orig);
    return o;
}
__device__ inline TopKDev uni_topk(const TopKDev& t) {
    TopKDev o;
    o.k = (int32_t)uni32((uint32_t)t.k);
    o.cnt = uni_ptr(t.cnt);
    o.lock = uni_ptr(t.lock);
    o.seq = uni_ptr(t.seq);
    o.list = uni_ptr(t.list);
    o.ring = uni_ptr(t.ring);
    o.all_f = uni_ptr(t.all_f);
    o.all_r = uni_ptr(t.all_r);
    o.footnote = (int32_t)uni32((uint32_t)t.footnote);
    return o;
}

// A claimed batch has ended (one thread of its workgroup): the clock reading
// first, then the release decrement that an idle workgroup reads with acquire.
__device__ inline void batch_ended(const JobLaunch& L) {
    if (!L.running) return;
    __hip_atomic_fetch_max(L.last_end, (unsigned long long)__builtin_amdgcn_s_memrealtime(), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_fetch_sub(L.running, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}

template <int WW, int B>
__global__ __launch_bounds__(B) void k_jobs(JobLaunch L, SlotPtrs base, uint32_t* slot_stamp) {
    using Lo = Layout<WW>;
    __shared__ RecLds<WW, B> R;
    __shared__ JobDesc J;
    __shared__ unsigned long long s_c;
    __shared__ int32_t s_slot;
    const int tid = threadIdx.x;
    const size_t slot = blockIdx.x;
    SlotPtrs P;
    P.ns = base.ns + slot * (size_t)L.ncap * Lo::SW;
    P.qa = base.qa + slot * (size_t)L.ncap;
    P.qb = base.qb + slot * (size_t)L.ncap;
    P.clr = base.clr + slot * (size_t)L.ncap;
    uint32_t stamp = slot_stamp[slot];
    unsigned long long jstart = ~0ull, jend = 0;  // range of the descriptor held in J
    for (;;) {
        if (tid == 0) {
            // claim the next published batch, or give up after idle_ticks
            // with nothing to claim (or at once when told to stop)
            unsigned long long got = ~0ull;
            const uint64_t t_idle = __builtin_amdgcn_s_memrealtime();
            uint32_t reps = 1;
            unsigned long long c = poll64(L.claim);
            for (;;) {
                // told to stop: claim nothing more (the batches in hand finish)
                if (L.stop && __hip_atomic_load(L.stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) != 0u) break;
                // relaxed: a claimed batch's descriptor is read with system-scope
                // loads, and its data after the acquire fence of a job switch
                const unsigned long long pub = __hip_atomic_load(L.published, __ATOMIC_RELAXED,
                                                                 __HIP_MEMORY_SCOPE_SYSTEM);
                if (c < pub) {
                    // a failed exchange means another workgroup claimed c; it
                    // leaves the counter's current value in c
                    if (__hip_atomic_compare_exchange_strong(L.claim, &c, c + 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT)) {
                        got = c;
                        if (L.running) __hip_atomic_fetch_add(L.running, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        break;
                    }
                    continue;
                }
                // Idle.  While a batch of this launch runs, or ended less than
                // idle_ticks ago, work may still follow from it (the rest of a
                // query is published once its seed batches end), so the
                // workgroup stays; the rule depends on device work alone, never
                // on host progress, which may itself wait for this launch.
                const uint64_t now = __builtin_amdgcn_s_memrealtime();
                const uint64_t idle = now - t_idle;
                if (idle >= L.idle_cap) break;
                if (idle >= L.idle_ticks) {
                    if (!L.running) break;
                    // acquire: an ended batch's clock reading is seen with its decrement
                    const uint32_t run = __hip_atomic_fetch_add(L.running, 0u, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                    if (run == 0u && (int64_t)(now - poll64(L.last_end)) >= (int64_t)L.idle_ticks) break;
                }
                backoff(reps);
                c = poll64(L.claim);
            }
            s_c = got;
            s_slot = -1;
        }
        __syncthreads();
        const unsigned long long c = uni64(s_c);
        if (c == ~0ull) break;
        if (c < jstart || c >= jend) {
            // the descriptor whose range holds c (exactly one: ranges do not
            // overlap, and the range of a claimed batch stays in the table
            // until its query has finished)
            for (uint32_t i = tid; i < L.njobs; i += B) {
                const unsigned long long w = sys_ld64(&L.jobs[i].range);
                if (range_offset(w, c) < range_count(w)) s_slot = (int32_t)i;
            }
            __syncthreads();
            const int32_t js = (int32_t)uni32((uint32_t)s_slot);
            if (js < 0) {  // cannot happen for a published batch; end rather than guess
                if (tid == 0) batch_ended(L);
                break;
            }
            // the slot's other fields were complete before its range was
            // written, and stay as they are until its query has finished,
            // which needs batch c
            const unsigned long long* src = reinterpret_cast<const unsigned long long*>(&L.jobs[js]);
            unsigned long long* dst = reinterpret_cast<unsigned long long*>(&J);
            for (int w = tid; w < (int)(sizeof(JobDesc) / 8); w += B) dst[w] = sys_ld64(&src[w]);
            // the query's graph, order and state were written by other
            // streams, possibly while this launch ran: every wave drops what
            // its caches may hold of them before it reads them
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            __syncthreads();
            const unsigned long long rw = uni64(J.range);
            const unsigned long long off = range_offset(rw, c);
            if (off >= range_count(rw)) {  // cannot happen (see above); end rather than guess
                if (tid == 0) batch_ended(L);
                break;
            }
            jstart = c - off;
            jend = jstart + range_count(rw);
        }
        const uint32_t b = uni32(J.bofs) + (uint32_t)(c - jstart);
        const uint32_t seed = uni32(J.seed), total = uni32(J.total);
        uint32_t* ctr = uni_ptr(J.ctr);
        const TopKDev T = uni_topk(J.T);
        QStats* st = uni_ptr(J.st);
        const DevGraph G = uni_graph(J.G);
        const int32_t* order = uni_ptr(J.order);
        if (b >= seed && tid == 0) {
            // a later batch waits (bounded) for the seed batches of its query,
            // so that it starts with a k-th best record to cut against
            const uint64_t t0 = __builtin_amdgcn_s_memrealtime();
            uint32_t reps = 1;
            while (poll32(T.seq) == 0u && poll32(&ctr[1]) < seed &&
                   __builtin_amdgcn_s_memrealtime() - t0 < kSeedWaitTicks)
                backoff(reps);
        }
        if (tid == 0) {
            R.narcs = 0;
            R.ent = 0;
        }
        __syncthreads();
        RecCounters K;
        record_batch<WW, B>(G, order, L.W, b, P, T, st, nullptr, G.deg, R, stamp, K);
        if (tid == 0) {
            atomicAdd(&st->levels, K.levels);
            atomicAdd(&st->batches, K.batches);
            atomicAdd(&st->discovered, K.disc);
            if (R.narcs) atomicAdd(&st->node_arcs, R.narcs);
            if (R.ent) atomicAdd(&st->frontier_entries, R.ent);
            for (int i = 0; i < 5; ++i) atomicAdd(&st->phase_ticks[i], K.ticks[i]);
            if (b < seed) {
                const uint32_t sd = __hip_atomic_fetch_add(&ctr[1], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
                uint32_t* seeded = uni_ptr(J.seeded);
                // the last seed batch tells the host, which then publishes the rest
                if (sd + 1 == seed && seeded)
                    __hip_atomic_store(seeded, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            const uint32_t f = __hip_atomic_fetch_add(&ctr[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
            uint32_t* prog = uni_ptr(J.progress);
            if (prog) __hip_atomic_fetch_max(prog, f + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
            if (f + 1 == total) {
                // the query's last batch: every other batch's list updates and
                // statistics happen before its increment, which this one read
                const int32_t cnt = ld32(T.cnt);
                Rec* out = uni_ptr(J.out);
                if (out) {
                    for (int32_t i = 0; i < cnt; ++i) {
                        unsigned long long* o = reinterpret_cast<unsigned long long*>(&out[i]);
                        const uint64_t* q = reinterpret_cast<const uint64_t*>(&T.list[i]);
                        for (int w = 0; w < 4; ++w) sys_st64(&o[w], ld64(&q[w]));
                    }
                }
                if (J.out_st) {
                    const uint64_t* q = reinterpret_cast<const uint64_t*>(st);
                    unsigned long long* os = uni_ptr(J.out_st);
                    for (int w = 0; w < (int)(sizeof(QStats) / 8); ++w) sys_st64(&os[w], ld64(&q[w]));
                }
                // the counters are ready for the next query that uses them
                __hip_atomic_store(&ctr[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&ctr[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                uint32_t* done = uni_ptr(J.done);
                if (done) __hip_atomic_store(done, (uint32_t)cnt + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
            }
            batch_ended(L);
        }
        __syncthreads();
    }
    if (tid == 0) slot_stamp[slot] = stamp;
}

// Node-id order 0 .. n-1 (any order gives the same answer, Section 2.1).
__global__ void k_iota(int32_t* a, int32_t n) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) a[i] = i;
}

// Zero `words` 8-byte words (the per-query state of a captured job launch:
// list headers, statistics and counters, so that every replay starts clean;
// a kernel rather than a memset node, which is what the capture records).
__global__ void k_zero_words(unsigned long long* p, size_t words) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ------------------------------------------- LDS-resident batched kernel
//
// For W = 64 most batches end after two levels, and the state of such a
// search is small: the nodes of the levels built so far (a few hundred) and
// the distinct nodes of the level being counted (~10^4).  This kernel keeps
// both in LDS hash tables, so that the only global traffic of a level is the
// adjacency lists it scans:
//   H_seen  node -> seen, cur, next-cur masks of the levels built so far
//   H_next  node -> mask of the level being counted (dedup of arc targets)
// A level whose arc count T exceeds the H_next capacity is counted in P
// passes, pass p taking the targets w with part(w) = p.  After the cut step
// the live bits of the level are built into H_seen by the same passes.  When
// the state would outgrow LDS (P too large, or H_seen too small for the new
// level) the batch moves to the global node records at a level boundary and
// continues with the global level step.

constexpr int kCapN = 8192;       // H_next entries
constexpr int kCapNLog = 13;
constexpr int kCapS = 1024;       // H_seen entries
constexpr int kCapSLog = 10;
constexpr uint32_t kPassCap = 4900;   // arcs per counting pass (H_next load <= 0.6)
constexpr uint32_t kSeenCap = 760;    // H_seen entries allowed after a build (load <= 0.74)
constexpr uint32_t kPassMax = 8;

struct LdsTab {
    int32_t nkey[kCapN];
    uint64_t nmask[kCapN];
    int32_t skey[kCapS];
    uint64_t sseen[kCapS], scur[kCapS], sncur[kCapS];
    int32_t fl[2][kCapS];   // frontier lists: slots of H_seen
    uint32_t nins, sfill, flen2, over;
    unsigned long long tsum;
    // record mode leaves H_seen unused: sseen and scur (contiguous) hold the
    // seen filter there
    __device__ uint32_t* filter() { return reinterpret_cast<uint32_t*>(sseen); }
};
static_assert(offsetof(LdsTab, scur) == offsetof(LdsTab, sseen) + sizeof(uint64_t) * kCapS, "filter layout");
static_assert(2 * sizeof(uint64_t) * kCapS * 8 >= kFiltBits, "filter fits sseen and scur");

__device__ inline uint32_t hmix(int32_t w) { return (uint32_t)w * 2654435761u; }
__device__ inline uint32_t hpart(int32_t w, uint32_t P) { return (((uint32_t)w * 0x85EBCA77u) >> 8) % P; }

__device__ inline int32_t lds_ld(const int32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// seen mask of w (0 when absent); H_seen is read-only while this runs
__device__ inline uint64_t tab_seen(const LdsTab& L, int32_t w) {
    uint32_t i = hmix(w) >> (32 - kCapSLog);
    for (int probe = 0; probe < kCapS; ++probe) {
        const int32_t k = L.skey[i];
        if (k == w) return L.sseen[i];
        if (k < 0) return 0;
        i = (i + 1) & (kCapS - 1);
    }
    return 0;
}

// slot of w in H_seen, inserting it if absent (-1 when full)
__device__ inline int tab_seen_claim(LdsTab& L, int32_t w) {
    uint32_t i = hmix(w) >> (32 - kCapSLog);
    for (int probe = 0; probe < kCapS; ++probe) {
        const int32_t k = lds_ld(&L.skey[i]);
        if (k == w) return (int)i;
        if (k < 0) {
            const int32_t prev = atomicCAS(&L.skey[i], -1, w);
            if (prev < 0) {
                atomicAdd(&L.sfill, 1u);
                return (int)i;
            }
            if (prev == w) return (int)i;
        }
        i = (i + 1) & (kCapS - 1);
    }
    return -1;
}

// slot of w in H_next, inserting it if absent (-1 when full)
__device__ inline int tab_next_claim(LdsTab& L, int32_t w) {
    uint32_t i = hmix(w) >> (32 - kCapNLog);
    for (int probe = 0; probe < kCapN; ++probe) {
        const int32_t k = lds_ld(&L.nkey[i]);
        if (k == w) return (int)i;
        if (k < 0) {
            const int32_t prev = atomicCAS(&L.nkey[i], -1, w);
            if (prev < 0) {
                atomicAdd(&L.nins, 1u);
                return (int)i;
            }
            if (prev == w) return (int)i;
        }
        i = (i + 1) & (kCapN - 1);
    }
    return -1;
}

constexpr int kLdsBlk = 1024;  // one workgroup per CU holds the tables; 16 waves share them

// Scratch of one pass: per frontier entry its first arc position, row start
// and live mask.
struct PassScratch {
    uint32_t eoff[kLdsBlk];
    int32_t ebeg[kLdsBlk];
    uint64_t em[kLdsBlk];
    uint32_t uscan[kLdsBlk / 64 + 1];
};

// Per level: the arcs of the frontier entries of F (slots of H_seen) with
// live bits in act, dealt out over the workgroup by a scan of their
// degrees.  Thread i holds frontier entry i (flen <= kCapS <= B) and writes
// its first arc position eoff, adjacency start ebeg and live bits em; the
// arc total is returned to every thread.  Computed once per level and shared
// by all passes of the level.
__device__ uint32_t tab_prologue(const DevGraph& G, const LdsTab& L, const int32_t* F, uint32_t flen, uint64_t act,
                                 PassScratch& X, unsigned long long* arcs, unsigned long long* entries) {
    constexpr int B = kLdsBlk;
    static_assert(kCapS <= B, "one thread per frontier entry");
    const int tid = threadIdx.x;
    uint32_t deg = 0;
    int32_t beg = 0;
    uint64_t m = 0;
    if ((uint32_t)tid < flen) {
        const int32_t slot = F[tid];
        m = L.scur[slot] & act;
        if (m) {
            const int32_t u = L.skey[slot];
            beg = G.rp[u];
            deg = (uint32_t)(G.rp[u + 1] - beg);
        }
    }
    if (entries) {
        const unsigned long long nlive = __ballot(deg != 0);
        if ((tid & 63) == 0 && nlive) atomicAdd(entries, (unsigned long long)__popcll(nlive));
    }
    uint32_t total;
    const uint32_t off = block_exscan<B>(deg, X.uscan, &total);
    X.eoff[tid] = off;
    X.ebeg[tid] = beg;
    X.em[tid] = m;
    if (arcs && tid == 0) *arcs += total;
    __syncthreads();
    return total;
}

// Record-mode prologue: frontier entries [e0, e1) of the list F on the
// node records (flen may exceed the workgroup), live bits from their cur
// words.  Same outputs as tab_prologue for the chunk.
__device__ uint32_t rec_prologue(const DevGraph& G, const SlotPtrs& P, const int32_t* F, uint32_t e0, uint32_t e1,
                                 uint64_t act, PassScratch& X, unsigned long long* arcs,
                                 unsigned long long* entries) {
    using Lo = Layout<1>;
    constexpr int B = kLdsBlk;
    const int tid = threadIdx.x;
    const uint32_t e = e0 + (uint32_t)tid;
    uint32_t deg = 0;
    int32_t beg = 0;
    uint64_t m = 0;
    if (e < e1) {
        const int32_t u = F[e];
        m = P.ns[(size_t)u * Lo::SW + Lo::CUR] & act;
        if (m) {
            beg = G.rp[u];
            deg = (uint32_t)(G.rp[u + 1] - beg);
        }
    }
    if (entries) {
        const unsigned long long nlive = __ballot(deg != 0);
        if ((tid & 63) == 0 && nlive) atomicAdd(entries, (unsigned long long)__popcll(nlive));
    }
    uint32_t total;
    const uint32_t off = block_exscan<B>(deg, X.uscan, &total);
    X.eoff[tid] = off;
    X.ebeg[tid] = beg;
    X.em[tid] = m;
    if (arcs && tid == 0) *arcs += total;
    __syncthreads();
    return total;
}

// One pass over the arcs [0, total) of a prologue: targets of part p whose
// live bits are not yet seen are ORed into H_next; with counting, the bits
// a thread sets first add to gamma / tgamma (the target's degree comes with
// the target from the packed adjacency).  The seen bits come from H_seen,
// or with kRec from the node records (ns), read without any global atomic.
// Each thread takes arcs tid, tid + B, ... (coalesced), finds the owner of
// each by binary search over the entries' first positions, and issues the
// loads of kInflight arcs before visiting any of them, so that one memory
// latency covers them all.
template <bool kCount, bool kRec>
__device__ void tab_arcs(const DevGraph& G, LdsTab& L, const uint64_t* ns, uint32_t total, uint32_t P, uint32_t p,
                         const PassScratch& X, uint32_t* cg, unsigned long long* ct,
                         const uint32_t* seen_filter = nullptr) {
    constexpr int B = kLdsBlk;
    constexpr int kInflight = 2;
    const uint32_t tid = threadIdx.x;
    for (uint32_t a0 = tid; a0 < total; a0 += kInflight * B) {
        int32_t w[kInflight], dg[kInflight];
        uint64_t m[kInflight], sv[kInflight];
#pragma unroll
        for (int u = 0; u < kInflight; ++u) {
            const uint32_t a = a0 + (uint32_t)u * B;
            m[u] = 0;
            w[u] = 0;
            dg[u] = 0;
            if (a < total) {
                uint32_t lo = 0, hi = B;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (X.eoff[mid] <= a) lo = mid + 1; else hi = mid;
                }
                const uint32_t i = lo - 1;
                const int32_t e = X.ebeg[i] + (int32_t)(a - X.eoff[i]);
                m[u] = X.em[i];
                if (kCount) {
                    const int2 wd = G.adj[e];
                    w[u] = wd.x;
                    dg[u] = wd.y;
                } else {
                    w[u] = G.col[e];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kInflight; ++u) {
            if (P > 1 && m[u] && hpart(w[u], P) != p) m[u] = 0;
            sv[u] = 0;
            if (kRec && m[u] && filter_maybe(seen_filter, w[u])) sv[u] = ns[(size_t)w[u] * Layout<1>::SW];
        }
#pragma unroll
        for (int u = 0; u < kInflight; ++u) {
            if (!m[u]) continue;
            const uint64_t nb = m[u] & ~(kRec ? sv[u] : tab_seen(L, w[u]));
            if (!nb) continue;
            const int slot = tab_next_claim(L, w[u]);
            if (slot < 0) {
                L.over = 1u;
                continue;
            }
            const uint64_t old = atomicOr((unsigned long long*)&L.nmask[slot], (unsigned long long)nb);
            const uint64_t first = nb & ~old;
            if (kCount && first) count_new(first, 0, (uint32_t)dg[u], cg, ct);
        }
    }
}

// One walk over the arcs [0, total) of a prologue without deduplication
// (the counts of trial_cut): for each arc u -> w, the live bits of u whose
// source has not seen w are counted with deg(w) for those sources, wave by
// wave (wave_count_nodes).  Seen bits from H_seen, or with kRec from the node
// records behind the seen filter.  H_next is not touched.
template <bool kRec>
__device__ void tab_cheap_arcs(const DevGraph& G, const LdsTab& L, const uint64_t* ns, uint32_t total,
                               const PassScratch& X, uint32_t* cg, unsigned long long* ct,
                               const uint32_t* seen_filter = nullptr) {
    constexpr int B = kLdsBlk;
    constexpr int kInflight = 1;
    const uint32_t tid = threadIdx.x;
    const uint32_t wbase = tid & ~63u;
    // wave-uniform loop: a wave runs while any of its lanes has an arc
    for (uint32_t r = 0; r + wbase < total; r += kInflight * B) {
        int32_t w[kInflight];
        uint32_t dg[kInflight];
        uint64_t m[kInflight];
#pragma unroll
        for (int u = 0; u < kInflight; ++u) {
            const uint32_t a = r + (uint32_t)u * B + tid;
            m[u] = 0;
            w[u] = 0;
            dg[u] = 0;
            if (a < total) {
                uint32_t lo = 0, hi = B;
                while (lo < hi) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (X.eoff[mid] <= a) lo = mid + 1; else hi = mid;
                }
                const uint32_t i = lo - 1;
                const int32_t e = X.ebeg[i] + (int32_t)(a - X.eoff[i]);
                m[u] = X.em[i];
                const int2 wd = G.adj[e];
                w[u] = wd.x;
                dg[u] = (uint32_t)wd.y;
            }
        }
#pragma unroll
        for (int u = 0; u < kInflight; ++u) {
            uint64_t nb = 0;
            if (m[u]) {
                uint64_t sv;
                if (kRec) sv = filter_maybe(seen_filter, w[u]) ? ns[(size_t)w[u] * Layout<1>::SW] : 0ull;
                else sv = tab_seen(L, w[u]);
                nb = m[u] & ~sv;
            }
            wave_count_nodes<1>(&nb, nb ? dg[u] : 0u, cg, ct);
        }
    }
}

// Clear H_next after a counting pass.
template <int B>
__device__ inline void tab_next_reset(LdsTab& L) {
    for (int i = threadIdx.x; i < kCapN; i += B) {
        L.nkey[i] = -1;
        L.nmask[i] = 0;
    }
}

// After a build pass: every H_next entry becomes (or updates) an H_seen entry
// and joins the next frontier; H_next is cleared.
template <int B>
__device__ inline void tab_build_pass(LdsTab& L, int32_t* Fn, uint64_t keep = ~0ull) {
    for (int i = threadIdx.x; i < kCapN; i += B) {
        const int32_t w = L.nkey[i];
        if (w < 0) continue;
        const uint64_t bits = L.nmask[i] & keep;
        L.nkey[i] = -1;
        L.nmask[i] = 0;
        if (!bits) continue;
        const int s = tab_seen_claim(L, w);
        if (s < 0) {
            L.over = 1u;
            continue;
        }
        L.sseen[s] |= bits;
        L.sncur[s] = bits;
        Fn[atomicAdd(&L.flen2, 1u)] = s;
    }
}

template <int WW>
__global__ __launch_bounds__(kLdsBlk) void k_batched_lds(DevGraph G, const int32_t* order, int W,
                                                        uint32_t nbatches, uint32_t* next_batch, SlotPtrs base,
                                                        TopKDev T, QStats* st, DeferList D, int force_spill,
                                                        int no_trial) {
    static_assert(WW == 1, "LDS-resident batches hold 64 sources");
    using Lo = Layout<1>;
    constexpr int B = kLdsBlk;
    __shared__ LdsTab L;
    __shared__ union {
        LdsExpand<1, B> e;   // global-record levels
        PassScratch x;       // LDS levels
    } U;
    LdsExpand<1, B>& LE = U.e;
    PassScratch& PX = U.x;
    __shared__ SrcState S[64];
    __shared__ uint32_t cg[kBlk];
    __shared__ unsigned long long ct[kBlk];
    __shared__ CutLds CL;
    __shared__ uint32_t s_flen, s_nlen, s_clen, s_b, s_mode, s_hasth;
    __shared__ uint64_t s_act[4];
    __shared__ unsigned long long s_arcs, s_narcs, s_ent, s_ent_lv;
    const int tid = threadIdx.x;
    const size_t slot = blockIdx.x;
    SlotPtrs P;
    P.ns = base.ns + slot * (size_t)G.n * Lo::SW;
    P.qa = base.qa + slot * (size_t)G.n;
    P.qb = base.qb + slot * (size_t)G.n;
    P.clr = base.clr + slot * (size_t)G.n;
    unsigned long long levels = 0, batches = 0, disc = 0, lds_lv = 0, rec_lv = 0, spills = 0;
    // whether a k-th best record has been published (the trial cut needs one)
    auto has_threshold = [&]() -> bool {
        if (tid == 0) s_hasth = __hip_atomic_load(T.seq, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0u ? 1u : 0u;
        __syncthreads();
        const bool h = uni32(s_hasth) != 0u;
        __syncthreads();
        return h;
    };
    unsigned long long rec_ticks = 0, rec_arcs = 0;
    unsigned long long ticks[5] = {0, 0, 0, 0, 0};
    tab_next_reset<B>(L);
    for (int i = tid; i < kCapS; i += B) {
        L.skey[i] = -1;
        L.sseen[i] = L.scur[i] = L.sncur[i] = 0;
    }
    if (tid == 0) {
        s_narcs = 0;
        s_ent = 0;
        L.nins = L.sfill = L.flen2 = L.over = 0;
    }
    __syncthreads();

    // move the LDS state of the batch into the global node records (level
    // boundary): seen/cur of every H_seen node, the frontier as node ids
    auto to_global = [&](const int32_t* F, uint32_t flen) {
        ++spills;
        if (tid == 0) s_clen = 0;
        __syncthreads();
        for (int i = tid; i < kCapS; i += B) {
            const int32_t w = L.skey[i];
            if (w >= 0) {
                uint64_t* rec = &P.ns[(size_t)w * Lo::SW];
                rec[0] = L.sseen[i];
                rec[Lo::CUR] = L.scur[i];
            }
            append_if(w >= 0, w, P.clr, &s_clen);
        }
        for (uint32_t e = tid; e < flen; e += B) P.qa[e] = L.skey[F[e]];
        __syncthreads();
        for (int i = tid; i < kCapS; i += B) {
            L.skey[i] = -1;
            L.sseen[i] = L.scur[i] = L.sncur[i] = 0;
        }
        if (tid == 0) {
            L.sfill = 0;
            s_mode = 1;
        }
        __syncthreads();
        // every node just written to the records is on the reset list
        const uint32_t nc = s_clen;
        for (uint32_t i = tid; i < nc; i += B) filter_set(L.filter(), P.clr[i]);
        __syncthreads();
    };

    for (;;) {
        if (tid == 0) s_b = atomicAdd(next_batch, 1u);
        __syncthreads();
        const uint32_t b = uni32(s_b);
        __syncthreads();
        if (b >= nbatches) break;
        ++batches;
        const uint64_t tb = __builtin_amdgcn_s_memrealtime();
        // sources: level 0 in H_seen
        if (tid == 0) {
            s_flen = 0;
            s_mode = 0;
        }
        __syncthreads();
        if (tid < W) {
            const int64_t i = (int64_t)b * W + tid;
            SrcState sv;
            sv.nd = 1;
            sv.fd = 0;
            sv.mvis = 0;
            if (i < G.n) {
                const int32_t v = order[i];
                sv.id = v;
                sv.oid = G.orig ? G.orig[v] : v;
                sv.x0 = G.x0[v];
                sv.x1 = G.x1[v];
                sv.tg = G.deg[v];
                sv.status = sv.x0 <= 1 ? S_TRIVIAL : S_LIVE;
                if (sv.status == S_LIVE) {
                    const int sl = tab_seen_claim(L, v);  // <= 64 distinct sources: always fits
                    const uint64_t bit = 1ull << tid;
                    L.sseen[sl] = bit;
                    L.scur[sl] = bit;
                    L.fl[0][atomicAdd(&s_flen, 1u)] = sl;
                }
            } else {
                sv.id = -1;
                sv.oid = -1;
                sv.x0 = sv.x1 = 0;
                sv.tg = 0;
                sv.status = S_EMPTY;
            }
            S[tid] = sv;
        }
        __syncthreads();
        uint32_t live = uni32(cut_step<1>(T, S, W, 0, false, nullptr, nullptr, false, true, st, s_act, CL, &D));
        uint32_t flen = uni32(s_flen), d = 0, cur = 0, stamp = 0;
        uint32_t trial_d = 0;  // level whose over-counted bound test has run (0: none; level 0 needs none)
        uint64_t tp = __builtin_amdgcn_s_memrealtime();
        ticks[0] += tp - tb;
        while (live) {
            if (uni32(s_mode) == 0) {
                // ---------------- LDS level
                const int32_t* F = L.fl[cur];
                bool counted = false;  // the level's arcs are already in node_arcs
                if (!no_trial && d >= 1 && trial_d != d + 1 && has_threshold()) {
                    // one walk without deduplication, then the bound test with
                    // those counts (trial_cut); the exact count below runs
                    // only for the sources it leaves
                    trial_d = d + 1;
                    if (tid < kBlk) {
                        cg[tid] = 0;
                        ct[tid] = 0;
                    }
                    const uint32_t tot0 = tab_prologue(G, L, F, flen, s_act[0], PX, &s_narcs, &s_ent);
                    tab_cheap_arcs<false>(G, L, nullptr, tot0, PX, cg, ct);
                    __syncthreads();
                    counted = true;
                    live = uni32(trial_cut(T, S, W, d + 1, cg, ct, st, s_act, CL));
                    const uint64_t tq = __builtin_amdgcn_s_memrealtime();
                    ticks[1] += tq - tp;
                    tp = tq;
                    if (!live) {
                        ++levels;
                        ++lds_lv;
                        break;
                    }
                }
                const uint64_t act = uni64(s_act[0]);
                if (tid < kBlk) {
                    cg[tid] = 0;
                    ct[tid] = 0;
                }
                if (tid == 0) {
                    L.nins = 0;
                    L.over = 0;
                    s_ent_lv = 0;
                }
                __syncthreads();
                // the prologue's arc total is the level's arc count, which sets
                // the passes (the frontier holds distinct nodes, so it is below
                // m < 2^31); its statistics are kept only if the level stays here
                const uint32_t tot = uni32(tab_prologue(G, L, F, flen, act, PX, nullptr,
                                                        counted ? nullptr : &s_ent_lv));
                const uint32_t npass = (tot + kPassCap - 1) / kPassCap;
                if (npass > kPassMax) {
                    to_global(F, flen);
                    continue;
                }
                if (!counted && tid == 0) {
                    s_narcs += tot;
                    s_ent += s_ent_lv;
                }
                const uint32_t np = npass > 0 ? npass : 1;
                // A single-pass level keeps its H_next (every target with the
                // bits of all sources counted) for the build, which then only
                // masks it with the surviving sources instead of walking the
                // level's arcs again.  Every other way out clears it.
                const bool keep_next = np == 1;
                uint32_t distinct = 0;
                for (uint32_t p = 0; p < np; ++p) {
                    tab_arcs<true, false>(G, L, nullptr, tot, np, p, PX, cg, ct);
                    __syncthreads();
                    if (!keep_next) {
                        tab_next_reset<B>(L);
                        __syncthreads();
                    }
                }
                distinct = uni32(L.nins);
                if (uni32(L.over)) {
                    // a pass overflowed H_next: count this level on the global records
                    if (tid < kBlk) {
                        cg[tid] = 0;
                        ct[tid] = 0;
                    }
                    if (keep_next) tab_next_reset<B>(L);
                    __syncthreads();
                    to_global(F, flen);
                    continue;
                }
                disc += distinct;
                ++lds_lv;
                uint64_t tq = __builtin_amdgcn_s_memrealtime();
                ticks[1] += tq - tp;
                tp = tq;
                ++d;
                ++levels;
                live = uni32(cut_step<1>(T, S, W, d, true, cg, ct, false, true, st, s_act, CL, &D));
                tq = __builtin_amdgcn_s_memrealtime();
                ticks[2] += tq - tp;
                tp = tq;
                if (!live) {
                    if (keep_next) {
                        tab_next_reset<B>(L);
                        __syncthreads();
                    }
                    break;
                }
                const uint64_t lact = uni64(s_act[0]);
                // nodes to build <= sum of gamma over the live sources
                if (tid == 0) L.tsum = 0;
                __syncthreads();
                if (tid < 64 && ((lact >> tid) & 1ull)) atomicAdd(&L.tsum, (unsigned long long)cg[tid]);
                __syncthreads();
                // distinct nodes of the new level with a live bit: at most the
                // pairs counted for the live sources, and at most the distinct
                // targets the count passes inserted
                const unsigned long long live_nodes = min((unsigned long long)uni64(L.tsum), (unsigned long long)distinct);
                if (force_spill || uni32(L.sfill) + live_nodes > kSeenCap) {
                    // the new level does not fit H_seen: build it on the global records
                    if (keep_next) {
                        tab_next_reset<B>(L);
                        __syncthreads();
                    }
                    to_global(F, flen);
                    if (tid == 0) s_nlen = 0;
                    __syncthreads();
                    ++stamp;
                    for (uint32_t e0 = 0; e0 < flen; e0 += B)
                        expand_entries<1, B, 1>(G, P, P.qa, e0, min(flen, e0 + B), s_act, P.qb, &s_nlen, stamp, LE,
                                             &s_arcs, &s_arcs);
                    __syncthreads();
                    const uint32_t nlen = uni32(s_nlen);
                    clear_cur<1>(P, P.qa, flen, 0, B);
                    if (tid == 0) s_flen = 0;
                    __syncthreads();
                    build_level<1>(P, P.qb, nlen, 0, B, s_act, true, P.qa, &s_flen, &s_clen, &s_arcs, L.filter());
                    __syncthreads();
                    flen = uni32(s_flen);
                    tq = __builtin_amdgcn_s_memrealtime();
                    ticks[3] += tq - tp;
                    tp = tq;
                    continue;
                }
                // build the live bits of the level into H_seen
                int32_t* Fn = L.fl[cur ^ 1];
                if (tid == 0) L.flen2 = 0;
                __syncthreads();
                if (keep_next) {
                    // H_next of the count holds, per target, the bits of every
                    // source counted; the survivors' bits are the new level
                    tab_build_pass<B>(L, Fn, lact);
                    __syncthreads();
                } else {
                    const uint32_t tot2 = tab_prologue(G, L, F, flen, lact, PX, nullptr, nullptr);
                    for (uint32_t p = 0; p < np; ++p) {
                        tab_arcs<false, false>(G, L, nullptr, tot2, np, p, PX, nullptr, nullptr);
                        __syncthreads();
                        tab_build_pass<B>(L, Fn);
                        __syncthreads();
                    }
                }
                for (uint32_t e = tid; e < flen; e += B) L.scur[F[e]] = 0;
                __syncthreads();
                const uint32_t fl2 = uni32(L.flen2);
                for (uint32_t e = tid; e < fl2; e += B) {
                    const int32_t sl = Fn[e];
                    L.scur[sl] = L.sncur[sl];
                    L.sncur[sl] = 0;
                }
                __syncthreads();
                flen = fl2;
                cur ^= 1;
                tq = __builtin_amdgcn_s_memrealtime();
                ticks[3] += tq - tp;
                tp = tq;
            } else {
                // ---------------- global level (state on the node records)
                const uint64_t tr0 = tp;
                const unsigned long long ra0 = uni64(s_narcs), en0 = uni64(s_ent);
                bool counted = false;
                if (!no_trial && d >= 1 && trial_d != d + 1 && has_threshold()) {
                    trial_d = d + 1;
                    if (tid < kBlk) {
                        cg[tid] = 0;
                        ct[tid] = 0;
                    }
                    __syncthreads();
                    const uint64_t act0 = uni64(s_act[0]);
                    for (uint32_t e0 = 0; e0 < flen; e0 += B) {
                        const uint32_t tot = rec_prologue(G, P, P.qa, e0, min(flen, e0 + B), act0, PX, &s_narcs,
                                                          &s_ent);
                        tab_cheap_arcs<true>(G, L, P.ns, tot, PX, cg, ct, L.filter());
                        __syncthreads();
                    }
                    counted = true;
                    live = uni32(trial_cut(T, S, W, d + 1, cg, ct, st, s_act, CL));
                    const uint64_t tq = __builtin_amdgcn_s_memrealtime();
                    ticks[1] += tq - tp;
                    tp = tq;
                    if (!live) {
                        ++levels;
                        ++rec_lv;
                        rec_ticks += tq - tr0;
                        rec_arcs += uni64(s_narcs) - ra0;
                        break;
                    }
                }
                const uint64_t act = uni64(s_act[0]);
                // When the level's arcs fit the LDS counting passes, count it in
                // H_next with the seen bits read from the node records (no global
                // atomics); the records take the level only if a source survives.
                if (tid == 0) L.tsum = 0;
                __syncthreads();
                {
                    unsigned long long tl = 0;
                    for (uint32_t e = tid; e < flen; e += B) {
                        const int32_t u = P.qa[e];
                        if (P.ns[(size_t)u * Lo::SW + Lo::CUR] & act) tl += G.deg[u];
                    }
                    if (tl) atomicAdd(&L.tsum, tl);
                }
                __syncthreads();
                const unsigned long long Tarcs = uni64(L.tsum);
                const uint32_t npass = (uint32_t)((Tarcs + kPassCap - 1) / kPassCap);
                bool hybrid = false;
                if (npass <= kPassMax) {
                    const uint32_t np = npass > 0 ? npass : 1;
                    if (tid < kBlk) {
                        cg[tid] = 0;
                        ct[tid] = 0;
                    }
                    if (tid == 0) {
                        L.nins = 0;
                        L.over = 0;
                    }
                    __syncthreads();
                    for (uint32_t p = 0; p < np; ++p) {
                        for (uint32_t e0 = 0; e0 < flen; e0 += B) {
                            const uint32_t tot = rec_prologue(G, P, P.qa, e0, min(flen, e0 + B), act, PX,
                                                              (p == 0 && !counted) ? &s_narcs : nullptr,
                                                              (p == 0 && !counted) ? &s_ent : nullptr);
                            tab_arcs<true, true>(G, L, P.ns, tot, np, p, PX, cg, ct, L.filter());
                            __syncthreads();
                        }
                        tab_next_reset<B>(L);
                        __syncthreads();
                    }
                    hybrid = uni32(L.over) == 0u;
                    if (!hybrid && tid == 0) {
                        s_narcs = ra0;  // recounted below
                        s_ent = en0;
                    }
                    __syncthreads();
                }
                if (hybrid) {
                    disc += uni32(L.nins);
                    ++rec_lv;
                    uint64_t tq = __builtin_amdgcn_s_memrealtime();
                    ticks[1] += tq - tp;
                    tp = tq;
                    ++d;
                    ++levels;
                    live = uni32(cut_step<1>(T, S, W, d, true, cg, ct, false, true, st, s_act, CL, &D));
                    tq = __builtin_amdgcn_s_memrealtime();
                    ticks[2] += tq - tp;
                    tp = tq;
                    if (live) {
                        // materialise the level for the surviving sources
                        ++stamp;
                        if (tid == 0) s_nlen = 0;
                        __syncthreads();
                        for (uint32_t e0 = 0; e0 < flen; e0 += B)
                            expand_entries<1, B, 1>(G, P, P.qa, e0, min(flen, e0 + B), s_act, P.qb, &s_nlen, stamp,
                                                 LE, &s_arcs, &s_arcs);
                        __syncthreads();
                        const uint32_t nlen = uni32(s_nlen);
                        clear_cur<1>(P, P.qa, flen, 0, B);
                        if (tid == 0) s_flen = 0;
                        __syncthreads();
                        build_level<1>(P, P.qb, nlen, 0, B, s_act, true, P.qa, &s_flen, &s_clen, &s_arcs,
                                       L.filter());
                        __syncthreads();
                        flen = uni32(s_flen);
                    }
                    tq = __builtin_amdgcn_s_memrealtime();
                    ticks[3] += tq - tp;
                    tp = tq;
                    rec_ticks += tq - tr0;
                    rec_arcs += uni64(s_narcs) - ra0;
                    continue;
                }
                ++stamp;
                if (tid < kBlk) {
                    cg[tid] = 0;
                    ct[tid] = 0;
                }
                if (tid == 0) s_nlen = 0;
                __syncthreads();
                for (uint32_t e0 = 0; e0 < flen; e0 += B)
                    expand_entries<1, B, 1>(G, P, P.qa, e0, min(flen, e0 + B), s_act, P.qb, &s_nlen, stamp, LE,
                                         &s_narcs, &s_ent);
                __syncthreads();
                const uint32_t nlen = uni32(s_nlen);
                count_level<1, B>(P, P.qb, nlen, cg, ct);
                __syncthreads();
                disc += nlen;
                ++rec_lv;
                uint64_t tq = __builtin_amdgcn_s_memrealtime();
                ticks[1] += tq - tp;
                tp = tq;
                ++d;
                ++levels;
                live = uni32(cut_step<1>(T, S, W, d, true, cg, ct, false, true, st, s_act, CL, &D));
                tq = __builtin_amdgcn_s_memrealtime();
                ticks[2] += tq - tp;
                tp = tq;
                clear_cur<1>(P, P.qa, flen, 0, B);
                if (tid == 0) s_flen = 0;
                __syncthreads();
                build_level<1>(P, P.qb, nlen, 0, B, s_act, live != 0, P.qa, &s_flen, &s_clen, &s_arcs,
                               L.filter());
                __syncthreads();
                flen = uni32(s_flen);
                tq = __builtin_amdgcn_s_memrealtime();
                ticks[3] += tq - tp;
                tp = tq;
                rec_ticks += tq - tr0;
                rec_arcs += uni64(s_narcs) - ra0;
            }
        }
        // reset the batch state: global records (when used) and the LDS tables
        if (uni32(s_mode) == 1) {
            const uint32_t nc = uni32(s_clen);
            for (uint32_t i = tid; i < nc; i += B) {
                uint64_t* rec = &P.ns[(size_t)P.clr[i] * Lo::SW];
                rec[0] = 0;
                rec[Lo::CUR] = 0;
            }
        }
        for (int i = tid; i < kCapS; i += B) {
            L.skey[i] = -1;
            L.sseen[i] = L.scur[i] = L.sncur[i] = 0;
        }
        if (tid == 0) L.sfill = 0;
        __syncthreads();
        ticks[4] += __builtin_amdgcn_s_memrealtime() - tp;
    }
    if (tid == 0) {
        atomicAdd(&st->levels, levels);
        atomicAdd(&st->batches, batches);
        atomicAdd(&st->discovered, disc);
        if (s_narcs) atomicAdd(&st->node_arcs, s_narcs);
        if (s_ent) atomicAdd(&st->frontier_entries, s_ent);
        for (int i = 0; i < 5; ++i) atomicAdd(&st->phase_ticks[i], ticks[i]);
        atomicAdd(&st->lds_levels, lds_lv);
        atomicAdd(&st->record_ticks, rec_ticks);
        atomicAdd(&st->record_arcs, rec_arcs);
        atomicAdd(&st->record_levels, rec_lv);
        atomicAdd(&st->spills, spills);
    }
}

// --------------------------------------------------------- host side

struct QueryBufs {
    DevBuf order, topk, ring, stats;
};

struct Timing {
    double seed_ms = 0, persistent_ms = 0, defer_ms = 0;
    QStats seed_stats{}, persist_stats{};
};

int device_cus() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) return 256;
    return cus;
}

unsigned clamp_grid(int64_t work_items, int64_t cap) {
    int64_t b = (work_items + kBlk - 1) / kBlk;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

// RAII owner of a captured graph and its executable.
struct GraphHolder {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~GraphHolder() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

// RAII pair of HIP events recorded on the query stream.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
    bc_status create() {
        BC_HIP(hipEventCreate(&a));
        BC_HIP(hipEventCreate(&b));
        return BC_OK;
    }
    bc_status ms(double* out) {
        float t = 0.f;
        BC_HIP(hipEventSynchronize(b));
        BC_HIP(hipEventElapsedTime(&t, a, b));
        *out = t;
        return BC_OK;
    }
};

// Level-synchronous slot of the workspace (sized for WW words per node).
template <int WW>
bc_status ensure_plain(Workspace& W_, const DevGraph& G, hipStream_t s) {
    if (W_.plain_ready && W_.ww == WW) return BC_OK;
    const size_t N = (size_t)G.n, words = N * Layout<WW>::SW;
    BC_TRY(W_.seen.alloc_on(sizeof(uint64_t) * words, s));
    BC_TRY(W_.qa.alloc_on(sizeof(int32_t) * N, s));
    BC_TRY(W_.qb.alloc_on(sizeof(int32_t) * N, s));
    BC_TRY(W_.clr.alloc_on(sizeof(int32_t) * N, s));
    BC_TRY(W_.srcs.alloc_on(sizeof(SrcState) * kBlk, s));
    BC_TRY(W_.ctl.alloc_on(sizeof(Ctl), s));
    if (!W_.hctl) BC_HIP(hipHostMalloc((void**)&W_.hctl, 64, hipHostMallocDefault));
    BC_HIP(hipMemsetAsync(W_.seen.p, 0, sizeof(uint64_t) * words, s));
    BC_HIP(hipMemsetAsync(W_.ctl.p, 0, sizeof(Ctl), s));
    if (N > 0) k_slot_init<WW><<<clamp_grid((int64_t)N, 4096), kBlk, 0, s>>>(G.deg, G.n, W_.seen.as<uint64_t>(), 1);
    W_.plain_ready = true;
    return BC_OK;
}

// Persistent slots of the workspace.
template <int WW>
bc_status ensure_batched(Workspace& W_, const DevGraph& G, int want, hipStream_t s) {
    if (W_.slots >= want && W_.ww == WW) return BC_OK;
    const size_t N = (size_t)G.n, words = N * Layout<WW>::SW;
    const size_t S_ = (size_t)want;
    W_.bseen.release();
    W_.bqa.release();
    W_.bqb.release();
    W_.bclr.release();
    W_.slot_stamp.release();
    W_.slots = 0;
    BC_TRY(W_.bseen.alloc_on(sizeof(uint64_t) * words * S_, s));
    BC_TRY(W_.bqa.alloc_on(sizeof(int32_t) * N * S_, s));
    BC_TRY(W_.bqb.alloc_on(sizeof(int32_t) * N * S_, s));
    BC_TRY(W_.bclr.alloc_on(sizeof(int32_t) * N * S_, s));
    BC_TRY(W_.slot_stamp.alloc_on(sizeof(uint32_t) * S_, s));
    BC_HIP(hipMemsetAsync(W_.bseen.p, 0, sizeof(uint64_t) * words * S_, s));
    BC_HIP(hipMemsetAsync(W_.slot_stamp.p, 0, sizeof(uint32_t) * S_, s));
    if (N > 0)
        k_slot_init<WW><<<clamp_grid((int64_t)(N * S_), 16384), kBlk, 0, s>>>(G.deg, G.n, W_.bseen.as<uint64_t>(),
                                                                               want);
    W_.slots = want;
    return BC_OK;
}

// Level-synchronous batches over order[0, count), batches [0, nb), on the
// plain slot of Wk (sized for WW words per node), adding their kernel time
// to *ms.
// Workgroups of a cooperative level launch: as many as the device holds at
// once, up to kCoopPerCu per compute unit (more make each grid barrier
// slower than they make a level faster); 0 when the device cannot launch
// the kernel cooperatively.
constexpr int kCoopPerCu = 1;

template <int WW>
int coop_grid() {
    int dev = 0, coop = 0, per_cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k_plain_coop<WW>), kBlk,
                                                     0) != hipSuccess) {
        (void)hipGetLastError();
        return 0;
    }
    return std::min(per_cu, kCoopPerCu) * device_cus();
}

// Debugging aid of the host-driven level loop (environment variable
// BC_CHECK_LISTS=1): after every level, copy the frontier and reset lists to
// the host and check that every listed id is a node (the lengths are checked
// on every run).  A violation fails the query before any kernel indexes
// the records with a bad id.
bool check_lists_enabled() {
    const char* e = std::getenv("BC_CHECK_LISTS");
    return e && e[0] == '1';
}

bc_status check_level_lists(const SlotPtrs& P, uint32_t flen, uint32_t clen, int32_t n, uint32_t level,
                            hipStream_t s) {
    std::vector<int32_t> h(std::max(flen, clen));
    const std::pair<const int32_t*, uint32_t> lists[2] = {{P.qa, flen}, {P.clr, clen}};
    for (int l = 0; l < 2; ++l) {
        if (lists[l].second == 0) continue;
        BC_HIP(hipMemcpyAsync(h.data(), lists[l].first, sizeof(int32_t) * lists[l].second, hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        for (uint32_t i = 0; i < lists[l].second; ++i)
            if (h[i] < 0 || h[i] >= n) {
                set_error("internal: level %u %s list entry %u is %d, not a node of 0..%d", level,
                          l == 0 ? "frontier" : "reset", i, h[i], n - 1);
                return BC_EDEVICE;
            }
    }
    return BC_OK;
}

// Workgroups per compute unit of the host loop's grid-stride level kernels
// other than push and pull (count, build and the clears).  Their lists are
// often short, and every workgroup of a launch takes a device-wide counter
// (the last one runs the level's cut step or publishes the list), so fewer
// workgroups finish a level sooner: 1 per compute unit measured faster than
// 2, 4 or 8 (BA n = 1M seed batches, R-MAT deferred re-runs).
constexpr int kLevelGrid = 1;

template <int WW>
bc_status run_plain_batches(const DevGraph& G, const int32_t* ord, int32_t count, uint32_t nb, Workspace& Wk,
                            TopKDev T, QStats* d_st, const LevelParams& lp, hipStream_t s, double* ms,
                            int graph_levels) {
    const bool check_lists = check_lists_enabled();
    const int W = 64 * WW;
    const int32_t n = G.n;
    const int cus = device_cus();
    if (Wk.ww != WW) {
        Wk.plain_ready = false;
        Wk.slots = 0;
        Wk.ww = WW;
    }
    BC_TRY(ensure_plain<WW>(Wk, G, s));
    SlotPtrs P{Wk.seen.as<uint64_t>(), Wk.qa.as<int32_t>(), Wk.qb.as<int32_t>(), Wk.clr.as<int32_t>()};
    SrcState* S = Wk.srcs.as<SrcState>();
    Ctl* C = Wk.ctl.as<Ctl>();
    uint32_t* hctl = Wk.hctl;
    const int cgrid = graph_levels == -1 && nb > 0 ? coop_grid<WW>() : 0;
    if (graph_levels == -1 && nb > 0 && cgrid == 0) {
        set_error("this device cannot run the level loop as one cooperative launch");
        return BC_EINVAL;
    }
    if (cgrid > 0) {
        // every level of every batch in one cooperative launch
        BC_HIP(hipMemsetAsync(&C->err, 0, sizeof(uint32_t), s));
        EventPair ev;
        BC_TRY(ev.create());
        DevGraph a_g = G;
        const int32_t* a_ord = ord;
        int32_t a_count = count;
        uint32_t a_b0 = 0, a_nb = nb;
        int a_w = W;
        SlotPtrs a_p = P;
        SrcState* a_s = S;
        Ctl* a_c = C;
        TopKDev a_t = T;
        QStats* a_st = d_st;
        LevelParams a_lp = lp;
        void* args[] = {&a_g, &a_ord, &a_count, &a_b0, &a_nb, &a_w, &a_p, &a_s, &a_c, &a_t, &a_st, &a_lp};
        BC_HIP(hipEventRecord(ev.a, s));
        BC_HIP(hipLaunchCooperativeKernel(reinterpret_cast<const void*>(k_plain_coop<WW>), dim3(cgrid), dim3(kBlk),
                                          args, 0, s));
        BC_HIP(hipEventRecord(ev.b, s));
        uint32_t err = 0;
        BC_HIP(hipMemcpyAsync(&err, &C->err, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        double t = 0;
        BC_TRY(ev.ms(&t));
        BC_HIP(hipStreamSynchronize(s));  // the copy of the error word
        if (err) {
            set_error("internal: a level list of the cooperative loop exceeded n = %d", n);
            return BC_EDEVICE;
        }
        *ms += t;
        return BC_OK;
    }
    // graph_levels > 0: capture that many gated level steps once and replay
    // them, reading the control block once per replay instead of per level
    GraphHolder gh;
    if (graph_levels > 0 && nb > 0) {
        if (!Wk.cap) BC_HIP(hipStreamCreateWithFlags(&Wk.cap, hipStreamNonBlocking));  // default priority
        BC_HIP(hipStreamBeginCapture(Wk.cap, hipStreamCaptureModeThreadLocal));
        for (int l = 0; l < graph_levels; ++l) {
            k_plain_expand<WW><<<8 * cus, kBlk, 0, Wk.cap>>>(G, P, C, d_st, 1);
            k_plain_count<WW><<<4 * cus, kBlk, 0, Wk.cap>>>(P, S, C, T, d_st, W, 1);
            k_plain_pull<WW><<<clamp_grid(n, 8 * cus), kBlk, 0, Wk.cap>>>(G, P, S, C, T, d_st, W, 1);
            k_plain_clearcur<WW><<<4 * cus, kBlk, 0, Wk.cap>>>(P, C, 1);
            k_plain_build<WW><<<4 * cus, kBlk, 0, Wk.cap>>>(G, P, C, lp, 1);
        }
        const hipError_t ce = hipStreamEndCapture(Wk.cap, &gh.graph);
        BC_HIP(ce);
        BC_HIP(hipGraphInstantiate(&gh.exec, gh.graph, nullptr, nullptr, 0));
    }
    EventPair ev;
    BC_TRY(ev.create());
    BC_HIP(hipEventRecord(ev.a, s));
    for (uint32_t b = 0; b < nb; ++b) {
        k_plain_init<WW><<<1, kBlk, 0, s>>>(G, ord, count, b, W, P, S, C, T, d_st);
        for (;;) {
            BC_HIP(hipMemcpyAsync(hctl, C, 64, hipMemcpyDeviceToHost, s));
            BC_HIP(hipStreamSynchronize(s));
            // control block words: d, flen, nlen, clen, live, pull, chunk, done, stamp, ran, front_arcs
            const uint32_t flen = hctl[1], live = hctl[4], pull = hctl[5];
            // every list holds distinct nodes, so no length can exceed n: a
            // longer one means the level step wrote out of order, and no
            // further kernel may index the lists with it
            if (flen > (uint32_t)n || hctl[2] > (uint32_t)n || hctl[3] > (uint32_t)n) {
                set_error("internal: level %u list lengths %u/%u/%u exceed n = %d", hctl[0], flen, hctl[2], hctl[3],
                          n);
                return BC_EDEVICE;
            }
            unsigned long long fa;
            std::memcpy(&fa, hctl + 10, sizeof(fa));
            if (check_lists) BC_TRY(check_level_lists(P, flen, hctl[3], n, hctl[0], s));
            if (!live) break;
            if (gh.exec) {
                BC_HIP(hipGraphLaunch(gh.exec, s));
                continue;
            }
            if (pull) {
                k_plain_pull<WW><<<clamp_grid(n, 8 * cus), kBlk, 0, s>>>(G, P, S, C, T, d_st, W, 0);
            } else {
                // one workgroup per claimed chunk, up to 8 per compute unit
                const int64_t chunks = ((int64_t)flen + expand_chunk(flen, fa) - 1) / expand_chunk(flen, fa);
                k_plain_expand<WW><<<clamp_grid(chunks * kBlk, 8 * cus), kBlk, 0, s>>>(G, P, C, d_st, 0);
                // new nodes <= arcs out of the frontier
                k_plain_count<WW><<<clamp_grid((int64_t)std::min<unsigned long long>(fa, (unsigned long long)n),
                                               kLevelGrid * cus), kBlk, 0, s>>>(P, S, C, T, d_st, W, 0);
            }
            k_plain_clearcur<WW><<<clamp_grid(flen, kLevelGrid * cus), kBlk, 0, s>>>(P, C, 0);
            // reached nodes <= arcs out of the frontier (push) or n (pull)
            const int64_t bound =
                pull ? (int64_t)n : (int64_t)std::min<unsigned long long>(fa, (unsigned long long)n);
            k_plain_build<WW><<<clamp_grid(bound, kLevelGrid * cus), kBlk, 0, s>>>(G, P, C, lp, 0);
        }
        k_plain_clear<WW><<<clamp_grid(n, kLevelGrid * cus), kBlk, 0, s>>>(P, C);
    }
    BC_HIP(hipEventRecord(ev.b, s));
    BC_HIP(hipGetLastError());
    double t = 0;
    BC_TRY(ev.ms(&t));
    *ms += t;
    return BC_OK;
}

// Seed batches of the batched mode: their width sw (a multiple of W; 0 in
// the options = W, or 256 when k > W: one wide level-synchronous batch costs
// less than several narrow ones and holds more of the deepest sources) and
// count (default ceil(k / sw), so that k sources complete before the
// persistent phase and the k-th best value exists).
struct SeedPlan {
    int sw;
    uint32_t batches;  // of width sw
};
SeedPlan seed_plan(const bc_opts& o, int32_t k, int32_t n, int W) {
    int sw = o.seed_width > 0 ? o.seed_width : (k > W ? 256 : W);
    if (sw < W || sw % W != 0) sw = W;
    const int64_t nb = ((int64_t)n + sw - 1) / sw;
    const int64_t sb = o.seed_batches >= 0 ? o.seed_batches : ((int64_t)k + sw - 1) / sw;
    return SeedPlan{sw, (uint32_t)std::min<int64_t>(std::max<int64_t>(sb, 0), nb)};
}

template <int WW>
bc_status run_ww(bc_graph* g, int32_t k, const bc_opts& o, const int32_t* d_order, TopKDev T, QStats* d_st,
                 Workspace& Wk, int W, Timing& tm, hipStream_t s) {
    using Lo = Layout<WW>;
    const DevGraph& G = g->dg;
    const int32_t n = G.n;
    const size_t N = (size_t)n;
    const uint32_t nbatches = (uint32_t)((n + W - 1) / W);
    const bool batched = o.mode == BC_MODE_BATCHED;
    uint32_t seed = nbatches;  // first batch (of width W) of the persistent phase
    SeedPlan sp{W, 0};
    if (batched) {
        sp = seed_plan(o, k, n, W);
        seed = (uint32_t)std::min<int64_t>((int64_t)sp.batches * (sp.sw / W), nbatches);
    }
    LevelParams lp{o.pull_alpha, o.pull_beta > 0.f ? o.pull_beta : 24.f, o.pull_alpha > 0.f ? 1 : 0};
    const int cus = device_cus();
    if (Wk.ww != WW) {
        // a different width: drop buffers sized for the old one
        Wk.plain_ready = false;
        Wk.slots = 0;
        Wk.ww = WW;
    }

    auto run_plain = [&](const int32_t* ord, int32_t count, uint32_t nb, double* ms) -> bc_status {
        return run_plain_batches<WW>(G, ord, count, nb, Wk, T, d_st, lp, s, ms, o.graph_levels);
    };

    if (!batched && seed > 0) BC_TRY(run_plain(d_order, n, seed, &tm.seed_ms));
    if (batched && sp.batches > 0) {
        if (sp.sw == W) {
            BC_TRY(run_plain(d_order, n, sp.batches, &tm.seed_ms));
        } else {
            // wider seed batches: the first sp.batches * sp.sw sources of the order
            Workspace wide(s);
            if (sp.sw == 128) BC_TRY(run_plain_batches<2>(G, d_order, n, sp.batches, wide, T, d_st, lp, s, &tm.seed_ms, o.graph_levels));
            else BC_TRY(run_plain_batches<4>(G, d_order, n, sp.batches, wide, T, d_st, lp, s, &tm.seed_ms, o.graph_levels));
            BC_HIP(hipStreamSynchronize(s));
        }
    }
    if (seed > 0) {
        BC_HIP(hipMemcpyAsync(&tm.seed_stats, d_st, sizeof(QStats), hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
    }

    if (batched && seed < nbatches) {
        int slots = o.slots > 0 ? o.slots : cus;
        // per-slot bytes: node records (SW words) and three int32 lists per node
        const size_t per_slot = N * (8 * Lo::SW + 12);
        size_t freeb = 0, totalb = 0;
        if (Wk.slots < slots && hipMemGetInfo(&freeb, &totalb) == hipSuccess && per_slot > 0) {
            const size_t have = (size_t)Wk.slots * per_slot;
            const size_t cap = ((size_t)(0.45 * (double)freeb) + have) / per_slot;
            if ((size_t)slots > cap) slots = (int)std::max<size_t>(cap, 1);
        }
        if ((uint32_t)slots > nbatches - seed) slots = (int)(nbatches - seed);
        BC_TRY(ensure_batched<WW>(Wk, G, slots, s));
        BC_TRY(Wk.nextb.alloc_on(sizeof(uint32_t), s));
        BC_HIP(hipMemcpyAsync(Wk.nextb.p, &seed, sizeof(uint32_t), hipMemcpyHostToDevice, s));
        SlotPtrs base{Wk.bseen.as<uint64_t>(), Wk.bqa.as<int32_t>(), Wk.bqb.as<int32_t>(), Wk.bclr.as<int32_t>()};
        BC_TRY(Wk.defer.alloc_on(sizeof(int32_t) * N + 64, s));
        uint32_t* dcnt = (uint32_t*)(Wk.defer.as<char>() + sizeof(int32_t) * N);
        BC_HIP(hipMemsetAsync(dcnt, 0, sizeof(uint32_t), s));
        DeferList D{Wk.defer.as<int32_t>(), dcnt,
                    o.defer_arcs < 0 ? 0ull : (uint64_t)(o.defer_arcs > 0 ? o.defer_arcs : 65536)};
        EventPair ev;
        BC_TRY(ev.create());
        BC_HIP(hipEventRecord(ev.a, s));
        const uint32_t chunk = (uint32_t)(o.chunk > 0 ? o.chunk : 1);
        if constexpr (WW == 1) {
            if (o.lds_tables >= 0)
                k_batched_lds<1><<<slots, kLdsBlk, 0, s>>>(G, d_order, W, nbatches, Wk.nextb.as<uint32_t>(), base,
                                                           T, d_st, D, o.lds_tables == 1 ? 1 : 0,
                                                           (o.bounds & BC_BOUND_NO_TRIAL) ? 1 : 0);
            else
                k_batched<WW, kBatchBlk><<<slots, kBatchBlk, 0, s>>>(G, d_order, W, nbatches, Wk.nextb.as<uint32_t>(),
                                                                     chunk, base, Wk.slot_stamp.as<uint32_t>(), T, d_st, D);
        } else {
            k_batched<WW, kBatchBlk><<<slots, kBatchBlk, 0, s>>>(G, d_order, W, nbatches, Wk.nextb.as<uint32_t>(),
                                                                 chunk, base, Wk.slot_stamp.as<uint32_t>(), T, d_st, D);
        }
        BC_HIP(hipEventRecord(ev.b, s));
        BC_HIP(hipGetLastError());
        BC_TRY(ev.ms(&tm.persistent_ms));
        BC_HIP(hipMemcpyAsync(&tm.persist_stats, d_st, sizeof(QStats), hipMemcpyDeviceToHost, s));
        uint32_t ndef = 0;
        BC_HIP(hipMemcpyAsync(&ndef, dcnt, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        if (ndef > 0) {
            // deferred sources, restarted level-synchronously against the
            // final-ish threshold, in batches of defer_width sources (by
            // default the narrowest width that holds them all in one batch,
            // else 256: a wide batch shares each full-graph level sweep among
            // more sources, a narrow one moves smaller node records)
            const int dw = o.defer_width > 0 ? o.defer_width : (ndef <= 64 ? 64 : (ndef <= 128 ? 128 : 256));
            const int32_t* dl = Wk.defer.as<int32_t>();
            const uint32_t dnb = (ndef + (uint32_t)dw - 1) / (uint32_t)dw;
            if (dw == W) {
                BC_TRY(run_plain(dl, (int32_t)ndef, dnb, &tm.defer_ms));
            } else {
                Workspace wide(s);
                if (dw == 64) BC_TRY(run_plain_batches<1>(G, dl, (int32_t)ndef, dnb, wide, T, d_st, lp, s, &tm.defer_ms, o.graph_levels));
                else if (dw == 128) BC_TRY(run_plain_batches<2>(G, dl, (int32_t)ndef, dnb, wide, T, d_st, lp, s, &tm.defer_ms, o.graph_levels));
                else BC_TRY(run_plain_batches<4>(G, dl, (int32_t)ndef, dnb, wide, T, d_st, lp, s, &tm.defer_ms, o.graph_levels));
                BC_HIP(hipStreamSynchronize(s));
            }
        }
    }
    BC_HIP(hipStreamSynchronize(s));
    return BC_OK;
}

}  // namespace

namespace {

// Top-k query, or (all_f != nullptr) the exact farness and reach of every
// node: the same batches with no list and no threshold, so nothing is cut.
bc_status run_query(bc_graph* g, int32_t k, bc_opts o, int32_t* ids, uint64_t* farness, uint32_t* reach,
                    int32_t* count, bc_stats* st_out, uint64_t* all_f, uint32_t* all_r, hipStream_t s,
                    bool private_ws) {
    auto t0 = std::chrono::steady_clock::now();
    const bool all = all_f != nullptr;
    if (all) {
        k = g->dg.n;
        if (o.seed_batches < 0) o.seed_batches = 0;  // no threshold to seed
    }
    const int32_t n = g->dg.n;
    const int W = o.width;
    if (W != 64 && W != 128 && W != 256) {
        set_error("width must be 64, 128 or 256 (got %d)", W);
        return BC_EINVAL;
    }
    if (o.mode != BC_MODE_PLAIN && o.mode != BC_MODE_BATCHED) {
        set_error("unknown mode %d", o.mode);
        return BC_EINVAL;
    }
    if (o.graph_levels < -1 || o.graph_levels > 64) {
        set_error("graph_levels must be in [-1, 64] (got %d)", o.graph_levels);
        return BC_EINVAL;
    }
    if (o.seed_width != 0 && o.seed_width != 64 && o.seed_width != 128 && o.seed_width != 256) {
        set_error("seed_width must be 0, 64, 128 or 256 (got %d)", o.seed_width);
        return BC_EINVAL;
    }
    if (o.defer_width != 0 && o.defer_width != 64 && o.defer_width != 128 && o.defer_width != 256) {
        set_error("defer_width must be 0, 64, 128 or 256 (got %d)", o.defer_width);
        return BC_EINVAL;
    }
    const int32_t kk = std::min(k, n);
    QStats hst;
    std::memset(&hst, 0, sizeof(hst));
    Timing tm;
    if (kk > 0) {
        QueryBufs B;
        BC_TRY(B.order.alloc_on(sizeof(int32_t) * (size_t)n, s));
        int32_t* d_order = B.order.as<int32_t>();
        BC_TRY(build_order(g, o, kk, d_order, s));
        // top-k list: cnt, lock, seq (16 B header) + k records; ring of n + 1
        // records (every-node mode: only the header, and the per-node outputs)
        const size_t hdr = 64;
        const size_t nrec = all ? 0 : (size_t)kk;
        BC_TRY(B.topk.alloc_on(hdr + sizeof(Rec) * nrec, s));
        BC_TRY(B.ring.alloc_on(sizeof(ThRec) * (all ? 1 : (size_t)n + 1), s));
        BC_TRY(B.stats.alloc_on(sizeof(QStats), s));
        DevBuf allf, allr;
        if (all) {
            BC_TRY(allf.alloc_on(sizeof(uint64_t) * (size_t)n, s));
            BC_TRY(allr.alloc_on(sizeof(uint32_t) * (size_t)n, s));
        }
        BC_HIP(hipMemsetAsync(B.topk.p, 0, hdr + sizeof(Rec) * nrec, s));
        BC_HIP(hipMemsetAsync(B.stats.p, 0, sizeof(QStats), s));
        TopKDev T;
        T.k = kk;
        char* hb = B.topk.as<char>();
        T.cnt = (int32_t*)hb;
        T.lock = (uint32_t*)(hb + 4);
        T.seq = (uint32_t*)(hb + 8);
        T.list = (Rec*)(hb + hdr);
        T.ring = B.ring.as<ThRec>();
        T.all_f = all ? allf.as<uint64_t>() : nullptr;
        T.all_r = all ? allr.as<uint32_t>() : nullptr;
        T.footnote = (!g->dg.directed && (o.bounds & BC_BOUND_FOOTNOTE)) ? 1 : 0;
        QStats* d_st = B.stats.as<QStats>();
        // the graph's cached workspace, or a private one when another query holds it
        std::unique_ptr<Workspace> own;
        Workspace* wk = nullptr;
        if (!private_ws) {
            std::lock_guard<std::mutex> lk(g->ws_mu);
            if (!g->ws_busy) {
                if (!g->ws || g->ws->stream != s) g->ws.reset(new Workspace(s));
                g->ws_busy = true;
                wk = g->ws.get();
            }
        }
        if (!wk) {
            own.reset(new Workspace(s));
            wk = own.get();
        }
        struct Release {
            bc_graph* g;
            bool shared;
            ~Release() {
                if (shared) {
                    std::lock_guard<std::mutex> lk(g->ws_mu);
                    g->ws_busy = false;
                }
            }
        } rel{g, own == nullptr};
        bc_status rs;
        if (W == 64) rs = run_ww<1>(g, kk, o, d_order, T, d_st, *wk, W, tm, s);
        else if (W == 128) rs = run_ww<2>(g, kk, o, d_order, T, d_st, *wk, W, tm, s);
        else rs = run_ww<4>(g, kk, o, d_order, T, d_st, *wk, W, tm, s);
        if (rs != BC_OK) {
            // a failed query may leave marks behind: never reuse its workspace
            std::lock_guard<std::mutex> lk(g->ws_mu);
            if (own == nullptr) g->ws.reset();
            return rs;
        }
        if (all) {
            BC_HIP(hipMemcpyAsync(all_f, allf.p, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToHost, s));
            BC_HIP(hipMemcpyAsync(all_r, allr.p, sizeof(uint32_t) * (size_t)n, hipMemcpyDeviceToHost, s));
        }
        int32_t cnt = 0;
        std::vector<Rec> recs(nrec);
        BC_HIP(hipMemcpyAsync(&cnt, T.cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        if (nrec) BC_HIP(hipMemcpyAsync(recs.data(), T.list, sizeof(Rec) * nrec, hipMemcpyDeviceToHost, s));
        BC_HIP(hipMemcpyAsync(&hst, d_st, sizeof(QStats), hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        if (all) {
            if (hst.n_done + hst.n_trivial != (unsigned long long)n) {
                set_error("internal: %llu of %d sources completed", hst.n_done + hst.n_trivial, n);
                return BC_EDEVICE;
            }
            cnt = 0;
        } else if (cnt != kk) {
            set_error("internal: top-k list holds %d of %d entries", cnt, kk);
            return BC_EDEVICE;
        }
        for (int32_t i = 0; i < cnt; ++i) {
            ids[i] = (int32_t)(uint32_t)(recs[i].idr & 0xFFFFFFFFu);
            reach[i] = (uint32_t)(recs[i].idr >> 32);
            farness[i] = recs[i].f;
        }
    }
    if (count) *count = all ? n : (kk > 0 ? kk : 0);
    auto t1 = std::chrono::steady_clock::now();
    if (st_out) {
        const uint32_t sz = st_out->size;
        bc_stats o2;
        std::memset(&o2, 0, sizeof(o2));
        o2.size = sizeof(bc_stats);
        o2.batches = (uint32_t)hst.batches;
        o2.m_vis = hst.m_vis;
        o2.node_arcs = hst.node_arcs;
        o2.levels = hst.levels;
        o2.pull_levels = hst.pull_levels;
        o2.n_cut = hst.n_cut;
        o2.n_done = hst.n_done;
        o2.n_trivial = hst.n_trivial;
        o2.preprocess_ms = g->preprocess_ms;
        o2.query_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        o2.seed_ms = tm.seed_ms;
        o2.persistent_ms = tm.persistent_ms;
        o2.frontier_entries = hst.frontier_entries;
        o2.discovered = hst.discovered;
        const bool pers = tm.persistent_ms > 0;
        o2.persistent_arcs = pers ? tm.persist_stats.node_arcs - tm.seed_stats.node_arcs : 0;
        o2.persistent_entries = pers ? tm.persist_stats.frontier_entries - tm.seed_stats.frontier_entries : 0;
        o2.persistent_discovered = pers ? tm.persist_stats.discovered - tm.seed_stats.discovered : 0;
        o2.defer_ms = tm.defer_ms;
        o2.n_deferred = hst.n_deferred;
        for (int i = 0; i < 5; ++i) o2.phase_ms[i] = (double)hst.phase_ticks[i] / 1e5;
        o2.lds_levels = hst.lds_levels;
        o2.record_levels = hst.record_levels;
        o2.spills = hst.spills;
        o2.record_ms = (double)hst.record_ticks / 1e5;
        o2.record_arcs = hst.record_arcs;
        std::memcpy(st_out, &o2, std::min<size_t>(sz ? sz : sizeof(bc_stats), sizeof(bc_stats)));
    }
    return BC_OK;
}

}  // namespace

// The order in which Algorithm 1 takes its sources (any order gives the
// same answer; Section 2.1): one of the BC_ORDER_* rules, written to
// d_order (n entries, a permutation).
bc_status build_order(bc_graph* g, const bc_opts& o, int32_t kk, int32_t* d_order, hipStream_t s) {
    const int32_t n = g->dg.n;
    const int W = o.width;
    int32_t ord = o.order == BC_ORDER_AUTO ? (o.mode == BC_MODE_BATCHED ? BC_ORDER_GROUPED : BC_ORDER_DEGREE)
                                            : o.order;
    // the order perceptron is trained on undirected graphs; on directed ones
    // the combined order falls back to the degree-based one
    if ((ord == BC_ORDER_LEARNED_GROUPED || ord == BC_ORDER_LEARNED_LOCALITY) && g->dg.directed) {
        if (!o.mlp) { set_error("learned orders need opts.mlp"); return BC_EINVAL; }
        ord = ord == BC_ORDER_LEARNED_GROUPED ? BC_ORDER_GROUPED : BC_ORDER_LOCALITY;
    }
    if (ord == BC_ORDER_DEGREE) {
        BC_TRY(order_by_degree(g, d_order, s));
    } else if (ord == BC_ORDER_GROUPED) {
        BC_TRY(order_grouped(g, d_order, s));
    } else if (ord == BC_ORDER_LOCALITY) {
        BC_TRY(order_locality(g, W, d_order, s));
    } else if (ord == BC_ORDER_GIVEN) {
        if (!o.perm) { set_error("BC_ORDER_GIVEN needs opts.perm"); return BC_EINVAL; }
        BC_TRY(order_given(g, o.perm, d_order, s));
    } else if (ord == BC_ORDER_SCORES) {
        if (!o.scores) { set_error("BC_ORDER_SCORES needs opts.scores"); return BC_EINVAL; }
        BC_TRY(order_by_scores(g, o.scores, false, d_order, s));
    } else if (ord == BC_ORDER_LEARNED || ord == BC_ORDER_LEARNED_GROUPED || ord == BC_ORDER_LEARNED_LOCALITY) {
        if (!o.mlp) { set_error("learned orders need opts.mlp"); return BC_EINVAL; }
        if (ord == BC_ORDER_LEARNED) {
            BC_TRY(order_learned(g, o.mlp, d_order, s));
        } else if (ord == BC_ORDER_LEARNED_LOCALITY) {
            // the k best-scored sources, then the locality order without them
            const SeedPlan sp = seed_plan(o, kk, n, W);
            const int64_t head =
                std::min<int64_t>((int64_t)n, std::min<int64_t>((int64_t)sp.batches * sp.sw, (int64_t)kk));
            DevBuf bys;
            BC_TRY(bys.alloc_on(sizeof(int32_t) * (size_t)(n > 0 ? n : 1), s));
            BC_TRY(order_learned(g, o.mlp, bys.as<int32_t>(), s));
            std::vector<int32_t> h((size_t)(head > 0 ? head : 1));
            if (head > 0) {
                BC_HIP(hipMemcpyAsync(h.data(), bys.p, sizeof(int32_t) * (size_t)head, hipMemcpyDeviceToHost, s));
                BC_HIP(hipStreamSynchronize(s));
            }
            BC_TRY(order_locality(g, W, d_order, s));
            if (head > 0) BC_TRY(order_front(g, h.data(), (int32_t)head, d_order, s, false));
        } else {
            const SeedPlan sp = seed_plan(o, kk, n, W);
            // the k best-scored sources first (the predicted top-k), then the
            // grouped order, which fills the rest of the seed batches with the
            // highest-degree nodes
            const int64_t head =
                std::min<int64_t>((int64_t)n, std::min<int64_t>((int64_t)sp.batches * sp.sw, (int64_t)kk));
            BC_TRY(order_learned_grouped(g, o.mlp, (int32_t)head, d_order, s));
        }
    } else {
        set_error("unknown order %d", o.order);
        return BC_EINVAL;
    }
    if (o.nfirst != 0) BC_TRY(order_front(g, o.first, o.nfirst, d_order, s));
    return BC_OK;
}

bc_status run_topk(bc_graph* g, int32_t k, const bc_opts& o, int32_t* ids, uint64_t* farness, uint32_t* reach,
                   int32_t* count, bc_stats* st, hipStream_t s, bool private_ws) {
    return run_query(g, k, o, ids, farness, reach, count, st, nullptr, nullptr, s, private_ws);
}

bc_status run_farness_all(bc_graph* g, const bc_opts& o, uint64_t* farness, uint32_t* reach, bc_stats* st,
                          hipStream_t s) {
    return run_query(g, 0, o, nullptr, nullptr, nullptr, nullptr, st, farness, reach, s, false);
}

// ------------------------------------------ top-k without any allocation
//
// One file-scope device array holds every buffer of a plain-mode query, so
// that bc_topk_static allocates nothing.  In host code `scratch` names a
// host-side stand-in; its device address is taken once per device with
// hipGetSymbolAddress, and only that address is ever passed to kernels or
// copies.

constexpr size_t kStaticBytes = (size_t)64 << 20;  // 64 MiB per device, held until the process ends
constexpr size_t kStaticHdr = 64;                   // list header: count, lock, sequence

}  // namespace bc

static __device__ __align__(256) unsigned char scratch[bc::kStaticBytes];

namespace bc {
namespace {

struct StaticScratch {
    std::mutex mu;        // serialises calls on one device (they share the array)
    void* ptr = nullptr;  // device address of `scratch` on this device
};
StaticScratch g_static[64];

size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

// Bytes of scratch a plain-mode query of W = 64 on n nodes with k results
// needs: control block, list, statistics, sources, threshold records, order,
// node records and the three node lists.
size_t static_need(int32_t n, int32_t kk) {
    const size_t N = (size_t)n;
    return al256(sizeof(Ctl)) + al256(kStaticHdr + sizeof(Rec) * (size_t)kk) + al256(sizeof(QStats)) +
           al256(sizeof(SrcState) * kBlk) + al256(sizeof(ThRec) * (N + 1)) + al256(sizeof(int32_t) * N) +
           al256(sizeof(uint64_t) * Layout<1>::SW * N) + 3 * al256(sizeof(int32_t) * N);
}

}  // namespace

bc_status run_topk_static(bc_graph* g, int32_t k, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* count) {
    int dev = 0;
    BC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("device %d out of range", dev);
        return BC_EDEVICE;
    }
    if (g->device != dev) {
        set_error("the graph lives on device %d, not the current %d", g->device, dev);
        return BC_EINVAL;
    }
    const int32_t n = g->dg.n;
    const int32_t kk = std::min(k, n);
    if (n == 0) {
        *count = 0;
        return BC_OK;
    }
    const size_t need = static_need(n, kk);
    if (need > kStaticBytes) {
        set_error("bc_topk_static: n = %d, k = %d needs %zu bytes of its static scratch, which holds %zu "
                  "(at most about %zu nodes)", n, k, need, kStaticBytes, (kStaticBytes - 65536) / 72);
        return BC_EINVAL;
    }
    StaticScratch& SS = g_static[dev];
    std::lock_guard<std::mutex> lk(SS.mu);
    if (!SS.ptr) BC_HIP(hipGetSymbolAddress(&SS.ptr, HIP_SYMBOL(scratch)));
    hipStream_t s = g->stream;
    const DevGraph& G = g->dg;
    char* base = static_cast<char*>(SS.ptr);
    size_t off = 0;
    auto take = [&](size_t b) {
        char* p = base + off;
        off += al256(b);
        return p;
    };
    Ctl* C = reinterpret_cast<Ctl*>(take(sizeof(Ctl)));
    char* hb = take(kStaticHdr + sizeof(Rec) * (size_t)kk);
    QStats* d_st = reinterpret_cast<QStats*>(take(sizeof(QStats)));
    SrcState* S = reinterpret_cast<SrcState*>(take(sizeof(SrcState) * kBlk));
    ThRec* ring = reinterpret_cast<ThRec*>(take(sizeof(ThRec) * ((size_t)n + 1)));
    int32_t* ord = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)n));
    SlotPtrs P;
    P.ns = reinterpret_cast<uint64_t*>(take(sizeof(uint64_t) * Layout<1>::SW * (size_t)n));
    P.qa = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)n));
    P.qb = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)n));
    P.clr = reinterpret_cast<int32_t*>(take(sizeof(int32_t) * (size_t)n));
    // every call starts from zeroed state (the array keeps the last call's
    // contents): control block, list header and records, statistics, node
    // records; then the degrees into the records' meta words
    const int cus = device_cus();
    auto zero = [&](void* p, size_t bytes) {
        const size_t words = al256(bytes) / 8;
        k_zero_words<<<clamp_grid((int64_t)words, 4 * cus), kBlk, 0, s>>>(static_cast<unsigned long long*>(p), words);
    };
    zero(C, sizeof(Ctl));
    zero(hb, kStaticHdr + sizeof(Rec) * (size_t)kk);
    zero(d_st, sizeof(QStats));
    zero(P.ns, sizeof(uint64_t) * Layout<1>::SW * (size_t)n);
    k_slot_init<1><<<clamp_grid((int64_t)n, 4096), kBlk, 0, s>>>(G.deg, n, P.ns, 1);
    // the graph's degree order when it holds one, else node-id order
    bool have_deg = false;
    {
        std::lock_guard<std::mutex> ck(g->cache_mu);
        have_deg = g->have_order_deg;
    }
    if (have_deg)
        BC_HIP(hipMemcpyAsync(ord, g->order_deg.p, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s));
    else
        k_iota<<<clamp_grid((int64_t)n, 4096), kBlk, 0, s>>>(ord, n);
    TopKDev T;
    T.k = kk;
    T.cnt = reinterpret_cast<int32_t*>(hb);
    T.lock = reinterpret_cast<uint32_t*>(hb + 4);
    T.seq = reinterpret_cast<uint32_t*>(hb + 8);
    T.list = reinterpret_cast<Rec*>(hb + kStaticHdr);
    T.ring = ring;
    T.all_f = nullptr;
    T.all_r = nullptr;
    T.footnote = 0;
    LevelParams lp{3.f, 24.f, 1};
    constexpr int W = 64;
    const uint32_t nb = (uint32_t)((n + W - 1) / W);
    uint32_t hctl[16];  // control block words: d, flen, nlen, clen, live, pull, ..., front_arcs at 10
    for (uint32_t b = 0; b < nb; ++b) {
        k_plain_init<1><<<1, kBlk, 0, s>>>(G, ord, n, b, W, P, S, C, T, d_st);
        for (;;) {
            BC_HIP(hipMemcpyAsync(hctl, C, sizeof(hctl), hipMemcpyDeviceToHost, s));
            BC_HIP(hipStreamSynchronize(s));
            const uint32_t flen = hctl[1], live = hctl[4], pull = hctl[5];
            if (flen > (uint32_t)n || hctl[2] > (uint32_t)n || hctl[3] > (uint32_t)n) {
                set_error("internal: level %u list lengths %u/%u/%u exceed n = %d", hctl[0], flen, hctl[2], hctl[3], n);
                return BC_EDEVICE;
            }
            unsigned long long fa;
            std::memcpy(&fa, hctl + 10, sizeof(fa));
            if (!live) break;
            if (pull) {
                k_plain_pull<1><<<clamp_grid(n, 8 * cus), kBlk, 0, s>>>(G, P, S, C, T, d_st, W, 0);
            } else {
                const int64_t chunks = ((int64_t)flen + expand_chunk(flen, fa) - 1) / expand_chunk(flen, fa);
                k_plain_expand<1><<<clamp_grid(chunks * kBlk, 8 * cus), kBlk, 0, s>>>(G, P, C, d_st, 0);
                k_plain_count<1><<<clamp_grid((int64_t)std::min<unsigned long long>(fa, (unsigned long long)n), 4 * cus),
                                   kBlk, 0, s>>>(P, S, C, T, d_st, W, 0);
            }
            k_plain_clearcur<1><<<clamp_grid(flen, 4 * cus), kBlk, 0, s>>>(P, C, 0);
            const int64_t bound = pull ? (int64_t)n : (int64_t)std::min<unsigned long long>(fa, (unsigned long long)n);
            k_plain_build<1><<<clamp_grid(bound, 4 * cus), kBlk, 0, s>>>(G, P, C, lp, 0);
        }
        k_plain_clear<1><<<clamp_grid(n, 4 * cus), kBlk, 0, s>>>(P, C);
    }
    BC_HIP(hipGetLastError());
    int32_t cnt = 0;
    BC_HIP(hipMemcpyAsync(&cnt, T.cnt, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));
    if (cnt != kk) {
        set_error("internal: top-k list holds %d of %d entries", cnt, kk);
        return BC_EDEVICE;
    }
    // results in chunks through a fixed host buffer on the stack
    Rec chunk[64];
    for (int32_t i0 = 0; i0 < cnt; i0 += 64) {
        const int32_t m = std::min(64, cnt - i0);
        BC_HIP(hipMemcpyAsync(chunk, T.list + i0, sizeof(Rec) * (size_t)m, hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        for (int32_t i = 0; i < m; ++i) {
            ids[i0 + i] = (int32_t)(uint32_t)(chunk[i].idr & 0xFFFFFFFFu);
            reach[i0 + i] = (uint32_t)(chunk[i].idr >> 32);
            farness[i0 + i] = chunk[i].f;
        }
    }
    *count = cnt;
    return BC_OK;
}

// ------------------------------------------------ many graphs, one launch

namespace {

// Per-query state of a job launch, one block per query in one buffer that a
// single fill kernel clears before every run: list header (count, lock,
// sequence), k list records, statistics, the two job counters.
constexpr size_t kHdr = 64;
size_t query_state_bytes(int32_t kk) {
    const size_t b = kHdr + sizeof(Rec) * (size_t)kk + sizeof(QStats) + 16;
    return (b + 255) & ~(size_t)255;
}

// bc_stats of one query of a job launch (every batch ran in the persistent kernel).
void multi_stats(const QStats& h, double preprocess_ms, double query_ms, double launch_ms, bc_stats* out) {
    const uint32_t sz = out->size;
    bc_stats o2;
    std::memset(&o2, 0, sizeof(o2));
    o2.size = sizeof(bc_stats);
    o2.batches = (uint32_t)h.batches;
    o2.m_vis = h.m_vis;
    o2.node_arcs = h.node_arcs;
    o2.levels = h.levels;
    o2.n_cut = h.n_cut;
    o2.n_done = h.n_done;
    o2.n_trivial = h.n_trivial;
    o2.preprocess_ms = preprocess_ms;
    o2.query_ms = query_ms;
    o2.persistent_ms = launch_ms;
    o2.frontier_entries = h.frontier_entries;
    o2.discovered = h.discovered;
    o2.persistent_arcs = h.node_arcs;
    o2.persistent_entries = h.frontier_entries;
    o2.persistent_discovered = h.discovered;
    for (int i = 0; i < 5; ++i) o2.phase_ms[i] = (double)h.phase_ticks[i] / 1e5;
    std::memcpy(out, &o2, std::min<size_t>(sz ? sz : sizeof(bc_stats), sizeof(bc_stats)));
}

}  // namespace

}  // namespace bc

// A prepared job launch over a fixed set of queries (graph, k): orders,
// per-query state, the descriptor table and shared node-record slots, and
// (when captured) the HIP graph that clears the state and runs the launch.
struct bc_multi {
    int W = 64;
    int32_t count = 0;
    std::vector<bc_graph*> graphs;
    std::vector<int32_t> kk;            // min(k, n) per query
    std::vector<int32_t> kreq;          // k per query (output offsets are sums of these)
    std::vector<size_t> state_off;      // offset of each query's state block
    hipStream_t s = nullptr;            // stream of the runs
    hipStream_t cap = nullptr;          // private capture stream
    bc::DevBuf orders, rings, state, jobs, ctl;
    bc::DevBuf ns, qa, qb, clr, stamps;
    int slots = 0;
    int32_t ncap = 0;
    size_t state_bytes = 0;
    unsigned long long nbatch = 0;      // published batches of the launch
    uint32_t njobs = 0;
    bool captured = false;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    ~bc_multi() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (s) (void)hipStreamSynchronize(s);
        if (cap) (void)hipStreamDestroy(cap);
    }
};

namespace bc {

namespace {

template <int WW>
void launch_jobs(bc_multi* p, hipStream_t st) {
    const size_t words = p->state_bytes / 8;
    k_zero_words<<<clamp_grid((int64_t)words, 1024), kBlk, 0, st>>>(p->state.as<unsigned long long>(), words);
    k_zero_words<<<1, 64, 0, st>>>(p->ctl.as<unsigned long long>(), 1);  // the claim counter
    JobLaunch L;
    L.jobs = p->jobs.as<JobDesc>();
    L.njobs = p->njobs;
    L.idle_ticks = 0;  // every batch is published before the launch: end when none is left
    L.idle_cap = 0;
    L.published = p->ctl.as<unsigned long long>() + 1;
    L.stop = nullptr;
    L.running = nullptr;
    L.last_end = nullptr;
    L.claim = p->ctl.as<unsigned long long>();
    L.W = p->W;
    L.ncap = p->ncap;
    SlotPtrs base{p->ns.as<uint64_t>(), p->qa.as<int32_t>(), p->qb.as<int32_t>(), p->clr.as<int32_t>()};
    k_jobs<WW, kBatchBlk><<<p->slots, kBatchBlk, 0, st>>>(L, base, p->stamps.as<uint32_t>());
}

void launch_jobs_any(bc_multi* p, hipStream_t st) {
    if (p->W == 64) launch_jobs<1>(p, st);
    else if (p->W == 128) launch_jobs<2>(p, st);
    else launch_jobs<4>(p, st);
}

}  // namespace

bc_status multi_create(bc_graph* const* graphs, int32_t count, const int32_t* ks, const bc_opts& o, hipStream_t s,
                       bool capture, bc_multi** out) {
    *out = nullptr;
    const int W = o.width;
    if (W != 64 && W != 128 && W != 256) {
        set_error("width must be 64, 128 or 256 (got %d)", W);
        return BC_EINVAL;
    }
    int dev = 0;
    BC_HIP(hipGetDevice(&dev));
    std::unique_ptr<bc_multi> p(new bc_multi());
    p->W = W;
    p->count = count;
    p->s = s;
    p->graphs.assign(graphs, graphs + count);
    p->kk.resize((size_t)count);
    p->kreq.assign(ks, ks + count);
    p->state_off.resize((size_t)count);
    const int SW = W == 64 ? Layout<1>::SW : (W == 128 ? Layout<2>::SW : Layout<4>::SW);
    size_t ord_total = 0, ring_total = 0;
    std::vector<size_t> ord_off((size_t)count), ring_off((size_t)count);
    for (int32_t i = 0; i < count; ++i) {
        bc_graph* g = graphs[i];
        if (!g) { set_error("graph %d is NULL", i); return BC_EINVAL; }
        if (g->device != dev) { set_error("graph %d lives on device %d, not the current %d", i, g->device, dev); return BC_EINVAL; }
        if (ks[i] <= 0) { set_error("k of query %d must be positive (got %d)", i, ks[i]); return BC_EINVAL; }
        const int32_t n = g->dg.n;
        p->kk[(size_t)i] = std::min(ks[i], n);
        p->ncap = std::max(p->ncap, n);
        p->state_off[(size_t)i] = p->state_bytes;
        p->state_bytes += query_state_bytes(p->kk[(size_t)i]);
        ord_off[(size_t)i] = ord_total;
        ring_off[(size_t)i] = ring_total;
        ord_total += (size_t)n;
        ring_total += (size_t)n + 1;
    }
    if (p->state_bytes == 0) p->state_bytes = 256;
    BC_TRY(p->orders.alloc_on(sizeof(int32_t) * std::max<size_t>(ord_total, 1), s));
    BC_TRY(p->rings.alloc_on(sizeof(ThRec) * std::max<size_t>(ring_total, 1), s));
    BC_TRY(p->state.alloc_on(p->state_bytes, s));
    BC_TRY(p->ctl.alloc_on(64, s));
    BC_HIP(hipMemsetAsync(p->state.p, 0, p->state_bytes, s));
    BC_HIP(hipMemsetAsync(p->ctl.p, 0, 64, s));
    // source orders (each graph's own rule, as bc_topk in batched mode)
    bc_opts ob = o;
    ob.mode = BC_MODE_BATCHED;
    ob.nfirst = 0;
    ob.first = nullptr;
    for (int32_t i = 0; i < count; ++i)
        if (p->kk[(size_t)i] > 0)
            BC_TRY(build_order(graphs[i], ob, p->kk[(size_t)i], p->orders.as<int32_t>() + ord_off[(size_t)i], s));
    // descriptors: the seed batches of every query first, then the rest of
    // each query, the most arcs first (the longest work starts earliest)
    std::vector<JobDesc> jd;
    std::vector<int32_t> rest;
    unsigned long long pos = 0;
    char* sb = p->state.as<char>();
    auto fill = [&](int32_t i, uint32_t bofs, uint32_t cnt) {
        bc_graph* g = graphs[i];
        const int32_t kq = p->kk[(size_t)i];
        const uint32_t nb = (uint32_t)((g->dg.n + W - 1) / W);
        char* q = sb + p->state_off[(size_t)i];
        JobDesc d;
        std::memset(&d, 0, sizeof(d));
        d.G = g->dg;
        d.order = p->orders.as<int32_t>() + ord_off[(size_t)i];
        d.T.k = kq;
        d.T.cnt = (int32_t*)q;
        d.T.lock = (uint32_t*)(q + 4);
        d.T.seq = (uint32_t*)(q + 8);
        d.T.list = (Rec*)(q + kHdr);
        d.T.ring = p->rings.as<ThRec>() + ring_off[(size_t)i];
        d.T.all_f = nullptr;
        d.T.all_r = nullptr;
        d.T.footnote = (!g->dg.directed && (o.bounds & BC_BOUND_FOOTNOTE)) ? 1 : 0;
        d.st = (QStats*)(q + kHdr + sizeof(Rec) * (size_t)kq);
        d.ctr = (uint32_t*)(q + kHdr + sizeof(Rec) * (size_t)kq + sizeof(QStats));
        d.range = pack_range(pos, cnt);
        d.bofs = bofs;
        d.total = nb;
        d.seed = std::min<uint32_t>(nb, (uint32_t)((kq + W - 1) / W));
        d.out = nullptr;
        d.out_st = nullptr;
        d.done = nullptr;
        d.seeded = nullptr;
        d.progress = nullptr;
        jd.push_back(d);
        pos += cnt;
    };
    for (int32_t i = 0; i < count; ++i) {
        if (p->kk[(size_t)i] <= 0) continue;
        const uint32_t nb = (uint32_t)((graphs[i]->dg.n + W - 1) / W);
        const uint32_t sd = std::min<uint32_t>(nb, (uint32_t)((p->kk[(size_t)i] + W - 1) / W));
        fill(i, 0, sd);
        if (sd < nb) rest.push_back(i);
    }
    std::stable_sort(rest.begin(), rest.end(), [&](int32_t a, int32_t b) { return graphs[a]->dg.m > graphs[b]->dg.m; });
    for (int32_t i : rest) {
        const uint32_t nb = (uint32_t)((graphs[i]->dg.n + W - 1) / W);
        const uint32_t sd = std::min<uint32_t>(nb, (uint32_t)((p->kk[(size_t)i] + W - 1) / W));
        fill(i, sd, nb - sd);
    }
    p->nbatch = pos;
    p->njobs = (uint32_t)jd.size();
    BC_TRY(p->jobs.alloc_on(sizeof(JobDesc) * std::max<size_t>(jd.size(), 1), s));
    if (!jd.empty())
        BC_HIP(hipMemcpyAsync(p->jobs.p, jd.data(), sizeof(JobDesc) * jd.size(), hipMemcpyHostToDevice, s));
    BC_HIP(hipMemcpyAsync(p->ctl.as<unsigned long long>() + 1, &p->nbatch, sizeof(unsigned long long),
                          hipMemcpyHostToDevice, s));
    // shared node-record slots for the largest graph, all zero at rest
    int slots = o.slots > 0 ? o.slots : device_cus();
    if ((unsigned long long)slots > p->nbatch) slots = (int)std::max<unsigned long long>(p->nbatch, 1);
    const size_t N = (size_t)std::max(p->ncap, 1);
    const size_t per_slot = N * (8 * (size_t)SW + 12);
    size_t freeb = 0, totalb = 0;
    if (hipMemGetInfo(&freeb, &totalb) == hipSuccess) {
        const size_t capn = (size_t)(0.45 * (double)freeb) / per_slot;
        if ((size_t)slots > capn) slots = (int)std::max<size_t>(capn, 1);
    }
    p->slots = slots;
    BC_TRY(p->ns.alloc_on(sizeof(uint64_t) * N * SW * (size_t)slots, s));
    BC_TRY(p->qa.alloc_on(sizeof(int32_t) * N * (size_t)slots, s));
    BC_TRY(p->qb.alloc_on(sizeof(int32_t) * N * (size_t)slots, s));
    BC_TRY(p->clr.alloc_on(sizeof(int32_t) * N * (size_t)slots, s));
    BC_TRY(p->stamps.alloc_on(sizeof(uint32_t) * (size_t)slots, s));
    BC_HIP(hipMemsetAsync(p->ns.p, 0, sizeof(uint64_t) * N * SW * (size_t)slots, s));
    BC_HIP(hipMemsetAsync(p->stamps.p, 0, sizeof(uint32_t) * (size_t)slots, s));
    BC_HIP(hipStreamSynchronize(s));
    if (capture && p->nbatch > 0) {
        BC_HIP(hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking));  // default priority
        BC_HIP(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
        launch_jobs_any(p.get(), p->cap);
        const hipError_t ce = hipStreamEndCapture(p->cap, &p->graph);
        BC_HIP(ce);
        BC_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
        p->captured = true;
    }
    *out = p.release();
    return BC_OK;
}

bc_status multi_run(bc_multi* p, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* counts, bc_stats* stats) {
    auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = p->s;
    double launch_ms = 0;
    std::vector<char> hs(p->state_bytes);
    if (p->nbatch > 0) {
        EventPair ev;
        BC_TRY(ev.create());
        BC_HIP(hipEventRecord(ev.a, s));
        if (p->captured) BC_HIP(hipGraphLaunch(p->exec, s));
        else launch_jobs_any(p, s);
        BC_HIP(hipEventRecord(ev.b, s));
        BC_HIP(hipGetLastError());
        BC_TRY(ev.ms(&launch_ms));
        BC_HIP(hipMemcpyAsync(hs.data(), p->state.p, p->state_bytes, hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
    }
    const double qms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    size_t off = 0;
    for (int32_t i = 0; i < p->count; ++i) {
        const int32_t kq = p->kk[(size_t)i];
        const char* q = hs.data() + p->state_off[(size_t)i];
        int32_t cnt = 0;
        QStats h;
        std::memset(&h, 0, sizeof(h));
        if (kq > 0) {
            std::memcpy(&cnt, q, sizeof(int32_t));
            std::memcpy(&h, q + kHdr + sizeof(Rec) * (size_t)kq, sizeof(QStats));
            if (cnt != kq) {
                set_error("internal: query %d top-k list holds %d of %d entries", i, cnt, kq);
                return BC_EDEVICE;
            }
            for (int32_t j = 0; j < cnt; ++j) {
                Rec r;
                std::memcpy(&r, q + kHdr + sizeof(Rec) * (size_t)j, sizeof(Rec));
                ids[off + (size_t)j] = (int32_t)(uint32_t)(r.idr & 0xFFFFFFFFu);
                reach[off + (size_t)j] = (uint32_t)(r.idr >> 32);
                farness[off + (size_t)j] = r.f;
            }
        }
        counts[i] = cnt;
        if (stats) multi_stats(h, p->graphs[(size_t)i]->preprocess_ms, qms, launch_ms, &stats[i]);
        off += (size_t)p->kreq[(size_t)i];
    }
    return BC_OK;
}

void multi_destroy(bc_multi* p) { delete p; }

// ------------------------------------------- serving queue of a running kernel
//
// A device-visible queue of top-k requests that a persistent job kernel
// drains while it runs: the host writes a request's descriptor into a ring in
// pinned host memory and raises the published batch total; workgroups that
// finish a batch claim the next published one, whichever request it belongs
// to, so a request that arrives while others are on the GPU starts as soon
// as a workgroup is free, and its batches run beside theirs.  The last batch
// of a request copies its list and statistics to the ring slot's result area
// (pinned host memory) and raises its done flag; the host polls the flags.
// The kernel ends after a bounded idle time with nothing to claim, or once
// its batches end after it is told to stop: at shutdown, or to let a lane's
// own device work that waits behind it run (kQueueYield).  The host launches
// it again when work is waiting.

struct QueueJob {
    int slot = -1;          // ring slot of the seed range (its done and seeded flags, its counters)
    int slot2 = -1;         // ring slot of the rest, published once the seed batches have finished
    bool rest_pending = false;
    uint32_t nb = 0, seed = 0;
    int32_t kk = 0;
    int32_t footnote = 0;
    bc_graph* g = nullptr;
    DevBuf order, ring, state;
};

struct DevQueue {
    int W = 64;
    int32_t ncap = 0;
    int slots = 0;
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    bool launched = false;
    char* host = nullptr;            // pinned: descriptors, results, statistics, flags, totals
    JobDesc* ring = nullptr;
    Rec* out = nullptr;
    unsigned long long* out_st = nullptr;
    uint32_t* done = nullptr;
    uint32_t* seeded = nullptr;
    uint32_t* progress = nullptr;
    unsigned long long* published = nullptr;
    uint32_t* stop = nullptr;
    char* dhost = nullptr;           // the same block as the device addresses it
    unsigned long long launches = 0;
    int waiters = 0;                 // lanes waiting for device work of their own (atomic builtins)
    long long wait_since = 0;        // steady-clock ns when the count last left zero (atomic builtins)
    bool yielding = false;           // stop raised to let a launch end for a waiting lane
    std::chrono::steady_clock::time_point t_launch{};
    DevBuf ctr, claim, ns, qa, qb, clr, stamps;
    std::mutex mu;
    std::condition_variable cv;
    std::vector<char> busy;
    unsigned long long total = 0;    // batches published so far
    ~DevQueue() {
        if (stream) (void)hipStreamSynchronize(stream);
        if (ev) (void)hipEventDestroy(ev);
        if (host) (void)hipHostFree(host);
        ns.release();
        qa.release();
        qb.release();
        clr.release();
        stamps.release();
        ctr.release();
        claim.release();
        if (stream) (void)hipStreamDestroy(stream);
    }
};

namespace {

// A serving kernel's workgroups wait for work while a batch of the launch
// runs or has just ended: one that left then would leave the batches
// published next (a request's rest, once its seed batches are done) to
// fewer workgroups until the whole launch ended.  With no batch running for
// a few milliseconds and nothing to claim they leave, so that the launch ends
// and the device is free for other work (a request's preparation on another
// stream may wait for that); the cap bounds the wait for a long batch.
constexpr uint64_t kQueueIdleTicks = 500000;        // 5 ms (100 MHz)
constexpr uint64_t kQueueIdleCap = 12000000000ull;  // 120 s idle in any case

size_t queue_host_bytes() {
    return sizeof(JobDesc) * kQueueCap + sizeof(Rec) * (size_t)kQueueCap * kQueueMaxK +
           sizeof(QStats) * kQueueCap + 3 * sizeof(uint32_t) * kQueueCap + 128;
}

template <class T>
T* dev_view(const DevQueue* q, T* host_ptr) {
    return reinterpret_cast<T*>(q->dhost + (reinterpret_cast<char*>(host_ptr) - q->host));
}

template <int WW>
void launch_queue(DevQueue* q) {
    JobLaunch L;
    L.jobs = reinterpret_cast<const JobDesc*>(q->dhost);
    L.njobs = kQueueCap;
    L.idle_ticks = kQueueIdleTicks;
    L.idle_cap = kQueueIdleCap;
    L.published = reinterpret_cast<const unsigned long long*>(q->dhost + ((char*)q->published - q->host));
    L.stop = reinterpret_cast<const uint32_t*>(q->dhost + ((char*)q->stop - q->host));
    L.claim = q->claim.as<unsigned long long>();
    L.running = reinterpret_cast<uint32_t*>(q->claim.as<char>() + 8);
    L.last_end = reinterpret_cast<unsigned long long*>(q->claim.as<char>() + 16);
    L.W = q->W;
    L.ncap = q->ncap;
    SlotPtrs base{q->ns.as<uint64_t>(), q->qa.as<int32_t>(), q->qb.as<int32_t>(), q->clr.as<int32_t>()};
    k_jobs<WW, kBatchBlk><<<q->slots, kBatchBlk, 0, q->stream>>>(L, base, q->stamps.as<uint32_t>());
}

// A lane's own device work (an upload, a source order, a whole-request
// query) goes to its stream, which may share a hardware queue with the
// running launch and then waits until that launch ends.  Once a lane has
// waited this long, and the launch has run at least as long, the launch is
// told to stop claiming (its workgroups finish their batches and leave) and
// is started again afterwards.
constexpr auto kQueueYield = std::chrono::milliseconds(2);

static long long steady_ns() {
    return (long long)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Launch the kernel when work is published and no launch is running
// (caller holds q->mu).  A running launch keeps its workgroups while a
// batch of it runs and ends a few milliseconds after the last one, or
// yields to a waiting lane.
bc_status pump_locked(DevQueue* q) {
    if (q->launched) {
        const hipError_t e = hipEventQuery(q->ev);
        if (e == hipErrorNotReady) {
            const long long yield_ns = std::chrono::nanoseconds(kQueueYield).count();
            if (!q->yielding && __atomic_load_n(&q->waiters, __ATOMIC_ACQUIRE) > 0 &&
                steady_ns() - __atomic_load_n(&q->wait_since, __ATOMIC_ACQUIRE) > yield_ns &&
                std::chrono::steady_clock::now() - q->t_launch > kQueueYield) {
                __atomic_store_n(q->stop, 1u, __ATOMIC_RELEASE);
                q->yielding = true;
            }
            return BC_OK;
        }
        BC_HIP(e);
        q->launched = false;
        if (q->yielding) {
            // the launch has ended: published batches not yet claimed go to the next one
            __atomic_store_n(q->stop, 0u, __ATOMIC_RELEASE);
            q->yielding = false;
        }
    }
    bool pending = false;
    for (int i = 0; i < kQueueCap && !pending; ++i) pending = q->busy[(size_t)i] != 0;
    if (!pending) return BC_OK;
    if (q->W == 64) launch_queue<1>(q);
    else if (q->W == 128) launch_queue<2>(q);
    else launch_queue<4>(q);
    BC_HIP(hipGetLastError());
    BC_HIP(hipEventRecord(q->ev, q->stream));
    q->launched = true;
    q->t_launch = std::chrono::steady_clock::now();
    ++q->launches;
    return BC_OK;
}

// Write a descriptor into a ring slot and make its batches claimable
// (caller holds q->mu).
void publish_locked(DevQueue* q, int slot, JobDesc d, uint32_t count) {
    // the slot is free, so its range is 0 and no workgroup takes it while the
    // other fields change; the range comes last, then the total that makes
    // the range's batches claimable
    d.range = 0;
    std::memcpy(&q->ring[slot], &d, sizeof(d));
    __atomic_store_n(&q->ring[slot].range, pack_range(q->total, count), __ATOMIC_RELEASE);
    q->total += count;
    __atomic_store_n(q->published, q->total, __ATOMIC_RELEASE);
}

// Take a finished query's range out of its slot (caller holds q->mu): a
// free slot matches no batch while a later request rewrites it.
void clear_slot_locked(DevQueue* q, int slot) {
    if (slot >= 0) __atomic_store_n(&q->ring[slot].range, 0ull, __ATOMIC_RELEASE);
}

JobDesc job_desc(const DevQueue* q, const QueueJob* j, uint32_t bofs) {
    const bc_graph* g = j->g;
    char* st = j->state.as<char>();
    JobDesc d;
    std::memset(&d, 0, sizeof(d));
    d.G = g->dg;
    d.order = j->order.as<int32_t>();
    d.T.k = j->kk;
    d.T.cnt = (int32_t*)st;
    d.T.lock = (uint32_t*)(st + 4);
    d.T.seq = (uint32_t*)(st + 8);
    d.T.list = (Rec*)(st + kHdr);
    d.T.ring = j->ring.as<ThRec>();
    d.T.footnote = j->footnote;
    d.st = (QStats*)(st + kHdr + sizeof(Rec) * (size_t)j->kk);
    d.ctr = q->ctr.as<uint32_t>() + 2 * j->slot;
    d.bofs = bofs;
    d.total = j->nb;
    d.seed = j->seed;
    d.out = dev_view(q, q->out + (size_t)j->slot * kQueueMaxK);
    d.out_st = dev_view(q, q->out_st + (size_t)j->slot * (sizeof(QStats) / 8));
    d.done = dev_view(q, q->done + j->slot);
    d.seeded = dev_view(q, q->seeded + j->slot);
    d.progress = dev_view(q, q->progress + j->slot);
    return d;
}

}  // namespace

bc_status devq_create(int W, int32_t ncap, int slots, DevQueue** out, uint64_t* device_bytes) {
    *out = nullptr;
    if (W != 64 && W != 128 && W != 256) {
        set_error("queue width must be 64, 128 or 256 (got %d)", W);
        return BC_EINVAL;
    }
    std::unique_ptr<DevQueue> q(new DevQueue());
    q->W = W;
    q->ncap = std::max(ncap, 1);
    q->slots = slots > 0 ? slots : device_cus();
    q->busy.assign(kQueueCap, 0);
    BC_HIP(hipStreamCreateWithFlags(&q->stream, hipStreamNonBlocking));  // default priority
    BC_HIP(hipEventCreateWithFlags(&q->ev, hipEventDisableTiming));
    const size_t hb = queue_host_bytes();
    BC_HIP(hipHostMalloc((void**)&q->host, hb, hipHostMallocCoherent | hipHostMallocMapped));
    std::memset(q->host, 0, hb);
    char* h = q->host;
    q->ring = reinterpret_cast<JobDesc*>(h);
    h += sizeof(JobDesc) * kQueueCap;
    q->out = reinterpret_cast<Rec*>(h);
    h += sizeof(Rec) * (size_t)kQueueCap * kQueueMaxK;
    q->out_st = reinterpret_cast<unsigned long long*>(h);
    h += sizeof(QStats) * kQueueCap;
    q->done = reinterpret_cast<uint32_t*>(h);
    h += sizeof(uint32_t) * kQueueCap;
    q->seeded = reinterpret_cast<uint32_t*>(h);
    h += sizeof(uint32_t) * kQueueCap;
    q->progress = reinterpret_cast<uint32_t*>(h);
    h += sizeof(uint32_t) * kQueueCap;
    q->published = reinterpret_cast<unsigned long long*>(h);
    q->stop = reinterpret_cast<uint32_t*>(h + 8);
    void* dp = nullptr;
    BC_HIP(hipHostGetDevicePointer(&dp, q->host, 0));
    q->dhost = reinterpret_cast<char*>(dp);
    const int SW = W == 64 ? Layout<1>::SW : (W == 128 ? Layout<2>::SW : Layout<4>::SW);
    const size_t N = (size_t)q->ncap, S_ = (size_t)q->slots;
    BC_TRY(q->ctr.alloc(sizeof(uint32_t) * 2 * kQueueCap));
    BC_TRY(q->claim.alloc(64));
    BC_TRY(q->ns.alloc(sizeof(uint64_t) * N * SW * S_));
    BC_TRY(q->qa.alloc(sizeof(int32_t) * N * S_));
    BC_TRY(q->qb.alloc(sizeof(int32_t) * N * S_));
    BC_TRY(q->clr.alloc(sizeof(int32_t) * N * S_));
    BC_TRY(q->stamps.alloc(sizeof(uint32_t) * S_));
    BC_HIP(hipMemsetAsync(q->ctr.p, 0, q->ctr.bytes, q->stream));
    BC_HIP(hipMemsetAsync(q->claim.p, 0, q->claim.bytes, q->stream));
    BC_HIP(hipMemsetAsync(q->ns.p, 0, q->ns.bytes, q->stream));
    BC_HIP(hipMemsetAsync(q->stamps.p, 0, q->stamps.bytes, q->stream));
    BC_HIP(hipStreamSynchronize(q->stream));
    if (device_bytes)
        *device_bytes = q->ns.bytes + q->qa.bytes + q->qb.bytes + q->clr.bytes + q->stamps.bytes + q->ctr.bytes + 64;
    *out = q.release();
    return BC_OK;
}

void devq_wait_begin(DevQueue* q) {
    if (q && __atomic_fetch_add(&q->waiters, 1, __ATOMIC_ACQ_REL) == 0)
        __atomic_store_n(&q->wait_since, steady_ns(), __ATOMIC_RELEASE);
}
void devq_wait_end(DevQueue* q) {
    if (q) __atomic_fetch_sub(&q->waiters, 1, __ATOMIC_ACQ_REL);
}

void devq_destroy(DevQueue* q) {
    if (!q) return;
    __atomic_store_n(q->stop, 1u, __ATOMIC_RELEASE);
    delete q;  // synchronises the queue stream: the kernel ends at its next claim
}

int devq_width(const DevQueue* q) { return q->W; }
int32_t devq_ncap(const DevQueue* q) { return q->ncap; }

bc_status devq_submit(DevQueue* q, bc_graph* g, int32_t k, const bc_opts& o_in, hipStream_t prep, QueueJob** out) {
    *out = nullptr;
    const int32_t n = g->dg.n;
    if (n <= 0 || n > q->ncap || k > kQueueMaxK || k <= 0) {
        set_error("request does not fit the queue (n %d of %d, k %d of %d)", n, q->ncap, k, kQueueMaxK);
        return BC_EINVAL;
    }
    const int W = q->W;
    std::unique_ptr<QueueJob> j(new QueueJob());
    j->g = g;
    j->kk = std::min(k, n);
    j->footnote = (!g->dg.directed && (o_in.bounds & BC_BOUND_FOOTNOTE)) ? 1 : 0;
    bc_opts o = o_in;
    o.mode = BC_MODE_BATCHED;
    o.width = W;
    const size_t sbytes = query_state_bytes(std::max(j->kk, 0));
    BC_TRY(j->order.alloc_on(sizeof(int32_t) * (size_t)std::max(n, 1), prep));
    BC_TRY(j->ring.alloc_on(sizeof(ThRec) * ((size_t)n + 1), prep));
    BC_TRY(j->state.alloc_on(sbytes, prep));
    BC_HIP(hipMemsetAsync(j->state.p, 0, sbytes, prep));
    {
        // the order is device work on the lane's stream (see kQueueYield)
        DevqWait wait(q);
        bc_status rs = BC_OK;
        if (j->kk > 0) rs = build_order(g, o, j->kk, j->order.as<int32_t>(), prep);
        const hipError_t se = hipStreamSynchronize(prep);  // drained on failure too
        BC_TRY(rs);
        BC_HIP(se);
    }
    j->nb = (uint32_t)((n + W - 1) / W);
    j->seed = std::min<uint32_t>(j->nb, (uint32_t)((j->kk + W - 1) / W));
    j->rest_pending = j->seed < j->nb;
    const int need = j->rest_pending ? 2 : 1;
    std::unique_lock<std::mutex> lk(q->mu);
    // free ring slots: one for the seed batches, one for the rest
    int got = 0;
    int sl[2] = {-1, -1};
    q->cv.wait(lk, [&] {
        got = 0;
        for (int i = 0; i < kQueueCap && got < need; ++i)
            if (!q->busy[(size_t)i]) sl[got++] = i;
        return got == need;
    });
    j->slot = sl[0];
    j->slot2 = sl[1];
    for (int i = 0; i < need; ++i) q->busy[(size_t)sl[i]] = 1;
    __atomic_store_n(&q->done[j->slot], 0u, __ATOMIC_RELAXED);
    __atomic_store_n(&q->seeded[j->slot], 0u, __ATOMIC_RELAXED);
    __atomic_store_n(&q->progress[j->slot], 0u, __ATOMIC_RELAXED);
    // the seed batches first: the rest is published when they have finished,
    // so that every later batch starts with a k-th best record and the
    // workgroups meanwhile take other requests' batches
    publish_locked(q, j->slot, job_desc(q, j.get(), 0), j->seed);
    BC_TRY(pump_locked(q));
    *out = j.release();
    return BC_OK;
}

bool devq_advance(DevQueue* q, QueueJob* j) {
    if (!j->rest_pending || __atomic_load_n(&q->seeded[j->slot], __ATOMIC_ACQUIRE) == 0u) return false;
    std::lock_guard<std::mutex> lk(q->mu);
    publish_locked(q, j->slot2, job_desc(q, j, j->seed), j->nb - j->seed);
    j->rest_pending = false;
    (void)pump_locked(q);
    return true;
}

unsigned long long devq_launches(DevQueue* q) {
    std::lock_guard<std::mutex> lk(q->mu);
    return q->launches;
}

unsigned long long devq_published(DevQueue* q) {
    std::lock_guard<std::mutex> lk(q->mu);
    return q->total;
}

void devq_progress(DevQueue* q, const QueueJob* j, uint64_t* done, uint64_t* total) {
    *done = __atomic_load_n(&q->progress[j->slot], __ATOMIC_RELAXED);
    *total = j->nb;
}

bool devq_done(DevQueue* q, const QueueJob* j) { return __atomic_load_n(&q->done[j->slot], __ATOMIC_ACQUIRE) != 0u; }

bc_status devq_collect(DevQueue* q, QueueJob* j, int32_t* ids, uint64_t* farness, uint32_t* reach, int32_t* count,
                       bc_stats* st, double query_ms) {
    const uint32_t dv = __atomic_load_n(&q->done[j->slot], __ATOMIC_ACQUIRE);
    const int32_t cnt = (int32_t)dv - 1;
    if (cnt != j->kk) {
        set_error("internal: queued request finished with %d of %d entries", cnt, j->kk);
        return BC_EDEVICE;
    }
    const Rec* r = q->out + (size_t)j->slot * kQueueMaxK;
    for (int32_t i = 0; i < cnt; ++i) {
        ids[i] = (int32_t)(uint32_t)(r[i].idr & 0xFFFFFFFFu);
        reach[i] = (uint32_t)(r[i].idr >> 32);
        farness[i] = r[i].f;
    }
    *count = cnt;
    if (st) {
        QStats h;
        std::memcpy(&h, q->out_st + (size_t)j->slot * (sizeof(QStats) / 8), sizeof(QStats));
        multi_stats(h, j->g->preprocess_ms, query_ms, 0.0, st);
    }
    return BC_OK;
}

void devq_release(DevQueue* q, QueueJob* j) {
    {
        std::lock_guard<std::mutex> lk(q->mu);
        clear_slot_locked(q, j->slot);
        clear_slot_locked(q, j->slot2);
        if (j->slot >= 0) q->busy[(size_t)j->slot] = 0;
        if (j->slot2 >= 0) q->busy[(size_t)j->slot2] = 0;
    }
    q->cv.notify_all();
    delete j;
}

void devq_free(QueueJob* j) { delete j; }

bc_status devq_pump(DevQueue* q) {
    std::lock_guard<std::mutex> lk(q->mu);
    return pump_locked(q);
}

}  // namespace bc
