// Learned source order.  Algorithm 1 returns the same top-k for every
// processing order; the order only decides how soon the k-th best value is
// known (Section 2.1).  The paper uses decreasing degree.  Here a small
// perceptron scores every node from three features and the sources are
// processed by decreasing score (ties by decreasing degree, then id):
//
//   x0 = log(1 + outdeg(v))
//   x1 = log(1 + sum of outdeg(u) over the out-arcs v -> u)
//   x2 = log(1 + core(v))   core(v): largest c such that v lies in a subgraph
//                           where every node keeps >= c out-neighbours
//
// each column standardised over the nodes ((x - mean) / population std; a
// column whose integers are all equal is 0).  core(v) is the fixed point of
// the in-place h-index iteration h(v) <- max{c : at least c out-neighbours u
// have h(u) >= c}, started from the out-degree: every estimate stays >= the
// core number, and a sweep that changes nothing leaves a fixed point, which
// is <= the core number.
//
// Perceptron 3 -> 64 -> 64 -> 1 with ReLU, fp32, parameters in one vector
//   W1[64][3] @0, b1 @192, W2[64][64] @256, b2 @4352, w3 @4416, b3 @4480.
// The trainer uses the loss sum w (y - t)^2 / sum w, its gradient and Adam.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>

#include "bc_internal.h"

namespace bc {

namespace {

constexpr int kBlk = 256;
constexpr int kH = 64;
constexpr int kOffW1 = 0, kOffB1 = 192, kOffW2 = 256, kOffB2 = 4352, kOffW3 = 4416, kOffB3 = 4480;
constexpr int kNP = BC_MLP_PARAMS;
static_assert(kOffB3 + 1 == kNP, "parameter layout");
constexpr int kTile = 128;        // samples per workgroup in the gradient kernel
constexpr int kRedBlocks = 512;   // partial sums of the feature statistics

inline unsigned grid_for(int64_t work, int64_t cap = 8192) {
    int64_t b = (work + kBlk - 1) / kBlk;
    if (b < 1) b = 1;
    if (b > cap) b = cap;
    return (unsigned)b;
}

__device__ inline uint32_t ld_relaxed(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// --------------------------------------------------------------- features

// s2[v] = sum of deg(u) over the out-arcs of v; h[v] = deg(v) (core start);
// integer min/max of the three integer columns (for the constant test).
__global__ void k_feat_init(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col,
                            const uint32_t* __restrict__ deg, uint64_t* __restrict__ s2, uint32_t* __restrict__ h,
                            unsigned long long* mm) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        uint64_t s = 0;
        for (int32_t e = rp[v]; e < rp[v + 1]; ++e) s += deg[col[e]];
        s2[v] = s;
        h[v] = deg[v];
        atomicMin(&mm[0], (unsigned long long)deg[v]);
        atomicMax(&mm[1], (unsigned long long)deg[v]);
        atomicMin(&mm[2], (unsigned long long)s);
        atomicMax(&mm[3], (unsigned long long)s);
    }
}

__device__ inline uint32_t count_at_least(const int32_t* __restrict__ col, int32_t b, int32_t e, const uint32_t* h,
                                          uint32_t c) {
    uint32_t cnt = 0;
    for (int32_t i = b; i < e; ++i) cnt += ld_relaxed(&h[col[i]]) >= c;
    return cnt;
}

// One in-place sweep of the h-index iteration over the nodes of degree <
// kHeavy (one thread each).  Estimates only decrease and other threads may
// lower them meanwhile; any value read is >= the core number, which keeps
// every update >= the core number.
constexpr uint32_t kHeavy = 256;

__global__ void k_hindex(int32_t n, const int32_t* __restrict__ rp, const int32_t* __restrict__ col, uint32_t* h,
                         uint32_t* changed) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        uint32_t hv = ld_relaxed(&h[v]);
        if (hv == 0 || (uint32_t)(rp[v + 1] - rp[v]) >= kHeavy) continue;
        int32_t b = rp[v], e = rp[v + 1];
        if (count_at_least(col, b, e, h, hv) >= hv) continue;
        // largest c in [0, hv - 1] with count(c) >= c (c = 0 always holds)
        uint32_t lo = 0, hi = hv - 1;
        while (lo < hi) {
            uint32_t mid = lo + (hi - lo + 1) / 2;
            if (count_at_least(col, b, e, h, mid) >= mid) lo = mid;
            else hi = mid - 1;
        }
        __hip_atomic_store(&h[v], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        *changed = 1u;
    }
}

// Nodes of degree >= kHeavy, one wave each (the lanes split the adjacency).
__global__ void k_heavy_list(int32_t n, const uint32_t* __restrict__ deg, int32_t* __restrict__ list,
                             uint32_t* __restrict__ len) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        if (deg[v] >= kHeavy) list[atomicAdd(len, 1u)] = (int32_t)v;
}

__device__ inline uint32_t wave_count_at_least(const int32_t* __restrict__ col, int32_t b, int32_t e,
                                               const uint32_t* h, uint32_t c, int lane) {
    uint32_t cnt = 0;
    for (int32_t i = b + lane; i < e; i += 64) cnt += ld_relaxed(&h[col[i]]) >= c;
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    return cnt;  // every lane holds the total
}

__global__ void k_hindex_heavy(const int32_t* __restrict__ list, const uint32_t* __restrict__ len,
                               const int32_t* __restrict__ rp, const int32_t* __restrict__ col, uint32_t* h,
                               uint32_t* changed) {
    const int lane = threadIdx.x & 63;
    const uint32_t nh = *len;
    const uint32_t waves = gridDim.x * (blockDim.x / 64);
    for (uint32_t q = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64; q < nh; q += waves) {
        const int32_t v = list[q];
        const uint32_t hv = ld_relaxed(&h[v]);
        if (hv == 0) continue;
        const int32_t b = rp[v], e = rp[v + 1];
        if (wave_count_at_least(col, b, e, h, hv, lane) >= hv) continue;
        uint32_t lo = 0, hi = hv - 1;
        while (lo < hi) {
            uint32_t mid = lo + (hi - lo + 1) / 2;
            if (wave_count_at_least(col, b, e, h, mid, lane) >= mid) lo = mid;
            else hi = mid - 1;
        }
        if (lane == 0) {
            __hip_atomic_store(&h[v], lo, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            *changed = 1u;
        }
    }
}

__device__ inline void raw3(int64_t v, const uint32_t* deg, const uint64_t* s2, const uint32_t* core, double r[3]) {
    r[0] = log1p((double)deg[v]);
    r[1] = log1p((double)s2[v]);
    r[2] = log1p((double)core[v]);
}

// Block sums of the raw features (pass 0) or of their squared deviations
// from the mean (pass 1), one row of 3 doubles per workgroup.
__global__ __launch_bounds__(kBlk) void k_feat_sums(int32_t n, const uint32_t* __restrict__ deg,
                                                    const uint64_t* __restrict__ s2,
                                                    const uint32_t* __restrict__ core, const double* __restrict__ mean,
                                                    double* __restrict__ part) {
    __shared__ double red[3][kBlk];
    double a[3] = {0.0, 0.0, 0.0};
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        double r[3];
        raw3(v, deg, s2, core, r);
        for (int j = 0; j < 3; ++j) {
            double d = mean ? r[j] - mean[j] : r[j];
            a[j] += mean ? d * d : d;
        }
    }
    for (int j = 0; j < 3; ++j) red[j][threadIdx.x] = a[j];
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
            for (int j = 0; j < 3; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = red[threadIdx.x][0];
}

// Sum the block rows in a fixed order; out[j] = total / n (mean or variance).
__global__ void k_feat_finish(int32_t n, int nparts, const double* __restrict__ part, double* __restrict__ out) {
    int j = threadIdx.x;
    if (j >= 3) return;
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += part[b * 3 + j];
    out[j] = s / (double)n;
}

__global__ void k_feat_write(int32_t n, const uint32_t* __restrict__ deg, const uint64_t* __restrict__ s2,
                             const uint32_t* __restrict__ core, const double* __restrict__ mean,
                             const double* __restrict__ var, const unsigned long long* __restrict__ mm,
                             float* __restrict__ x) {
    bool cst[3] = {mm[0] == mm[1], mm[2] == mm[3], mm[4] == mm[5]};
    double sd[3];
    for (int j = 0; j < 3; ++j) sd[j] = sqrt(var[j]);
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        double r[3];
        raw3(v, deg, s2, core, r);
        for (int j = 0; j < 3; ++j) x[v * 3 + j] = cst[j] ? 0.f : (float)((r[j] - mean[j]) / sd[j]);
    }
}

__global__ void k_core_minmax(int32_t n, const uint32_t* __restrict__ core, unsigned long long* mm) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        atomicMin(&mm[4], (unsigned long long)core[v]);
        atomicMax(&mm[5], (unsigned long long)core[v]);
    }
}

__global__ void k_minmax_init(unsigned long long* mm) {
    if (threadIdx.x < 6) mm[threadIdx.x] = (threadIdx.x & 1) ? 0ull : ~0ull;
}

// ------------------------------------------------------------ perceptron

__device__ inline void load_params(const float* __restrict__ p, float* s) {
    for (int i = threadIdx.x; i < kNP; i += blockDim.x) s[i] = p[i];
}

// h1 = relu(W1 x + b1) for one sample
__device__ inline void layer1(const float* P, float x0, float x1, float x2, float h1[kH]) {
#pragma unroll
    for (int i = 0; i < kH; ++i) {
        float a = P[kOffB1 + i];
        a = fmaf(P[kOffW1 + i * 3 + 0], x0, a);
        a = fmaf(P[kOffW1 + i * 3 + 1], x1, a);
        a = fmaf(P[kOffW1 + i * 3 + 2], x2, a);
        h1[i] = fmaxf(a, 0.f);
    }
}

// h2_j = relu(W2[j] . h1 + b2_j)
__device__ inline float unit2(const float* P, const float h1[kH], int j) {
    float a = P[kOffB2 + j];
#pragma unroll
    for (int i = 0; i < kH; ++i) a = fmaf(P[kOffW2 + j * kH + i], h1[i], a);
    return fmaxf(a, 0.f);
}

// Weights are read at wave-uniform addresses straight from the parameter
// vector (scalar loads, no LDS staging); one sample per thread.
__global__ __launch_bounds__(kBlk) void k_mlp_forward(const float* __restrict__ P, const float* __restrict__ x,
                                                      int64_t count, float* __restrict__ y) {
    int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < count; s += stride) {
        float h1[kH];
        layer1(P, x[s * 3], x[s * 3 + 1], x[s * 3 + 2], h1);
        float out = P[kOffB3];
#pragma unroll 1
        for (int j = 0; j < kH; ++j) out = fmaf(P[kOffW3 + j], unit2(P, h1, j), out);
        y[s] = out;
    }
}

// Loss gradient over one tile of kTile samples per workgroup, with the
// unnormalised output gradient dy = 2 w (y - t); the reduction kernel sums
// the tiles in a fixed order and divides by sum w.  Per tile row (sample):
// X (3), DY, H1/H2 (forward activations), G2 = dL/d(pre-activation of layer
// 2), G1 = dL/d(pre-activation of layer 1).  Partial row per tile:
// the kNP gradient entries, then sum w r^2 and sum w.
struct GradLds {
    float P[kNP];
    float X[kTile][3];
    float DY[kTile];
    float H1[kTile][kH];
    float H2[kTile][kH];
    float G2[kTile][kH];
    float G1[kTile][kH];
    float WR2[kTile], WS[kTile];
};

__global__ __launch_bounds__(kBlk) void k_mlp_grad(const float* __restrict__ params, const float* __restrict__ x,
                                                   const float* __restrict__ t, const float* __restrict__ w,
                                                   int64_t rows, const int32_t* __restrict__ idx, int64_t count,
                                                   float* __restrict__ part, uint32_t* __restrict__ bad) {
    __shared__ GradLds L;
    load_params(params, L.P);
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * kTile;
    __syncthreads();
    if (tid < kTile) {
        int64_t s = base + tid;
        float x0 = 0.f, x1 = 0.f, x2 = 0.f, ws = 0.f, tv = 0.f;
        int64_t v = s < count ? (idx ? (int64_t)idx[s] : s) : -1;
        if (s < count && (v < 0 || v >= rows)) {
            *bad = 1u;  // the sample is left out (weight 0); the call fails
            v = -1;
        }
        if (v >= 0) {
            x0 = x[v * 3];
            x1 = x[v * 3 + 1];
            x2 = x[v * 3 + 2];
            ws = w ? w[v] : 1.f;
            tv = t[v];
        }
        L.X[tid][0] = x0;
        L.X[tid][1] = x1;
        L.X[tid][2] = x2;
        float h1[kH];
        layer1(L.P, x0, x1, x2, h1);
        float out = L.P[kOffB3];
        for (int j = 0; j < kH; ++j) {
            float h2 = unit2(L.P, h1, j);
            L.H2[tid][j] = h2;
            out = fmaf(L.P[kOffW3 + j], h2, out);
        }
        float r = out - tv;
        float dy = 2.f * ws * r;  // ws = 0 outside the sample range
        L.DY[tid] = dy;
        L.WR2[tid] = ws * r * r;
        L.WS[tid] = ws;
        float g1[kH];
#pragma unroll
        for (int i = 0; i < kH; ++i) g1[i] = 0.f;
        for (int j = 0; j < kH; ++j) {
            float g2 = L.H2[tid][j] > 0.f ? dy * L.P[kOffW3 + j] : 0.f;
            L.G2[tid][j] = g2;
#pragma unroll
            for (int i = 0; i < kH; ++i) g1[i] = fmaf(L.P[kOffW2 + j * kH + i], g2, g1[i]);
        }
#pragma unroll
        for (int i = 0; i < kH; ++i) {
            L.H1[tid][i] = h1[i];
            L.G1[tid][i] = h1[i] > 0.f ? g1[i] : 0.f;
        }
    }
    __syncthreads();
    float* out = part + (size_t)blockIdx.x * (kNP + 2);
    // dW2[j][i0 .. i0+15] = sum over the tile of G2[s][j] H1[s][i]
    {
        const int j = tid >> 2, i0 = (tid & 3) * 16;
        float a[16];
#pragma unroll
        for (int q = 0; q < 16; ++q) a[q] = 0.f;
        for (int s = 0; s < kTile; ++s) {
            float g = L.G2[s][j];
#pragma unroll
            for (int q = 0; q < 16; ++q) a[q] = fmaf(g, L.H1[s][i0 + q], a[q]);
        }
#pragma unroll
        for (int q = 0; q < 16; ++q) out[kOffW2 + j * kH + i0 + q] = a[q];
    }
    // the small entries: W1 (192), b1 (64), b2 (64), w3 (64), b3, loss sums
    for (int e = tid; e < 192 + 64 + 64 + 64 + 1 + 2; e += kBlk) {
        float a = 0.f;
        int dst;
        if (e < 192) {
            int i = e / 3, c = e % 3;
            for (int s = 0; s < kTile; ++s) a = fmaf(L.G1[s][i], L.X[s][c], a);
            dst = kOffW1 + e;
        } else if (e < 256) {
            int i = e - 192;
            for (int s = 0; s < kTile; ++s) a += L.G1[s][i];
            dst = kOffB1 + i;
        } else if (e < 320) {
            int j = e - 256;
            for (int s = 0; s < kTile; ++s) a += L.G2[s][j];
            dst = kOffB2 + j;
        } else if (e < 384) {
            int j = e - 320;
            for (int s = 0; s < kTile; ++s) a = fmaf(L.DY[s], L.H2[s][j], a);
            dst = kOffW3 + j;
        } else if (e == 384) {
            for (int s = 0; s < kTile; ++s) a += L.DY[s];
            dst = kOffB3;
        } else if (e == 385) {
            for (int s = 0; s < kTile; ++s) a += L.WR2[s];
            dst = kNP;
        } else {
            for (int s = 0; s < kTile; ++s) a += L.WS[s];
            dst = kNP + 1;
        }
        out[dst] = a;
    }
}

// grad[p] = (sum over tiles, in tile order, in double) / sum w; loss likewise.
__global__ void k_mlp_grad_reduce(int ntiles, const float* __restrict__ part, float* __restrict__ grad,
                                  double* __restrict__ loss) {
    __shared__ double s_sw;
    if (threadIdx.x == 0) {
        double sw = 0.0;
        for (int b = 0; b < ntiles; ++b) sw += part[(size_t)b * (kNP + 2) + kNP + 1];
        s_sw = sw;
    }
    __syncthreads();
    const double sw = s_sw;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < kNP + 1; p += gridDim.x * blockDim.x) {
        double a = 0.0;
        for (int b = 0; b < ntiles; ++b) a += part[(size_t)b * (kNP + 2) + p];
        double v = sw > 0.0 ? a / sw : 0.0;
        if (p < kNP) grad[p] = (float)v;
        else *loss = v;
    }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, int count, float lr, float b1, float b2, float eps, float c1, float c2) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    float gi = g[i];
    float mi = b1 * m[i] + (1.f - b1) * gi;
    float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi * c1) / (sqrtf(vi * c2) + eps);
}

}  // namespace

// Features of the graph into g->feat (n x 3 float) and g->core (u32), built
// once per graph.
bc_status graph_features(bc_graph* g, hipStream_t s) {
    std::lock_guard<std::mutex> lk(g->cache_mu);
    if (g->have_feat) return BC_OK;
    const int32_t n = g->dg.n;
    BC_TRY(galloc(g, g->feat, sizeof(float) * 3 * (size_t)std::max(n, 1), s));
    BC_TRY(galloc(g, g->core, sizeof(uint32_t) * (size_t)std::max(n, 1), s));
    if (n == 0) {
        g->have_feat = true;
        return BC_OK;
    }
    DevBuf s2, mm, flag, part, stat, heavy, nheavy;
    BC_TRY(s2.alloc_on(sizeof(uint64_t) * (size_t)n, s));
    BC_TRY(heavy.alloc_on(sizeof(int32_t) * (size_t)n, s));
    BC_TRY(nheavy.alloc_on(sizeof(uint32_t), s));
    BC_TRY(mm.alloc_on(sizeof(unsigned long long) * 6, s));
    BC_TRY(flag.alloc_on(sizeof(uint32_t), s));
    BC_TRY(part.alloc_on(sizeof(double) * 3 * kRedBlocks, s));
    BC_TRY(stat.alloc_on(sizeof(double) * 6, s));
    uint32_t* h = g->core.as<uint32_t>();
    k_minmax_init<<<1, 64, 0, s>>>(mm.as<unsigned long long>());
    k_feat_init<<<grid_for(n), kBlk, 0, s>>>(n, g->dg.rp, g->dg.col, g->dg.deg, s2.as<uint64_t>(), h,
                                             mm.as<unsigned long long>());
    BC_HIP(hipMemsetAsync(nheavy.p, 0, sizeof(uint32_t), s));
    k_heavy_list<<<grid_for(n), kBlk, 0, s>>>(n, g->dg.deg, heavy.as<int32_t>(), nheavy.as<uint32_t>());
    // h-index sweeps until one changes nothing; every sweep that changes
    // something lowers the sum of the estimates, so this ends
    for (;;) {
        BC_HIP(hipMemsetAsync(flag.p, 0, sizeof(uint32_t), s));
        k_hindex<<<grid_for(n), kBlk, 0, s>>>(n, g->dg.rp, g->dg.col, h, flag.as<uint32_t>());
        k_hindex_heavy<<<1024, kBlk, 0, s>>>(heavy.as<int32_t>(), nheavy.as<uint32_t>(), g->dg.rp, g->dg.col, h,
                                             flag.as<uint32_t>());
        uint32_t changed = 0;
        BC_HIP(hipMemcpyAsync(&changed, flag.p, sizeof(changed), hipMemcpyDeviceToHost, s));
        BC_HIP(hipStreamSynchronize(s));
        ++g->core_sweeps;
        if (!changed) break;
    }
    k_core_minmax<<<grid_for(n), kBlk, 0, s>>>(n, h, mm.as<unsigned long long>());
    const unsigned nb = grid_for(n, kRedBlocks);
    double* mean = stat.as<double>();
    double* var = mean + 3;
    k_feat_sums<<<nb, kBlk, 0, s>>>(n, g->dg.deg, s2.as<uint64_t>(), h, nullptr, part.as<double>());
    k_feat_finish<<<1, 64, 0, s>>>(n, (int)nb, part.as<double>(), mean);
    k_feat_sums<<<nb, kBlk, 0, s>>>(n, g->dg.deg, s2.as<uint64_t>(), h, mean, part.as<double>());
    k_feat_finish<<<1, 64, 0, s>>>(n, (int)nb, part.as<double>(), var);
    k_feat_write<<<grid_for(n), kBlk, 0, s>>>(n, g->dg.deg, s2.as<uint64_t>(), h, mean, var,
                                              mm.as<unsigned long long>(), g->feat.as<float>());
    BC_HIP(hipGetLastError());
    BC_HIP(hipStreamSynchronize(s));
    g->have_feat = true;
    return BC_OK;
}

bc_status mlp_forward(const float* params, const float* x, int64_t count, float* y, hipStream_t s) {
    if (count == 0) return BC_OK;
    k_mlp_forward<<<grid_for(count, 16384), kBlk, 0, s>>>(params, x, count, y);
    BC_HIP(hipGetLastError());
    return BC_OK;
}

bc_status mlp_loss_grad(const float* params, const float* x, const float* t, const float* w, int64_t rows,
                        const int32_t* idx, int64_t count, float* grad, double* loss, hipStream_t s) {
    if (!idx && count > rows) {
        set_error("count %lld exceeds rows %lld", (long long)count, (long long)rows);
        return BC_EINVAL;
    }
    const int64_t ntiles = std::max<int64_t>(1, (count + kTile - 1) / kTile);
    if (ntiles > (int64_t)1 << 24) {
        set_error("too many samples in one gradient call (%lld)", (long long)count);
        return BC_EINVAL;
    }
    DevBuf part, dres;
    BC_TRY(part.alloc_on(sizeof(float) * (kNP + 2) * (size_t)ntiles, s));
    BC_TRY(dres.alloc_on(sizeof(double) * 2, s));
    BC_HIP(hipMemsetAsync(dres.p, 0, sizeof(double) * 2, s));
    uint32_t* d_bad = reinterpret_cast<uint32_t*>(dres.as<double>() + 1);
    k_mlp_grad<<<(unsigned)ntiles, kBlk, 0, s>>>(params, x, t, w, rows, idx, count, part.as<float>(), d_bad);
    k_mlp_grad_reduce<<<(kNP + 1 + kBlk - 1) / kBlk, kBlk, 0, s>>>((int)ntiles, part.as<float>(), grad,
                                                                     dres.as<double>());
    BC_HIP(hipGetLastError());
    double res[2] = {0.0, 0.0};
    BC_HIP(hipMemcpyAsync(res, dres.p, sizeof(res), hipMemcpyDeviceToHost, s));
    BC_HIP(hipStreamSynchronize(s));  // `part` is released on return
    uint32_t bad = 0;
    std::memcpy(&bad, &res[1], sizeof(bad));
    if (bad) {
        set_error("idx holds an entry outside [0, rows)");
        return BC_EINVAL;
    }
    if (loss) *loss = res[0];
    return BC_OK;
}

bc_status mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                   float beta2, float eps, hipStream_t s) {
    const double c1 = 1.0 / (1.0 - std::pow((double)beta1, (double)step));
    const double c2 = 1.0 / (1.0 - std::pow((double)beta2, (double)step));
    k_adam<<<(kNP + kBlk - 1) / kBlk, kBlk, 0, s>>>(params, grad, m, v, kNP, lr, beta1, beta2, eps, (float)c1,
                                                    (float)c2);
    BC_HIP(hipGetLastError());
    return BC_OK;
}

}  // namespace bc
