// Learned index over the tree: training and lookup kernels.
//
// Stage 1 (root): x = (key - kmin) * scale in FP64, rounded to FP32;
// j = clamp(floor(a x + b), 0, M-1).  Stage 2 (model j): a linear model
// p = slope x_j + icpt, or an MLP p = b2 + sum_u w2_u relu(w1_u x_j + b1_u)
// with 32 hidden units, on the model's own normalised key x_j.  The
// prediction is the leaf's position in key order (the leaf chain order at
// training time).
//
// Training (all on the device, deterministic reduction orders):
//   leaf positions   list ranking of the leaf chain by pointer jumping
//   directory        dir[pos] = (first key of the leaf, leaf id)
//   root             least squares of pos*M/L on the fences (FP64 sums)
//   model ranges     the root is monotone, so model j owns a contiguous run
//                    of fences
//   leaf models      least squares per model on its fences; the MLP uses
//                    hinge units relu(x - t_u) with knots t_u at the run's
//                    quantiles and output weights from the normal equations
//                    (FP64 Cholesky) -- a one-hidden-layer ReLU network whose
//                    output layer is fitted in closed form
//   bounds           every key of the tree is pushed through the same
//                    inference functions the lookup uses; lo_j / hi_j are
//                    the exact min / max of (true position - prediction)
//                    over the keys routed to model j, per model kind; the
//                    kind with the smaller window is kept
//
// Lookup: predict, clamp the window [p + lo, p + hi] to the directory,
// find the last fence <= key in it, read that leaf's key and value lines.
// A match is a hit.  No match is an authoritative miss only when the leaf's
// first and last keys bracket the key (the tree routes every key in that
// interval to this leaf); otherwise -- the window missed, the leaf split
// since training, the model has no bounds -- the query walks the tree in
// the same kernel.  So results equal the tree's for any model state.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <vector>
#include <cmath>

#include "../../include/gtree.h"
#include "common.h"
#include "traverse.h"
#include "handle.h"

namespace gt {

constexpr int kHidden = 32;
constexpr int kLiG = 8;             // lanes per query
constexpr int kLiBlock = 256;
constexpr uint32_t kKindLinear = 0, kKindMlp = 1, kKindTree = 2;
constexpr int kFitPoints = 4096;    // points per model used for the MLP fit

struct LiHeader {
    uint64_t kmin_root;
    double root_scale;
    float root_a, root_b;
    uint32_t L;          // leaves in the directory
    uint32_t M;
    uint64_t n_keys;
    unsigned long long lookups, fallbacks;
    uint32_t trained;
    uint32_t pad[49];
};
static_assert(sizeof(LiHeader) == 256, "LiHeader size");

struct ModelRec {
    uint64_t kmin;
    double scale;
    uint32_t kind;
    int32_t lo, hi;
    float slope, icpt, b2;
    uint32_t n_keys;     // keys routed here at training
    uint32_t pad[5];
    float w1[kHidden];
    float b1[kHidden];
    float w2[kHidden];
    uint32_t pad2[16];
};
static_assert(sizeof(ModelRec) == 512, "ModelRec size");

template <class K>
struct alignas(sizeof(K) == 8 ? 16 : 8) DirEntry {
    K fence;
    uint32_t leaf;
};
static_assert(sizeof(DirEntry<uint64_t>) == 16 && sizeof(DirEntry<uint32_t>) == 8, "DirEntry size");

// Compact per-model record read by the lookup (staged into LDS).
struct ModelLite {
    uint64_t kmin;
    double scale;
    float slope, icpt;
    int32_t lo_hi;       // lo in the low 16 bits, hi in the high 16 (signed)
    uint32_t kind;
};
static_assert(sizeof(ModelLite) == 32, "ModelLite size");

// Root parameters passed to the lookup by value (no dependent header load).
struct LiArgs {
    uint64_t kmin_root;
    double root_scale;
    float root_a, root_b;
    uint32_t L, M;
    uint32_t identity;   // directory position == leaf id for every position
    uint32_t pad;
};

template <class K>
struct LiView {
    LiHeader* hdr;
    ModelRec* models;
    ModelLite* lite;
    uint32_t* identity;
    DirEntry<K>* dir;
    uint32_t* nxt0; uint32_t* nxt1; uint32_t* rank0; uint32_t* rank1;
    uint32_t* pos_of_leaf;
    uint32_t* start;       // M + 1
    int32_t* bnd;          // 4 * M: lo_lin, hi_lin, lo_mlp, hi_mlp
    uint32_t* cnt;         // M
    double* partial;       // kMaxPartials * 5
    float* mlp_ok;         // M (1 = MLP fitted)
};

constexpr int kMaxPartials = 4096;

// ------------------------------------------------------------ inference

// (key - kmin) * scale with the difference taken in FP64 on either side of
// kmin (u64 differences can exceed the int64 range)
__device__ __forceinline__ float norm_x(uint64_t key, uint64_t kmin, double scale) {
    const double d = key >= kmin ? static_cast<double>(key - kmin) : -static_cast<double>(kmin - key);
    return static_cast<float>(d * scale);
}

template <class H>
__device__ __forceinline__ uint32_t root_index(const H& h, uint64_t key) {
    const float x = norm_x(key, h.kmin_root, h.root_scale);
    float f = __fmaf_rn(h.root_a, x, h.root_b);
    f = fminf(fmaxf(f, 0.0f), static_cast<float>(h.M - 1));
    return static_cast<uint32_t>(floorf(f));
}

__device__ __forceinline__ int32_t clamp_pos(float f, uint32_t L) {
    f = fminf(fmaxf(f, -1.0e9f), 1.0e9f);
    int32_t p = static_cast<int32_t>(floorf(f));
    if (p < 0) p = 0;
    if (p > static_cast<int32_t>(L) - 1) p = static_cast<int32_t>(L) - 1;
    return p;
}

__device__ __forceinline__ float linear_eval(const ModelRec& m, float x) { return __fmaf_rn(m.slope, x, m.icpt); }

// MLP output evaluated by a group of 8 lanes (4 hidden units each), summed
// with an xor tree so every lane of the group holds the same bits.
__device__ __forceinline__ float mlp_eval_group(const ModelRec* m, float x, int gl) {
    const float4 w1 = reinterpret_cast<const float4*>(m->w1)[gl];
    const float4 b1 = reinterpret_cast<const float4*>(m->b1)[gl];
    const float4 w2 = reinterpret_cast<const float4*>(m->w2)[gl];
    float part = 0.0f;
    part = __fmaf_rn(w2.x, fmaxf(0.0f, __fmaf_rn(w1.x, x, b1.x)), part);
    part = __fmaf_rn(w2.y, fmaxf(0.0f, __fmaf_rn(w1.y, x, b1.y)), part);
    part = __fmaf_rn(w2.z, fmaxf(0.0f, __fmaf_rn(w1.z, x, b1.z)), part);
    part = __fmaf_rn(w2.w, fmaxf(0.0f, __fmaf_rn(w1.w, x, b1.w)), part);
    part += __shfl_xor(part, 1, 64);
    part += __shfl_xor(part, 2, 64);
    part += __shfl_xor(part, 4, 64);
    return part + m->b2;
}

// Predicted position of `key` under model m of the given kind.
__device__ __forceinline__ int32_t predict(const ModelRec* m, uint32_t kind, uint64_t key, uint32_t L, int gl) {
    const float x = norm_x(key, m->kmin, m->scale);
    const float f = kind == kKindMlp ? mlp_eval_group(m, x, gl) : linear_eval(*m, x);
    return clamp_pos(f, L);
}

// ------------------------------------------------------------- training

__device__ __forceinline__ uint64_t gid() { return blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; }
__device__ __forceinline__ uint64_t gsz() { return static_cast<uint64_t>(gridDim.x) * blockDim.x; }

__global__ void k_rank_init(const uint2* lmeta, uint32_t n, uint32_t* nxt, uint32_t* rank) {
    for (uint64_t i = gid(); i < n; i += gsz()) {
        const uint32_t x = lmeta[i].y;
        nxt[i] = x;
        rank[i] = x == kNone ? 0u : 1u;
    }
}

__global__ void k_rank_jump(const uint32_t* nin, const uint32_t* rin, uint32_t* nout, uint32_t* rout, uint32_t n) {
    for (uint64_t i = gid(); i < n; i += gsz()) {
        const uint32_t x = nin[i];
        if (x == kNone) {
            nout[i] = kNone;
            rout[i] = rin[i];
        } else {
            nout[i] = nin[x];
            rout[i] = rin[i] + rin[x];
        }
    }
}

template <class K>
__global__ void k_directory(TreeView<K> t, LiView<K> li, const uint32_t* rank, uint32_t n) {
    for (uint64_t i = gid(); i < n; i += gsz()) {
        const uint32_t pos = n - 1 - rank[i];
        DirEntry<K> e;
        e.fence = t.lkeys[i * kSlots];
        e.leaf = static_cast<uint32_t>(i);
        li.dir[pos] = e;
        li.pos_of_leaf[i] = pos;
    }
    if (gid() == 0) {
        DirEntry<K> e;
        e.fence = kmax<K>();
        e.leaf = kNone;
        li.dir[n] = e;
    }
}

// FP64 block sum in a fixed order (tree over LDS), blockDim = 256
__device__ __forceinline__ double block_sum(double v, double* sh) {
    sh[threadIdx.x] = v;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (threadIdx.x < static_cast<unsigned>(s)) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

// root sums: block b covers fences [b*n/nb, (b+1)*n/nb)
template <class K>
__global__ __launch_bounds__(256) void k_root_partial(LiView<K> li, uint32_t L, uint32_t M, uint64_t kmin,
                                                      double scale) {
    __shared__ double sh[256];
    const uint64_t b0 = part_start(blockIdx.x, L, gridDim.x), b1 = part_start(blockIdx.x + 1, L, gridDim.x);
    double s[5] = {0, 0, 0, 0, 0};
    for (uint64_t p = b0 + threadIdx.x; p < b1; p += blockDim.x) {
        const double x = norm_x(static_cast<uint64_t>(li.dir[p].fence), kmin, scale);
        const double y = static_cast<double>(p) * M / L;
        s[0] += 1.0; s[1] += x; s[2] += y; s[3] += x * x; s[4] += x * y;
    }
    for (int k = 0; k < 5; ++k) {
        const double r = block_sum(s[k], sh);
        if (threadIdx.x == 0) li.partial[blockIdx.x * 5 + k] = r;
    }
}

template <class K>
__global__ __launch_bounds__(256) void k_root_final(LiView<K> li, uint32_t nb, uint64_t kmin, double scale,
                                                    uint32_t L, uint32_t M) {
    if (threadIdx.x != 0) return;
    double s[5] = {0, 0, 0, 0, 0};
    for (uint32_t b = 0; b < nb; ++b)
        for (int k = 0; k < 5; ++k) s[k] += li.partial[b * 5 + k];
    const double n = s[0], den = n * s[3] - s[1] * s[1];
    double a = den > 0 ? (n * s[4] - s[1] * s[2]) / den : 0.0;
    if (!(a > 0)) a = 0.0;
    const double b = n > 0 ? (s[2] - a * s[1]) / n : 0.0;
    LiHeader* h = li.hdr;
    h->kmin_root = kmin;
    h->root_scale = scale;
    h->root_a = static_cast<float>(a);
    h->root_b = static_cast<float>(b);
    h->L = L;
    h->M = M;
}

// model j owns fences [start[j], start[j+1])
template <class K>
__global__ void k_ranges(LiView<K> li, uint32_t L, uint32_t M) {
    const LiHeader h = *li.hdr;
    for (uint64_t p = gid(); p < L; p += gsz()) {
        const uint32_t j = root_index(h, static_cast<uint64_t>(li.dir[p].fence));
        const int64_t jp = p ? static_cast<int64_t>(root_index(h, static_cast<uint64_t>(li.dir[p - 1].fence))) : -1;
        for (int64_t jj = jp + 1; jj <= static_cast<int64_t>(j); ++jj) li.start[jj] = static_cast<uint32_t>(p);
        if (p + 1 == L)
            for (uint32_t jj = j + 1; jj <= M; ++jj) li.start[jj] = L;
    }
}

// Solve (G + ridge) w = r by Cholesky, n <= 33, FP64, one thread.
__device__ bool cholesky_solve(double* G, double* r, int n) {
    double tr = 0;
    for (int i = 0; i < n; ++i) tr += G[i * n + i];
    const double ridge = 1e-10 * (tr / n) + 1e-12;
    for (int i = 0; i < n; ++i) G[i * n + i] += ridge;
    for (int j = 0; j < n; ++j) {
        double d = G[j * n + j];
        for (int k = 0; k < j; ++k) d -= G[j * n + k] * G[j * n + k];
        if (!(d > 0)) return false;
        d = sqrt(d);
        G[j * n + j] = d;
        for (int i = j + 1; i < n; ++i) {
            double v = G[i * n + j];
            for (int k = 0; k < j; ++k) v -= G[i * n + k] * G[j * n + k];
            G[i * n + j] = v / d;
        }
    }
    for (int i = 0; i < n; ++i) {  // L y = r
        double v = r[i];
        for (int k = 0; k < i; ++k) v -= G[i * n + k] * r[k];
        r[i] = v / G[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {  // L^T w = y
        double v = r[i];
        for (int k = i + 1; k < n; ++k) v -= G[k * n + i] * r[k];
        r[i] = v / G[i * n + i];
    }
    return true;
}

// One workgroup per model: linear and MLP fits on the model's fences.
template <class K>
__global__ __launch_bounds__(256) void k_fit(LiView<K> li, uint32_t M) {
    constexpr int NF = kHidden + 1;
    __shared__ double sh[256];
    __shared__ float xs[kFitPoints];
    __shared__ float ys[kFitPoints];
    __shared__ float knot[kHidden];
    __shared__ double G[NF * NF];
    __shared__ double rr[NF];
    const uint32_t j = blockIdx.x;
    if (j >= M) return;
    ModelRec* m = li.models + j;
    const uint32_t b = li.start[j], e = li.start[j + 1];
    const uint32_t n = e - b;
    if (threadIdx.x == 0) {
        m->kind = n ? kKindLinear : kKindTree;
        m->lo = 0;
        m->hi = 0;
        m->n_keys = 0;
    }
    if (n == 0) {
        if (threadIdx.x == 0) { m->kmin = 0; m->scale = 1.0; m->slope = 0; m->icpt = 0; m->b2 = 0; li.mlp_ok[j] = 0; }
        return;
    }
    const uint64_t kmin = static_cast<uint64_t>(li.dir[b].fence);
    const uint64_t klast = static_cast<uint64_t>(li.dir[e - 1].fence);
    const double scale = klast > kmin ? 1.0 / static_cast<double>(klast - kmin) : 1.0;
    // linear least squares on all fences of the run
    double s[5] = {0, 0, 0, 0, 0};
    for (uint32_t p = b + threadIdx.x; p < e; p += blockDim.x) {
        const double x = norm_x(static_cast<uint64_t>(li.dir[p].fence), kmin, scale);
        const double y = static_cast<double>(p);
        s[0] += 1.0; s[1] += x; s[2] += y; s[3] += x * x; s[4] += x * y;
    }
    for (int k = 0; k < 5; ++k) s[k] = block_sum(s[k], sh);
    const double den = s[0] * s[3] - s[1] * s[1];
    const double a = den > 1e-300 ? (s[0] * s[4] - s[1] * s[2]) / den : 0.0;
    const double c = (s[2] - a * s[1]) / s[0];
    // MLP: up to kFitPoints evenly spaced fences of the run
    const uint32_t np = n < static_cast<uint32_t>(kFitPoints) ? n : static_cast<uint32_t>(kFitPoints);
    for (uint32_t i = threadIdx.x; i < np; i += blockDim.x) {
        const uint32_t p = b + static_cast<uint32_t>(part_start(i, n, np));
        xs[i] = norm_x(static_cast<uint64_t>(li.dir[p].fence), kmin, scale);
        ys[i] = static_cast<float>(p);
    }
    __syncthreads();
    if (threadIdx.x < kHidden) knot[threadIdx.x] = xs[part_start(threadIdx.x, np, kHidden)];
    __syncthreads();
    bool ok = false;
    if (np >= static_cast<uint32_t>(4 * NF)) {
        // Gram matrix of the features relu(x - t_u) (u < 32) and 1
        for (int q = threadIdx.x; q < NF * NF + NF; q += blockDim.x) {
            double acc = 0.0;
            if (q < NF * NF) {
                const int ua = q / NF, ub = q % NF;
                for (uint32_t i = 0; i < np; ++i) {
                    const double fa = ua < kHidden ? fmax(0.0, static_cast<double>(xs[i]) - knot[ua]) : 1.0;
                    const double fb = ub < kHidden ? fmax(0.0, static_cast<double>(xs[i]) - knot[ub]) : 1.0;
                    acc += fa * fb;
                }
                G[q] = acc;
            } else {
                const int ua = q - NF * NF;
                for (uint32_t i = 0; i < np; ++i) {
                    const double fa = ua < kHidden ? fmax(0.0, static_cast<double>(xs[i]) - knot[ua]) : 1.0;
                    acc += fa * ys[i];
                }
                rr[ua] = acc;
            }
        }
        __syncthreads();
        if (threadIdx.x == 0) ok = cholesky_solve(G, rr, NF);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        m->kmin = kmin;
        m->scale = scale;
        m->slope = static_cast<float>(a);
        m->icpt = static_cast<float>(c);
        li.mlp_ok[j] = ok ? 1.0f : 0.0f;
        if (ok) {
            for (int u = 0; u < kHidden; ++u) {
                m->w1[u] = 1.0f;
                m->b1[u] = -knot[u];
                m->w2[u] = static_cast<float>(rr[u]);
            }
            m->b2 = static_cast<float>(rr[kHidden]);
        } else {
            for (int u = 0; u < kHidden; ++u) { m->w1[u] = 0; m->b1[u] = 0; m->w2[u] = 0; }
            m->b2 = 0;
        }
    }
}

__global__ void k_bounds_init(int32_t* bnd, uint32_t* cnt, uint32_t M) {
    for (uint64_t j = gid(); j < M; j += gsz()) {
        bnd[4 * j + 0] = INT32_MAX; bnd[4 * j + 1] = INT32_MIN;
        bnd[4 * j + 2] = INT32_MAX; bnd[4 * j + 3] = INT32_MIN;
        cnt[j] = 0;
    }
}

// Every key of the tree, one 8-lane group per key, through both model kinds.
template <class K>
__global__ __launch_bounds__(kLiBlock) void k_bounds(TreeView<K> t, LiView<K> li, uint32_t nleaves) {
    const LiHeader h = *li.hdr;
    const int gl = lane_id() % kLiG;
    const uint64_t group = gid() / kLiG, ngroups = gsz() / kLiG;
    const uint64_t total = static_cast<uint64_t>(nleaves) * kSlots;
    for (uint64_t x = group; x < total; x += ngroups) {
        const uint32_t leaf = static_cast<uint32_t>(x / kSlots), slot = static_cast<uint32_t>(x % kSlots);
        if (slot >= t.lmeta[leaf].x) continue;  // group-uniform
        const uint64_t key = static_cast<uint64_t>(t.lkeys[x]);
        const int32_t pos = static_cast<int32_t>(li.pos_of_leaf[leaf]);
        const uint32_t j = root_index(h, key);
        const ModelRec* m = li.models + j;
        const int32_t plin = predict(m, kKindLinear, key, h.L, gl);
        const bool mlp = li.mlp_ok[j] != 0.0f;
        const int32_t pmlp = mlp ? predict(m, kKindMlp, key, h.L, gl) : 0;
        if (gl == 0) {
            atomicMin(&li.bnd[4 * j + 0], pos - plin);
            atomicMax(&li.bnd[4 * j + 1], pos - plin);
            if (mlp) {
                atomicMin(&li.bnd[4 * j + 2], pos - pmlp);
                atomicMax(&li.bnd[4 * j + 3], pos - pmlp);
            }
            atomicAdd(&li.cnt[j], 1u);
        }
    }
}

template <class K>
__global__ void k_choose(LiView<K> li, uint32_t M, uint32_t kind_pref, uint32_t max_window) {
    for (uint64_t j = gid(); j < M; j += gsz()) {
        ModelRec* m = li.models + j;
        const uint32_t c = li.cnt[j];
        m->n_keys = c;
        uint32_t kind = kKindTree;
        int32_t lo = 0, hi = 0;
        if (c > 0) {
            const int64_t wl = static_cast<int64_t>(li.bnd[4 * j + 1]) - li.bnd[4 * j + 0];
            const bool mlp = li.mlp_ok[j] != 0.0f;
            const int64_t wm = mlp ? static_cast<int64_t>(li.bnd[4 * j + 3]) - li.bnd[4 * j + 2] : INT64_MAX;
            bool use_mlp;
            if (kind_pref == 1) use_mlp = false;
            else if (kind_pref == 2) use_mlp = mlp;
            else use_mlp = wm < wl;
            kind = use_mlp ? kKindMlp : kKindLinear;
            lo = use_mlp ? li.bnd[4 * j + 2] : li.bnd[4 * j + 0];
            hi = use_mlp ? li.bnd[4 * j + 3] : li.bnd[4 * j + 1];
            if (static_cast<int64_t>(hi) - lo + 1 > static_cast<int64_t>(max_window) || lo < -32768 ||
                hi > 32767) {
                kind = kKindTree;
                lo = hi = 0;
            }
        }
        m->kind = kind;
        m->lo = lo;
        m->hi = hi;
        ModelLite ml;
        ml.kmin = m->kmin;
        ml.scale = m->scale;
        ml.slope = m->slope;
        ml.icpt = m->icpt;
        ml.lo_hi = static_cast<int32_t>((static_cast<uint32_t>(static_cast<uint16_t>(static_cast<int16_t>(lo)))) |
                                        (static_cast<uint32_t>(static_cast<uint16_t>(static_cast<int16_t>(hi))) << 16));
        ml.kind = kind;
        li.lite[j] = ml;
    }
}

__global__ void k_identity(const uint32_t* pos_of_leaf, uint32_t n, uint32_t* flag) {
    for (uint64_t i = gid(); i < n; i += gsz())
        if (pos_of_leaf[i] != i) *flag = 0u;
}

template <class K>
__global__ void k_li_finish(LiView<K> li, uint64_t n_keys) {
    if (gid() == 0) {
        li.hdr->n_keys = n_keys;
        li.hdr->lookups = 0;
        li.hdr->fallbacks = 0;
        li.hdr->trained = 1;
    }
}

__global__ void k_set_bounds(ModelRec* models, ModelLite* lite, uint32_t M, int32_t lo, int32_t hi) {
    for (uint64_t j = gid(); j < M; j += gsz()) {
        if (models[j].kind != kKindTree) {
            models[j].lo = lo;
            models[j].hi = hi;
            lite[j].lo_hi = static_cast<int32_t>(
                (static_cast<uint32_t>(static_cast<uint16_t>(static_cast<int16_t>(lo)))) |
                (static_cast<uint32_t>(static_cast<uint16_t>(static_cast<int16_t>(hi))) << 16));
        }
    }
}

// --------------------------------------------------------------- lookup

// Directory window search by one 8-lane group: the last position in
// [wl, wh] whose fence is <= key, or -1; *leaf receives its leaf id.
template <class K>
__device__ __forceinline__ int64_t window_search(const DirEntry<K>* dir, int32_t wl, int32_t wh, K key, int gl,
                                                 int gbase, uint32_t* leaf) {
    int64_t cand = -1;
    uint32_t cleaf = kNone;
    for (int32_t base = wl; base <= wh; base += 2 * kLiG) {
        const int32_t e0 = base + 2 * gl, e1 = e0 + 1;
        DirEntry<K> d0, d1;
        d0.fence = kmax<K>(); d0.leaf = kNone;
        d1 = d0;
        if (e0 <= wh) d0 = dir[e0];
        if (e1 <= wh) d1 = dir[e1];
        const bool le0 = e0 <= wh && d0.fence <= key;
        const bool le1 = e1 <= wh && d1.fence <= key;
        const uint64_t m0 = group_bits<kLiG>(__ballot(le0), gbase);
        const uint64_t m1 = group_bits<kLiG>(__ballot(le1), gbase);
        int best = -1;  // local index 2*lane + e
        if (m1) best = 2 * (63 - __builtin_clzll(m1)) + 1;
        if (m0) {
            const int b0 = 2 * (63 - __builtin_clzll(m0));
            best = b0 > best ? b0 : best;
        }
        if (best >= 0) {
            const uint32_t l0 = shfl_u32(d0.leaf, gbase + best / 2);
            const uint32_t l1 = shfl_u32(d1.leaf, gbase + best / 2);
            cleaf = (best & 1) ? l1 : l0;
            cand = base + best;
        }
        // fences ascend: stop at the first chunk that holds a fence above the key
        const uint64_t gt0 = group_bits<kLiG>(__ballot(e0 <= wh && !le0), gbase);
        const uint64_t gt1 = group_bits<kLiG>(__ballot(e1 <= wh && !le1), gbase);
        if (gt0 | gt1) break;
    }
    *leaf = cleaf;
    return cand;
}

constexpr int kDirect = 8;  // leaves a group reads at once on the direct path

// Leaf verdict shared by both search paths: hit, authoritative miss (the
// leaf's first and last keys bracket the key), or neither.
template <class K>
struct Verdict {
    bool hit = false, bracket = false;
    K val = kmax<K>();
};

template <class K>
__device__ __forceinline__ void judge_leaf(const typename Trav<K, kLiG>::KV& kv, const typename Trav<K, kLiG>::KV& vv,
                                           K key, int gbase, Verdict<K>& v) {
    using T = Trav<K, kLiG>;
    const uint32_t slot = T::match_slot(kv, key, gbase);
    const K first = static_cast<K>(__shfl(kv.v[0], gbase, 64));
    const K last = static_cast<K>(__shfl(kv.v[T::KPL - 1], gbase + kLiG - 1, 64));
    const K x = T::pick_value(vv, slot < kSlots ? slot : 0u, gbase);
    if (slot < kSlots) {
        v.hit = true;
        v.val = x;
    }
    if (key >= first && key <= last) v.bracket = true;
}

template <class K, bool STAGE>
__global__ __launch_bounds__(kLiBlock) void k_li_lookup(TreeView<K> t, LiView<K> li, LiArgs a,
                                                        const K* __restrict__ q, uint64_t B, K* __restrict__ vout,
                                                        uint8_t* __restrict__ fout) {
    using T = Trav<K, kLiG>;
    extern __shared__ __align__(16) uint8_t lds[];
    const ModelLite* tab = li.lite;
    if constexpr (STAGE) {
        const uint4* src = reinterpret_cast<const uint4*>(li.lite);
        uint4* dst = reinterpret_cast<uint4*>(lds);
        for (uint32_t i = threadIdx.x; i < a.M * (sizeof(ModelLite) / 16); i += blockDim.x) dst[i] = src[i];
        __syncthreads();
        tab = reinterpret_cast<const ModelLite*>(lds);
    }
    const int lane = lane_id();
    const int gl = lane % kLiG, gbase = lane - gl;
    const uint64_t group = gid() / kLiG, ngroups = gsz() / kLiG;
    uint32_t nfb = 0;
    for (uint64_t i = group; i < B; i += ngroups) {
        const K key = q[i];
        const uint32_t j = root_index(a, static_cast<uint64_t>(key));
        const ModelLite m = tab[j];
        bool fb = m.kind == kKindTree;
        Verdict<K> v;
        if (!fb) {
            const float x = norm_x(static_cast<uint64_t>(key), m.kmin, m.scale);
            const float f = m.kind == kKindMlp ? mlp_eval_group(li.models + j, x, gl) : __fmaf_rn(m.slope, x, m.icpt);
            const int32_t p = clamp_pos(f, a.L);
            const int32_t lo = static_cast<int16_t>(m.lo_hi & 0xFFFF), hi = static_cast<int16_t>(m.lo_hi >> 16);
            int32_t wl = p + lo, wh = p + hi;
            if (wl < 0) wl = 0;
            if (wh > static_cast<int32_t>(a.L) - 1) wh = static_cast<int32_t>(a.L) - 1;
            if (a.identity) {
                // positions are leaf ids: read the window's leaves at once
                bool done = false;
                for (int32_t base = wl; base <= wh && !done; base += kDirect) {
                    typename T::KV kv[kDirect], vv[kDirect];
#pragma unroll
                    for (int u = 0; u < kDirect; ++u) {
                        if (base + u <= wh) {
                            kv[u] = T::load_keys(t.lkeys + static_cast<uint64_t>(base + u) * kSlots, gl);
                            vv[u] = T::load_keys(t.lvals + static_cast<uint64_t>(base + u) * kSlots, gl);
                        }
                    }
#pragma unroll
                    for (int u = 0; u < kDirect; ++u)
                        if (base + u <= wh) judge_leaf<K>(kv[u], vv[u], key, gbase, v);
                    done = v.hit || v.bracket;
                }
                fb = !(v.hit || v.bracket);
            } else {
                uint32_t leaf = kNone;
                const int64_t cand = window_search<K>(li.dir, wl, wh, key, gl, gbase, &leaf);
                if (cand < 0) {
                    if (wl == 0) leaf = li.dir[0].leaf;  // below every fence: the first leaf
                    else fb = true;
                }
                if (!fb) {
                    const typename T::KV kv = T::load_keys(t.lkeys + static_cast<uint64_t>(leaf) * kSlots, gl);
                    const typename T::KV vv = T::load_keys(t.lvals + static_cast<uint64_t>(leaf) * kSlots, gl);
                    judge_leaf<K>(kv, vv, key, gbase, v);
                    fb = !(v.hit || v.bracket);
                }
            }
        }
        if (fb) {
            // the tree decides: plain root-to-leaf walk
            K kk[1] = {key};
            uint32_t lf[1];
            descend<K, kLiG, 1, false>(t, t.mirror, kMirrorMaxNodes, 0, kk, lf, gl, gbase);
            const typename T::KV kv = T::load_keys(t.lkeys + static_cast<uint64_t>(lf[0]) * kSlots, gl);
            const typename T::KV vv = T::load_keys(t.lvals + static_cast<uint64_t>(lf[0]) * kSlots, gl);
            v = Verdict<K>();
            judge_leaf<K>(kv, vv, key, gbase, v);
            nfb += gl == 0 ? 1u : 0u;
        }
        if (gl == 0) {
            vout[i] = v.hit ? v.val : kmax<K>();
            fout[i] = v.hit ? 1 : 0;
        }
    }
    // counters: one atomic per wave
    uint64_t wsum = nfb;
    for (int d = 32; d > 0; d >>= 1) wsum += __shfl_xor(wsum, d, 64);
    if (lane == 0 && wsum) atomicAdd(&li.hdr->fallbacks, static_cast<unsigned long long>(wsum));
    if (gid() == 0) atomicAdd(&li.hdr->lookups, static_cast<unsigned long long>(B));
}

template <class K>
__global__ __launch_bounds__(kLiBlock) void k_li_predict(LiView<K> li, const K* __restrict__ q, uint64_t B,
                                                         uint32_t* mo, int32_t* po, int32_t* lo, int32_t* hi,
                                                         uint8_t* ko) {
    const LiHeader h = *li.hdr;
    const int gl = lane_id() % kLiG;
    const uint64_t group = gid() / kLiG, ngroups = gsz() / kLiG;
    for (uint64_t i = group; i < B; i += ngroups) {
        const uint64_t key = static_cast<uint64_t>(q[i]);
        const uint32_t j = root_index(h, key);
        const ModelRec* m = li.models + j;
        const uint32_t kind = m->kind;
        const int32_t p = kind == kKindTree ? 0 : predict(m, kind, key, h.L, gl);
        if (gl == 0) {
            mo[i] = j;
            po[i] = p;
            lo[i] = m->lo;
            hi[i] = m->hi;
            ko[i] = static_cast<uint8_t>(kind);
        }
    }
}

}  // namespace gt

// ------------------------------------------------------------------ host

using namespace gt;

struct gt_learned {
    gt_tree* t;
    gt_li_params p;
    uint32_t M;
    uint8_t* arena;
    uint64_t arena_bytes;
    bool trained;
    uint64_t leaf_cap;
    uint64_t off_models, off_dir, off_nxt0, off_nxt1, off_rank0, off_rank1, off_pos, off_start, off_bnd, off_cnt,
        off_partial, off_mlp, off_lite, off_ident;
    LiArgs args;
};

namespace {

uint64_t al256(uint64_t x) { return (x + 255) / 256 * 256; }

uint32_t models_of(const gt_li_params* p) { return p && p->models ? p->models : 1024u; }

uint64_t layout_li(gt_learned* li, uint64_t leaf_cap, uint32_t M, int kb) {
    uint64_t off = al256(sizeof(LiHeader));
    const uint64_t de = kb == 8 ? sizeof(DirEntry<uint64_t>) : sizeof(DirEntry<uint32_t>);
    uint64_t o_models = off; off += al256(static_cast<uint64_t>(M) * sizeof(ModelRec));
    uint64_t o_dir = off; off += al256((leaf_cap + 1) * de);
    uint64_t o_n0 = off; off += al256(leaf_cap * 4);
    uint64_t o_n1 = off; off += al256(leaf_cap * 4);
    uint64_t o_r0 = off; off += al256(leaf_cap * 4);
    uint64_t o_r1 = off; off += al256(leaf_cap * 4);
    uint64_t o_pos = off; off += al256(leaf_cap * 4);
    uint64_t o_start = off; off += al256((M + 1ull) * 4);
    uint64_t o_bnd = off; off += al256(4ull * M * 4);
    uint64_t o_cnt = off; off += al256(M * 4ull);
    uint64_t o_part = off; off += al256(kMaxPartials * 5ull * 8);
    uint64_t o_mlp = off; off += al256(M * 4ull);
    uint64_t o_lite = off; off += al256(static_cast<uint64_t>(M) * sizeof(ModelLite));
    uint64_t o_ident = off; off += 256;
    if (li) {
        li->off_lite = o_lite; li->off_ident = o_ident;
        li->off_models = o_models; li->off_dir = o_dir; li->off_nxt0 = o_n0; li->off_nxt1 = o_n1;
        li->off_rank0 = o_r0; li->off_rank1 = o_r1; li->off_pos = o_pos; li->off_start = o_start;
        li->off_bnd = o_bnd; li->off_cnt = o_cnt; li->off_partial = o_part; li->off_mlp = o_mlp;
    }
    return off;
}

template <class K>
LiView<K> li_view(const gt_learned* li) {
    LiView<K> v;
    uint8_t* a = li->arena;
    v.hdr = reinterpret_cast<LiHeader*>(a);
    v.models = reinterpret_cast<ModelRec*>(a + li->off_models);
    v.dir = reinterpret_cast<DirEntry<K>*>(a + li->off_dir);
    v.nxt0 = reinterpret_cast<uint32_t*>(a + li->off_nxt0);
    v.nxt1 = reinterpret_cast<uint32_t*>(a + li->off_nxt1);
    v.rank0 = reinterpret_cast<uint32_t*>(a + li->off_rank0);
    v.rank1 = reinterpret_cast<uint32_t*>(a + li->off_rank1);
    v.pos_of_leaf = reinterpret_cast<uint32_t*>(a + li->off_pos);
    v.start = reinterpret_cast<uint32_t*>(a + li->off_start);
    v.bnd = reinterpret_cast<int32_t*>(a + li->off_bnd);
    v.cnt = reinterpret_cast<uint32_t*>(a + li->off_cnt);
    v.partial = reinterpret_cast<double*>(a + li->off_partial);
    v.mlp_ok = reinterpret_cast<float*>(a + li->off_mlp);
    v.lite = reinterpret_cast<ModelLite*>(a + li->off_lite);
    v.identity = reinterpret_cast<uint32_t*>(a + li->off_ident);
    return v;
}

uint32_t grid_of(uint64_t n, uint32_t block, uint32_t cap = 16384) {
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return static_cast<uint32_t>(g);
}

#define LI_HIP(x)                                 \
    do {                                          \
        if ((x) != hipSuccess) return GT_ERR_HIP; \
    } while (0)

template <class K>
gt_status train_t(gt_learned* li, hipStream_t s) {
    gt_tree* t = li->t;
    DevHeader dh;
    LI_HIP(hipMemcpyAsync(&dh, t->hdr, sizeof dh, hipMemcpyDeviceToHost, s));
    LI_HIP(hipStreamSynchronize(s));
    const uint32_t M = li->M;
    LiView<K> v = li_view<K>(li);
    TreeView<K> tv = view<K>(t);
    if (dh.n_keys == 0) {
        LI_HIP(hipMemsetAsync(v.hdr, 0, sizeof(LiHeader), s));
        LI_HIP(hipStreamSynchronize(s));
        li->trained = false;
        return GT_OK;
    }
    const uint32_t n = dh.leaf_used;
    if (n > li->leaf_cap) return GT_ERR_CAPACITY;
    hipLaunchKernelGGL(k_rank_init, dim3(grid_of(n, 256)), dim3(256), 0, s, t->lmeta, n, v.nxt0, v.rank0);
    uint32_t* ni = v.nxt0; uint32_t* ri = v.rank0; uint32_t* no = v.nxt1; uint32_t* ro = v.rank1;
    for (uint64_t span = 1; span < n; span <<= 1) {
        hipLaunchKernelGGL(k_rank_jump, dim3(grid_of(n, 256)), dim3(256), 0, s, ni, ri, no, ro, n);
        uint32_t* a = ni; ni = no; no = a;
        uint32_t* b = ri; ri = ro; ro = b;
    }
    hipLaunchKernelGGL(k_directory<K>, dim3(grid_of(n, 256)), dim3(256), 0, s, tv, v, ri, n);
    // root normalisation: smallest first key .. largest key of the tree
    DirEntry<K> d0;
    LI_HIP(hipMemcpyAsync(&d0, v.dir, sizeof d0, hipMemcpyDeviceToHost, s));
    uint32_t last_leaf_pos = n - 1;
    DirEntry<K> dl;
    LI_HIP(hipMemcpyAsync(&dl, v.dir + last_leaf_pos, sizeof dl, hipMemcpyDeviceToHost, s));
    LI_HIP(hipStreamSynchronize(s));
    K kmaxkey;
    LI_HIP(hipMemcpyAsync(&kmaxkey, tv.lkeys + static_cast<uint64_t>(dl.leaf) * kSlots + kSlots - 1, sizeof(K),
                          hipMemcpyDeviceToHost, s));
    LI_HIP(hipStreamSynchronize(s));
    const uint64_t kmin = static_cast<uint64_t>(d0.fence), kmx = static_cast<uint64_t>(kmaxkey);
    const double scale = kmx > kmin ? 1.0 / static_cast<double>(kmx - kmin) : 1.0;
    const uint32_t nb = n < static_cast<uint32_t>(kMaxPartials) ? (n < 1 ? 1 : n) : kMaxPartials;
    hipLaunchKernelGGL(k_root_partial<K>, dim3(nb), dim3(256), 0, s, v, n, M, kmin, scale);
    hipLaunchKernelGGL(k_root_final<K>, dim3(1), dim3(64), 0, s, v, nb, kmin, scale, n, M);
    hipLaunchKernelGGL(k_ranges<K>, dim3(grid_of(n, 256)), dim3(256), 0, s, v, n, M);
    hipLaunchKernelGGL(k_fit<K>, dim3(M), dim3(256), 0, s, v, M);
    hipLaunchKernelGGL(k_bounds_init, dim3(grid_of(M, 256)), dim3(256), 0, s, v.bnd, v.cnt, M);
    hipLaunchKernelGGL(k_bounds<K>, dim3(grid_of(static_cast<uint64_t>(n) * kSlots * kLiG, kLiBlock, 8192)),
                       dim3(kLiBlock), 0, s, tv, v, n);
    uint32_t mw = li->p.max_window ? li->p.max_window : 64u;
    if (mw > 4096u) mw = 4096u;  // windows are packed in 16 bits
    hipLaunchKernelGGL(k_choose<K>, dim3(grid_of(M, 256)), dim3(256), 0, s, v, M, li->p.kind, mw);
    hipLaunchKernelGGL(k_li_finish<K>, dim3(1), dim3(64), 0, s, v, dh.n_keys);
    const uint32_t one = 1;
    LI_HIP(hipMemcpyAsync(v.identity, &one, 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_identity, dim3(grid_of(n, 256)), dim3(256), 0, s, v.pos_of_leaf, n, v.identity);
    if (hipGetLastError() != hipSuccess) return GT_ERR_HIP;
    LiHeader h;
    uint32_t ident = 0;
    LI_HIP(hipMemcpyAsync(&h, v.hdr, sizeof h, hipMemcpyDeviceToHost, s));
    LI_HIP(hipMemcpyAsync(&ident, v.identity, 4, hipMemcpyDeviceToHost, s));
    LI_HIP(hipStreamSynchronize(s));
    li->args.kmin_root = h.kmin_root;
    li->args.root_scale = h.root_scale;
    li->args.root_a = h.root_a;
    li->args.root_b = h.root_b;
    li->args.L = h.L;
    li->args.M = h.M;
    li->args.identity = (li->p.search == 2) ? ident : 0u;
    li->args.pad = 0;
    li->trained = true;
    return GT_OK;
}

}  // namespace

extern "C" {

uint64_t li_arena_bytes(const gt_tree* t, const gt_li_params* p) {
    if (!t) return 0;
    if (p && (p->models > 4096 || p->kind > 2 || p->search > 2 || p->stage > 2 || p->reserved[0] || p->reserved[1]))
        return 0;
    return layout_li(nullptr, t->leaf_cap, models_of(p), t->kb);
}

gt_status li_create(gt_tree* t, const gt_li_params* p, void* arena, uint64_t arena_bytes, gt_learned** out) {
    if (!t || !arena || !out) return GT_ERR_INVALID;
    if (p && (p->models > 4096 || p->kind > 2 || p->search > 2 || p->stage > 2 || p->reserved[0] || p->reserved[1]))
        return GT_ERR_INVALID;
    const uint32_t M = models_of(p);
    if (layout_li(nullptr, t->leaf_cap, M, t->kb) > arena_bytes) return GT_ERR_CAPACITY;
    gt_learned* li = new gt_learned();
    li->t = t;
    if (p) li->p = *p;
    li->M = M;
    li->arena = reinterpret_cast<uint8_t*>(arena);
    li->leaf_cap = t->leaf_cap;
    li->arena_bytes = layout_li(li, t->leaf_cap, M, t->kb);
    li->trained = false;
    if (hipMemset(arena, 0, sizeof(LiHeader)) != hipSuccess) {
        delete li;
        return GT_ERR_HIP;
    }
    *out = li;
    return GT_OK;
}

gt_status li_train(gt_learned* li, hipStream_t stream) {
    if (!li) return GT_ERR_INVALID;
    return li->t->kb == 8 ? train_t<uint64_t>(li, stream) : train_t<uint32_t>(li, stream);
}

gt_status li_lookup_batch(gt_learned* li, const void* keys, uint64_t B, void* values_out, uint8_t* found_out,
                          hipStream_t stream) {
    if (!li) return GT_ERR_INVALID;
    if (B == 0) return GT_OK;
    if (!keys || !values_out || !found_out) return GT_ERR_INVALID;
    if (!li->trained) return tree_lookup_batch(li->t, keys, B, values_out, found_out, stream);
    const uint32_t grid = grid_of(B * kLiG, kLiBlock, 2048);
    // the model table goes to LDS when it is small; large batches keep it in
    // L2, where the staging would cost more than it saves
    const uint32_t lds = li->M * static_cast<uint32_t>(sizeof(ModelLite));
    const bool stage = li->p.stage == 1 && lds <= 48u * 1024u && B <= (1u << 16);
    if (li->t->kb == 8) {
        if (stage)
            hipLaunchKernelGGL((k_li_lookup<uint64_t, true>), dim3(grid), dim3(kLiBlock), lds, stream,
                               view<uint64_t>(li->t), li_view<uint64_t>(li), li->args,
                               reinterpret_cast<const uint64_t*>(keys), B, reinterpret_cast<uint64_t*>(values_out),
                               found_out);
        else
            hipLaunchKernelGGL((k_li_lookup<uint64_t, false>), dim3(grid), dim3(kLiBlock), 0, stream,
                               view<uint64_t>(li->t), li_view<uint64_t>(li), li->args,
                               reinterpret_cast<const uint64_t*>(keys), B, reinterpret_cast<uint64_t*>(values_out),
                               found_out);
    } else {
        if (stage)
            hipLaunchKernelGGL((k_li_lookup<uint32_t, true>), dim3(grid), dim3(kLiBlock), lds, stream,
                               view<uint32_t>(li->t), li_view<uint32_t>(li), li->args,
                               reinterpret_cast<const uint32_t*>(keys), B, reinterpret_cast<uint32_t*>(values_out),
                               found_out);
        else
            hipLaunchKernelGGL((k_li_lookup<uint32_t, false>), dim3(grid), dim3(kLiBlock), 0, stream,
                               view<uint32_t>(li->t), li_view<uint32_t>(li), li->args,
                               reinterpret_cast<const uint32_t*>(keys), B, reinterpret_cast<uint32_t*>(values_out),
                               found_out);
    }
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status li_predict(gt_learned* li, const void* keys, uint64_t B, uint32_t* model_out, int32_t* pred_out,
                     int32_t* lo_out, int32_t* hi_out, uint8_t* kind_out, hipStream_t stream) {
    if (!li || (B && (!keys || !model_out || !pred_out || !lo_out || !hi_out || !kind_out))) return GT_ERR_INVALID;
    if (!li->trained) return GT_ERR_INVALID;
    if (B == 0) return GT_OK;
    const uint32_t grid = grid_of(B * kLiG, kLiBlock, 2048);
    if (li->t->kb == 8)
        hipLaunchKernelGGL(k_li_predict<uint64_t>, dim3(grid), dim3(kLiBlock), 0, stream, li_view<uint64_t>(li),
                           reinterpret_cast<const uint64_t*>(keys), B, model_out, pred_out, lo_out, hi_out, kind_out);
    else
        hipLaunchKernelGGL(k_li_predict<uint32_t>, dim3(grid), dim3(kLiBlock), 0, stream, li_view<uint32_t>(li),
                           reinterpret_cast<const uint32_t*>(keys), B, model_out, pred_out, lo_out, hi_out, kind_out);
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status li_set_bounds(gt_learned* li, int32_t lo, int32_t hi, hipStream_t stream) {
    if (!li || lo > hi) return GT_ERR_INVALID;
    if (lo < -30000 || hi > 30000) return GT_ERR_INVALID;
    hipLaunchKernelGGL(k_set_bounds, dim3(grid_of(li->M, 256)), dim3(256), 0, stream,
                       reinterpret_cast<ModelRec*>(li->arena + li->off_models),
                       reinterpret_cast<ModelLite*>(li->arena + li->off_lite), li->M, lo, hi);
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status li_stats(gt_learned* li, gt_li_stats* out, hipStream_t stream) {
    if (!li || !out) return GT_ERR_INVALID;
    LiHeader h;
    std::vector<ModelRec> ms(li->M);
    LI_HIP(hipMemcpyAsync(&h, li->arena, sizeof h, hipMemcpyDeviceToHost, stream));
    LI_HIP(hipMemcpyAsync(ms.data(), li->arena + li->off_models, ms.size() * sizeof(ModelRec), hipMemcpyDeviceToHost,
                          stream));
    LI_HIP(hipStreamSynchronize(stream));
    memset(out, 0, sizeof *out);
    out->trained_leaves = li->trained ? h.L : 0;
    out->trained_keys = li->trained ? h.n_keys : 0;
    out->lookups = h.lookups;
    out->fallbacks = h.fallbacks;
    out->models = li->M;
    double wsum = 0;
    uint32_t used = 0;
    for (const ModelRec& m : ms) {
        if (!li->trained) break;
        if (m.kind == kKindLinear) out->linear_models++;
        else if (m.kind == kKindMlp) out->mlp_models++;
        else out->tree_models++;
        if (m.kind != kKindTree) {
            const uint32_t w = static_cast<uint32_t>(m.hi - m.lo + 1);
            wsum += w;
            used++;
            if (w > out->max_window) out->max_window = w;
        }
    }
    out->mean_window = used ? wsum / used : 0.0;
    return GT_OK;
}

gt_status li_destroy(gt_learned* li) {
    if (!li) return GT_ERR_INVALID;
    delete li;
    return GT_OK;
}

}  // extern "C"
