// Learned index over the tree: training and lookup kernels.
//
// Model.  Stage 1 (root): f = a (key - kmin) + c, evaluated in FP64;
// j = clamp(floor(f), 0, M-1) picks the leaf model and x = f - j, rounded to
// FP32, is that model's input: the key's place inside the model's share of
// the key range.  Stage 2 (leaf model j), FP32: either a line p = s x + t or
// a one-hidden-layer ReLU network with 32 units,
//     p = w_b + w_0 x + sum_{u=1..31} w_u relu(x - u/32)
// (unit 0's knot sits at the left end of the model's range, where relu(x)
// and x agree).  With its knots on the uniform grid u/32 the network is
// linear on every piece [m/32, (m+1)/32), so it is stored and evaluated as
// 32 (slope, intercept) pairs selected by m = clamp(floor(32 x), 0, 31):
// the same function, one fused multiply-add per query, and one 16-byte
// record per piece that also carries the piece's exact error bounds.  A
// linear model fills its 32 pieces with the same line.  The prediction is
// a leaf position in key order (the leaf chain at training time).
//
// Training (all on the device, deterministic reduction orders):
//   leaf positions   the tree expanded level by level from the root (each
//                    level's nodes in key order, so the last level lists
//                    the leaves in key order, the order of the leaf chain)
//   directory        dir[pos] = (first key of the leaf, leaf id)
//   root             least squares of pos*M/L on the fences (FP64 sums)
//   model ranges     the root is monotone, so model j owns a contiguous run
//                    of fences; one fence on either side anchors its fit
//   leaf models      least squares on those fences in FP64: the line, and
//                    the network's output layer from the normal equations
//                    (Cholesky)
//   bounds           every key of the tree goes through the same piece
//                    evaluation the lookup runs; per piece and model kind,
//                    lo / hi are the exact min / max of (true position -
//                    prediction) over the keys routed there
//   choice           per model, the kind with the smaller key-weighted
//                    window; a piece whose window exceeds the limit sends
//                    its keys down the tree
//
// Lookup: route, read the piece, clamp the window [p + lo, p + hi].  On a
// bulk-loaded tree (directory = identity: position i is leaf i) small
// batches read the window's leaves at once (latency: one dependent access
// after the piece); otherwise, and for large batches (bound by the rate of
// line requests, where reading 3-4 leaves per query costs more than a
// fence search), the last fence <= key in the window picks the leaf.  A
// match is a hit.  While the tree is unchanged since training and the
// bounds are the trained ones, every present key lies in its window, so a
// window without the key proves it absent.  Otherwise (after inserts, after
// the bounds were overwritten, in a piece without bounds) a query whose
// window does not hold it walks the tree in the same kernel.  Results equal
// the tree's for any model state.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>
#include <vector>
#include <cmath>
#include <algorithm>
#include <utility>

#include "../../include/gtree.h"
#include "common.h"
#include "traverse.h"
#include "handle.h"
#include "prims.h"

namespace gt {

constexpr int kSeg = 32;                          // hidden units = pieces per leaf model
constexpr int kLiG = 8;                           // lanes per query
constexpr int kLiBlock = 256;
constexpr uint32_t kKindLinear = 0, kKindMlp = 1, kKindTree = 2;
constexpr int kFitPoints = 4096;                  // points per model for the network fit
constexpr int kDirect = 4;                        // leaves a group reads at once on the direct path
constexpr uint32_t kDirectMaxWin = 16;            // direct reads only while every window is this narrow
constexpr int kWalkMax = 4;                       // leaves a stale miss may follow along the chain
constexpr double kGateTreeShare = 0.25;           // decline: more of the keys go down the tree than this
constexpr double kGateMeanWindow = 16.0;          // decline: a wider key-weighted mean window (leaves)
constexpr uint64_t kDirectMaxBatch = 1ull << 13;   // default: direct window reads up to this batch
constexpr uint64_t kSmallLookup = 1ull << 13;      // batches up to this size use 64-thread workgroups

struct LiHeader {
    uint64_t kmin_root;
    double root_a, root_c;
    uint32_t L;          // leaves in the directory
    uint32_t M;
    uint64_t n_keys;
    unsigned long long lookups, fallbacks;
    uint32_t trained;
    uint32_t epoch;      // tree epoch at training
    unsigned long long keys_tree;    // trained keys whose piece sends them down the tree
    unsigned long long window_sum;   // sum over the other keys of their piece's window (leaves)
    uint32_t max_win;                // widest window of a piece that holds keys
    uint32_t pad[43];
};
static_assert(sizeof(LiHeader) == 256, "LiHeader size");

// One piece of a leaf model as the lookup reads it.  Prediction:
// base + floor(slope * x + icpt), clamped to the directory; lo > hi marks a
// piece whose keys go down the tree.
struct alignas(16) Piece {
    float slope, icpt;
    int16_t lo, hi;
    uint32_t base;
};
static_assert(sizeof(Piece) == 16, "Piece size");

// Training record of one leaf model: both candidate kinds.
struct ModelFit {
    float lin_s, lin_t;   // the line, relative to base
    uint32_t base;        // position offset of the model's predictions
    uint32_t kind;        // kind in use after the choice
    uint32_t n_keys;      // keys routed here
    uint32_t mlp_ok;      // network fitted
    uint32_t pad[2];
    float A[kSeg];        // network pieces: slopes
    float C[kSeg];        // and intercepts, relative to base
};
static_assert(sizeof(ModelFit) == 288, "ModelFit size");

template <class K>
struct alignas(sizeof(K) == 8 ? 16 : 8) DirEntry {
    K fence;
    uint32_t leaf;
};
static_assert(sizeof(DirEntry<uint64_t>) == 16 && sizeof(DirEntry<uint32_t>) == 8, "DirEntry size");

// Root parameters, passed to the lookup by value (no dependent header load).
struct LiArgs {
    uint64_t kmin;
    double a, c;
    uint32_t L, M;
    uint32_t epoch;      // tree epoch at training
    uint32_t identity;   // directory position == leaf id for every position
    uint32_t exact;      // bounds are the trained ones (not overwritten)
    uint32_t pad;
};

template <class K>
struct LiView {
    LiHeader* hdr;
    ModelFit* fit;         // M
    Piece* piece;          // M * kSeg
    uint32_t* identity;
    DirEntry<K>* dir;      // L + 1 (the last entry: largest key, no leaf)
    uint32_t* nxt0; uint32_t* nxt1; uint32_t* rank0; uint32_t* rank1;  // training scratch
    uint32_t* lvl;         // kMaxLevels: nodes per tree level while positions are computed
    void* scan_tmp;
    uint32_t* pos_of_leaf;
    uint32_t* start;       // M + 1
    int32_t* bnd;          // 4 per piece: lo, hi of the line; lo, hi of the network
    uint32_t* cnt;         // keys per piece
    double* partial;       // kMaxPartials * 5
};

constexpr int kMaxPartials = 4096;

// ------------------------------------------------------------ inference

// key - kmin in FP64 on either side of kmin (u64 differences can exceed the
// int64 range)
__device__ __forceinline__ double key_diff(uint64_t key, uint64_t kmin) {
    return key >= kmin ? static_cast<double>(key - kmin) : -static_cast<double>(kmin - key);
}

struct Route {
    uint32_t j, m;
    float x;
};

__device__ __forceinline__ uint32_t piece_of(float x) {
    const float s = floorf(x * static_cast<float>(kSeg));
    return static_cast<uint32_t>(fminf(fmaxf(s, 0.0f), static_cast<float>(kSeg - 1)));
}

__device__ __forceinline__ Route route(const LiArgs& a, uint64_t key) {
    const double f = fma(a.a, key_diff(key, a.kmin), a.c);
    const double fj = fmin(fmax(floor(f), 0.0), static_cast<double>(a.M - 1));
    Route r;
    r.j = static_cast<uint32_t>(fj);
    r.x = static_cast<float>(f - fj);
    r.m = piece_of(r.x);
    return r;
}

// model j's input for any key (equal to route().x for the keys routed to j)
__device__ __forceinline__ float x_in(const LiArgs& a, uint32_t j, uint64_t key) {
    return static_cast<float>(fma(a.a, key_diff(key, a.kmin), a.c) - static_cast<double>(j));
}

__device__ __forceinline__ int32_t piece_pos(float slope, float icpt, uint32_t base, float x, uint32_t L) {
    float f = __fmaf_rn(slope, x, icpt);
    f = fminf(fmaxf(f, -1.0e9f), 1.0e9f);
    int64_t p = static_cast<int64_t>(base) + static_cast<int64_t>(floorf(f));
    if (p < 0) p = 0;
    if (p > static_cast<int64_t>(L) - 1) p = static_cast<int64_t>(L) - 1;
    return static_cast<int32_t>(p);
}

__device__ __forceinline__ Piece load_piece(const Piece* tab, uint32_t j, uint32_t m) {
    const uint4 raw = *reinterpret_cast<const uint4*>(tab + (static_cast<uint64_t>(j) * kSeg + m));
    Piece e;
    __builtin_memcpy(&e, &raw, sizeof e);
    return e;
}

__device__ __forceinline__ LiArgs args_of(const LiHeader* h) {
    LiArgs a;
    a.kmin = h->kmin_root;
    a.a = h->root_a;
    a.c = h->root_c;
    a.L = h->L;
    a.M = h->M;
    a.epoch = h->epoch;
    a.identity = 0;
    a.exact = 0;
    a.pad = 0;
    return a;
}

// ------------------------------------------------------------- training

__device__ __forceinline__ uint64_t gid() { return blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; }
__device__ __forceinline__ uint64_t gsz() { return static_cast<uint64_t>(gridDim.x) * blockDim.x; }

// Leaf positions in key order, by expanding the tree from the root one level
// at a time: a level's nodes are listed in key order, so their children,
// taken node after node in slot order, are the next level in key order, and
// the last expansion gives each leaf its position.  Sixteen lanes per node
// read its child line; the level's size stays on the device.
__global__ void k_bfs_init(uint32_t* list, uint32_t* m_dev, uint32_t root, uint32_t* pos, uint32_t root_is_leaf) {
    if (gid() == 0) {
        list[0] = root;
        m_dev[0] = 1;
        if (root_is_leaf) pos[root & ~kLeafTag] = 0;
    }
}

__global__ void k_bfs_count(const uint32_t* __restrict__ ichild, const uint32_t* __restrict__ list,
                            const uint32_t* __restrict__ m_dev, uint32_t* __restrict__ cnt) {
    const uint64_t m16 = static_cast<uint64_t>(*m_dev) * kSlots;
    for (uint64_t g = gid(); g < m16; g += gsz()) {
        const uint64_t i = g / kSlots;
        const uint32_t sl = static_cast<uint32_t>(g % kSlots);
        const bool has = ichild[static_cast<uint64_t>(list[i]) * kSlots + sl] != kNone;
        const uint64_t m = __ballot(has);
        const int lane = lane_id(), gb = lane & ~(kSlots - 1);
        if (sl == 0) cnt[i] = static_cast<uint32_t>(__popcll((m >> gb) & 0xFFFFull));
    }
}

__global__ void k_bfs_scatter(const uint32_t* __restrict__ ichild, const uint32_t* __restrict__ list,
                              const uint32_t* __restrict__ m_dev, const uint32_t* __restrict__ cnt,
                              const uint32_t* __restrict__ off, uint32_t* __restrict__ next,
                              uint32_t* __restrict__ pos, uint32_t last) {
    const uint64_t m16 = static_cast<uint64_t>(*m_dev) * kSlots;
    for (uint64_t g = gid(); g < m16; g += gsz()) {
        const uint64_t i = g / kSlots;
        const uint32_t sl = static_cast<uint32_t>(g % kSlots);
        if (sl < cnt[i]) {
            const uint32_t ref = ichild[static_cast<uint64_t>(list[i]) * kSlots + sl];
            if (last) pos[ref & ~kLeafTag] = off[i] + sl;
            else next[off[i] + sl] = ref;
        }
    }
}

__global__ void k_pos_clear(uint32_t* pos, uint32_t n) {
    for (uint64_t i = gid(); i < n; i += gsz()) pos[i] = kNone;
}

// Directory entry per leaf position.  Leaf ids run to `ids`; the L leaves the
// walk from the root reached hold positions 0..L-1, the others (leaves a
// delete's merge gave up) keep "none" and are skipped.
template <class K>
__global__ void k_directory(TreeView<K> t, LiView<K> li, uint32_t ids, uint32_t L) {
    for (uint64_t i = gid(); i < ids; i += gsz()) {
        const uint32_t pos = li.pos_of_leaf[i];
        if (pos >= L) continue;
        DirEntry<K> e;
        e.fence = t.lkeys[i * kSlots];
        e.leaf = static_cast<uint32_t>(i);
        li.dir[pos] = e;
    }
    if (gid() == 0) {
        DirEntry<K> e;
        e.fence = kmax<K>();
        e.leaf = kNone;
        li.dir[L] = e;
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

// root sums: block b covers fences [b*n/nb, (b+1)*n/nb); x = (fence - kmin) * scale
template <class K>
__global__ __launch_bounds__(256) void k_root_partial(LiView<K> li, uint32_t L, uint32_t M, uint64_t kmin,
                                                      double scale) {
    __shared__ double sh[256];
    const uint64_t b0 = part_start(blockIdx.x, L, gridDim.x), b1 = part_start(blockIdx.x + 1, L, gridDim.x);
    double s[5] = {0, 0, 0, 0, 0};
    for (uint64_t p = b0 + threadIdx.x; p < b1; p += blockDim.x) {
        const double x = key_diff(static_cast<uint64_t>(li.dir[p].fence), kmin) * scale;
        const double y = static_cast<double>(p) * M / L;
        s[0] += 1.0; s[1] += x; s[2] += y; s[3] += x * x; s[4] += x * y;
    }
    for (int k = 0; k < 5; ++k) {
        const double r = block_sum(s[k], sh);
        if (threadIdx.x == 0) li.partial[blockIdx.x * 5 + k] = r;
    }
}

// f = a' x + c with x = (key - kmin) * scale, stored as a = a' * scale.
// One workgroup of 256: strided partial sums, then the fixed-order tree.
template <class K>
__global__ __launch_bounds__(256) void k_root_final(LiView<K> li, uint32_t nb, uint64_t kmin, double scale,
                                                    uint32_t L, uint32_t M, uint32_t epoch) {
    __shared__ double sh[256];
    double s[5] = {0, 0, 0, 0, 0};
    for (uint32_t b = threadIdx.x; b < nb; b += blockDim.x)
        for (int k = 0; k < 5; ++k) s[k] += li.partial[b * 5 + k];
    for (int k = 0; k < 5; ++k) s[k] = block_sum(s[k], sh);
    if (threadIdx.x != 0) return;
    const double n = s[0], den = n * s[3] - s[1] * s[1];
    double a = den > 0 ? (n * s[4] - s[1] * s[2]) / den : 0.0;
    if (!(a > 0)) a = 0.0;
    const double c = n > 0 ? (s[2] - a * s[1]) / n : 0.0;
    LiHeader* h = li.hdr;
    h->kmin_root = kmin;
    h->root_a = a * scale;
    h->root_c = c;
    h->L = L;
    h->M = M;
    h->epoch = epoch;
}

// model j owns fences [start[j], start[j+1])
template <class K>
__global__ void k_ranges(LiView<K> li, uint32_t L, uint32_t M) {
    const LiArgs a = args_of(li.hdr);
    for (uint64_t p = gid(); p < L; p += gsz()) {
        const uint32_t j = route(a, static_cast<uint64_t>(li.dir[p].fence)).j;
        const int64_t jp = p ? static_cast<int64_t>(route(a, static_cast<uint64_t>(li.dir[p - 1].fence)).j) : -1;
        for (int64_t jj = jp + 1; jj <= static_cast<int64_t>(j); ++jj) li.start[jj] = static_cast<uint32_t>(p);
        if (p + 1 == L)
            for (uint32_t jj = j + 1; jj <= M; ++jj) li.start[jj] = L;
    }
}

// Solve G w = r (G symmetric positive definite, n <= 64, row-major in LDS)
// by one wave: Cholesky right-looking (step j takes the pivot, scales column
// j below it and updates the trailing lower triangle, its elements dealt
// over the lanes), then the two triangular solves with r held one entry per
// lane.  A small ridge (relative to the mean diagonal) keeps G definite.
// One wave's LDS accesses take effect in order, so no barrier is needed
// between the steps.  Returns false (uniformly) when a pivot is not positive.
__device__ bool cholesky_solve_wave(double* G, double* r, int n) {
    const int lane = lane_id();
    double dg = lane < n ? G[lane * n + lane] : 0.0;
    for (int o = 32; o > 0; o >>= 1) dg += __shfl_xor(dg, o, 64);
    const double ridge = 1e-10 * (dg / n) + 1e-12;
    if (lane < n) G[lane * n + lane] += ridge;
    __builtin_amdgcn_wave_barrier();
    for (int j = 0; j < n; ++j) {
        const double pv = G[j * n + j];
        if (!(pv > 0)) return false;
        const double dj = sqrt(pv);
        if (lane > j && lane < n) G[lane * n + j] /= dj;
        if (lane == j) G[j * n + j] = dj;
        __builtin_amdgcn_wave_barrier();
        const int m = n - j - 1, cnt = m * (m + 1) / 2;
        for (int e = lane; e < cnt; e += 64) {
            // e -> (ii, kk), kk <= ii, row-major over the trailing triangle
            int ii = static_cast<int>((sqrt(8.0 * e + 1.0) - 1.0) * 0.5);
            if ((ii + 1) * (ii + 2) / 2 <= e) ++ii;
            if (ii * (ii + 1) / 2 > e) --ii;
            const int kk = e - ii * (ii + 1) / 2;
            const int i = j + 1 + ii, k = j + 1 + kk;
            G[i * n + k] -= G[i * n + j] * G[k * n + j];
        }
        __builtin_amdgcn_wave_barrier();
    }
    double ri = lane < n ? r[lane] : 0.0;
    for (int k = 0; k < n; ++k) {  // L y = r
        const double yk = __shfl(ri, k, 64) / G[k * n + k];
        if (lane == k) ri = yk;
        else if (lane > k && lane < n) ri -= G[lane * n + k] * yk;
    }
    for (int k = n - 1; k >= 0; --k) {  // L^T w = y
        const double wk = __shfl(ri, k, 64) / G[k * n + k];
        if (lane == k) ri = wk;
        else if (lane < k) ri -= G[k * n + lane] * wk;
    }
    if (lane < n) r[lane] = ri;
    return true;
}

// feature u of the network at x: unit 0 is x, units 1..31 relu(x - u/32),
// feature 32 the bias
__device__ __forceinline__ double feature(int u, double x) {
    if (u == 0) return x;
    if (u < kSeg) return fmax(0.0, x - static_cast<double>(u) / kSeg);
    return 1.0;
}

// One workgroup per model: the line and the network, fitted to the fences
// of the model's run and its two neighbours, targets relative to `base`.
template <class K>
__global__ __launch_bounds__(256) void k_fit(LiView<K> li, uint32_t L, uint32_t M) {
    constexpr int NF = kSeg + 1;
    __shared__ double sh[256];
    __shared__ float xs[kFitPoints];
    __shared__ float ys[kFitPoints];
    __shared__ double G[NF * NF];
    __shared__ double rr[NF];
    __shared__ int solved;
    const uint32_t j = blockIdx.x;
    if (j >= M) return;
    const LiArgs a = args_of(li.hdr);
    ModelFit* mf = li.fit + j;
    const uint32_t b = li.start[j], e = li.start[j + 1];
    const uint32_t p0 = b > 0 ? b - 1 : 0;
    const uint32_t p1 = e < L ? e : L - 1;  // inclusive, >= p0
    const uint32_t np = p1 - p0 + 1;
    // line: least squares over every point
    double s[5] = {0, 0, 0, 0, 0};
    for (uint32_t p = p0 + threadIdx.x; p <= p1; p += blockDim.x) {
        const double x = x_in(a, j, static_cast<uint64_t>(li.dir[p].fence));
        const double y = static_cast<double>(p - p0);
        s[0] += 1.0; s[1] += x; s[2] += y; s[3] += x * x; s[4] += x * y;
    }
    for (int k = 0; k < 5; ++k) s[k] = block_sum(s[k], sh);
    const double den = s[0] * s[3] - s[1] * s[1];
    const double slope = den > 1e-12 * s[0] * s[3] ? (s[0] * s[4] - s[1] * s[2]) / den : 0.0;
    const double icpt = (s[2] - slope * s[1]) / s[0];
    // network: up to kFitPoints evenly spaced points
    const uint32_t nq = np < static_cast<uint32_t>(kFitPoints) ? np : static_cast<uint32_t>(kFitPoints);
    for (uint32_t i = threadIdx.x; i < nq; i += blockDim.x) {
        const uint32_t p = p0 + static_cast<uint32_t>(part_start(i, np, nq));
        xs[i] = x_in(a, j, static_cast<uint64_t>(li.dir[p].fence));
        ys[i] = static_cast<float>(p - p0);
    }
    if (threadIdx.x == 0) solved = 0;
    __syncthreads();
    if (nq >= 8) {
        constexpr int NT = NF * (NF + 1) / 2;
        // The points come in increasing x (fences in key order through one
        // monotone map), and the features are x, relu(x - u/32) and 1, so
        // every normal-equation entry is a polynomial in five suffix sums
        // over the points beyond a knot b: S0, S1, S2 (powers of x), T0, T1
        // (y and x y).  For knots a <= b:
        //   sum x relu(x-b) = S2(b) - b S1(b),  sum relu(x-b) = S1(b) - b S0(b),
        //   sum relu(x-a) relu(x-b) = S2(b) - (a+b) S1(b) + a b S0(b),
        //   sum relu(x-b) y = T1(b) - b T0(b).
        // Each thread sums kPer consecutive points; a block scan of those
        // sums plus a short run inside one thread's points gives the prefix
        // at each knot's first point beyond it (fixed order, so repeatable).
        // Points out of order (never expected) fall back to direct sums.
        constexpr int kPer = kFitPoints / 256;  // the workgroup is 256 threads
        static_assert(kFitPoints % 256 == 0, "whole runs per thread");
        __shared__ double tp[5][257];
        __shared__ double suf[5][kSeg];
        const uint32_t t0 = threadIdx.x * kPer;
        bool unsorted = false;
        double qs[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int k = 0; k < kPer; ++k) {
            const uint32_t i = t0 + k;
            if (i < nq) {
                const double x = xs[i], y = ys[i];
                qs[0] += 1.0; qs[1] += x; qs[2] += x * x; qs[3] += y; qs[4] += x * y;
                if (i + 1 < nq && xs[i + 1] < xs[i]) unsorted = true;
            }
        }
        if (__syncthreads_or(unsorted ? 1 : 0) == 0) {
            for (int c = 0; c < 5; ++c) {
                double tot;
                const double ex = block_excl_scan<double>(qs[c], sh, &tot);
                tp[c][threadIdx.x] = ex;
                if (threadIdx.x == 0) tp[c][256] = tot;
            }
            __syncthreads();
            if (threadIdx.x < static_cast<unsigned>(kSeg)) {
                const int u = threadIdx.x;
                uint32_t idx = 0;  // first point beyond knot u/32 (u = 0: all points)
                if (u > 0) {
                    const double b = static_cast<double>(u) / kSeg;
                    uint32_t lo = 0, hi = nq;
                    while (lo < hi) {
                        const uint32_t mid = (lo + hi) >> 1;
                        if (static_cast<double>(xs[mid]) > b) hi = mid;
                        else lo = mid + 1;
                    }
                    idx = lo;
                }
                const uint32_t tr = idx / kPer;
                double pre[5];
                for (int c = 0; c < 5; ++c) pre[c] = tp[c][tr];
                for (uint32_t i = tr * kPer; i < idx; ++i) {
                    const double x = xs[i], y = ys[i];
                    pre[0] += 1.0; pre[1] += x; pre[2] += x * x; pre[3] += y; pre[4] += x * y;
                }
                for (int c = 0; c < 5; ++c) suf[c][u] = tp[c][256] - pre[c];
            }
            __syncthreads();
            for (int q = threadIdx.x; q < NT + NF; q += blockDim.x) {
                if (q < NT) {
                    int ua = 0, rem = q;
                    while (rem >= NF - ua) { rem -= NF - ua; ++ua; }
                    const int ub = ua + rem;  // ua <= ub
                    double acc;
                    if (ua == kSeg) {
                        acc = suf[0][0];
                    } else if (ua == 0) {
                        const double b = static_cast<double>(ub) / kSeg;
                        acc = ub == 0 ? suf[2][0] : ub == kSeg ? suf[1][0] : suf[2][ub] - b * suf[1][ub];
                    } else {
                        const double a = static_cast<double>(ua) / kSeg, b = static_cast<double>(ub) / kSeg;
                        acc = ub == kSeg ? suf[1][ua] - a * suf[0][ua]
                                         : suf[2][ub] - (a + b) * suf[1][ub] + a * b * suf[0][ub];
                    }
                    G[ua * NF + ub] = acc;
                    G[ub * NF + ua] = acc;
                } else {
                    const int ua = q - NT;
                    const double b = static_cast<double>(ua) / kSeg;
                    rr[ua] = ua == 0 ? suf[4][0] : ua == kSeg ? suf[3][0] : suf[4][ua] - b * suf[3][ua];
                }
            }
        } else {
            // normal equations by direct sums, upper triangle and right-hand side
            for (int q = threadIdx.x; q < NT + NF; q += blockDim.x) {
                double acc = 0.0;
                if (q < NT) {
                    int ua = 0, rem = q;
                    while (rem >= NF - ua) { rem -= NF - ua; ++ua; }
                    const int ub = ua + rem;
                    for (uint32_t i = 0; i < nq; ++i) acc += feature(ua, xs[i]) * feature(ub, xs[i]);
                    G[ua * NF + ub] = acc;
                    G[ub * NF + ua] = acc;
                } else {
                    const int ua = q - NT;
                    for (uint32_t i = 0; i < nq; ++i) acc += feature(ua, xs[i]) * static_cast<double>(ys[i]);
                    rr[ua] = acc;
                }
            }
        }
        __syncthreads();
        if (threadIdx.x < 64) {
            const bool ok = cholesky_solve_wave(G, rr, NF);
            if (threadIdx.x == 0) solved = ok ? 1 : 0;
        }
        __syncthreads();
    }
    // pieces of the network: slope_m = sum_{u<=m} w_u,
    // intercept_m = w_b - sum_{1<=u<=m} w_u u/32
    if (threadIdx.x < static_cast<unsigned>(kSeg)) {
        const int m = threadIdx.x;
        double A = 0.0, C = solved ? rr[kSeg] : 0.0;
        if (solved)
            for (int u = 0; u <= m; ++u) {
                A += rr[u];
                if (u > 0) C -= rr[u] * static_cast<double>(u) / kSeg;
            }
        mf->A[m] = static_cast<float>(A);
        mf->C[m] = static_cast<float>(C);
    }
    if (threadIdx.x == 0) {
        mf->lin_s = static_cast<float>(slope);
        mf->lin_t = static_cast<float>(icpt);
        mf->base = p0;
        mf->mlp_ok = solved;
        mf->kind = kKindLinear;
        mf->n_keys = 0;
    }
}

__global__ void k_bounds_init(int32_t* bnd, uint32_t* cnt, uint32_t cells) {
    for (uint64_t j = gid(); j < cells; j += gsz()) {
        bnd[4 * j + 0] = INT32_MAX; bnd[4 * j + 1] = INT32_MIN;
        bnd[4 * j + 2] = INT32_MAX; bnd[4 * j + 3] = INT32_MIN;
        cnt[j] = 0;
    }
}

// Every key of the tree, one lane per key slot, through both kinds of its
// model.  Neighbouring slots almost always share a piece: a wave whose 64
// slots all do reduces them in registers and keeps the piece's bounds until
// its run of windows reaches another piece, then issues one set of atomics.
template <class K>
__global__ __launch_bounds__(kLiBlock) void k_bounds(TreeView<K> t, LiView<K> li, uint32_t nleaves) {
    const LiArgs a = args_of(li.hdr);
    const uint64_t total = static_cast<uint64_t>(nleaves) * kSlots;
    const int lane = lane_id();
    // each wave takes a contiguous run of 64-slot windows and carries the
    // bounds of its current piece across windows (consecutive windows mostly
    // share a piece), so a piece's atomics go out once per run, not once per
    // window
    const uint64_t nwin = (total + 63) / 64, nwave = gsz() / 64;
    const uint64_t per = (nwin + nwave - 1) / nwave;
    const uint64_t wb = (gid() / 64) * per, we = wb + per < nwin ? wb + per : nwin;
    uint32_t cur = UINT32_MAX, ccnt = 0;
    int32_t clmin = INT32_MAX, clmax = INT32_MIN, cmmin = INT32_MAX, cmmax = INT32_MIN;
    auto flush = [&]() {
        if (cur != UINT32_MAX && lane == 0) {
            atomicMin(&li.bnd[4 * cur + 0], clmin);
            atomicMax(&li.bnd[4 * cur + 1], clmax);
            if (cmmin <= cmmax) {
                atomicMin(&li.bnd[4 * cur + 2], cmmin);
                atomicMax(&li.bnd[4 * cur + 3], cmmax);
            }
            atomicAdd(&li.cnt[cur], ccnt);
        }
    };
    for (uint64_t wi = wb; wi < we; ++wi) {
        const uint64_t x = wi * 64 + static_cast<uint64_t>(lane);
        bool valid = false;
        uint32_t cell = 0;
        int32_t rl = 0, rm = 0;
        bool mok = false;
        if (x < total) {
            const uint32_t leaf = static_cast<uint32_t>(x / kSlots), slot = static_cast<uint32_t>(x % kSlots);
            if (slot < t.lmeta[leaf].x) {
                valid = true;
                const uint64_t key = static_cast<uint64_t>(t.lkeys[x]);
                const int32_t pos = static_cast<int32_t>(li.pos_of_leaf[leaf]);
                const Route r = route(a, key);
                const ModelFit* f = li.fit + r.j;
                cell = r.j * kSeg + r.m;
                rl = pos - piece_pos(f->lin_s, f->lin_t, f->base, r.x, a.L);
                mok = f->mlp_ok != 0;
                if (mok) rm = pos - piece_pos(f->A[r.m], f->C[r.m], f->base, r.x, a.L);
            }
        }
        // the window's pieces in lane order (almost always one, at a piece
        // boundary two): each is reduced over its lanes, then merged into the
        // running piece or, when it differs, flushes the running one first
        uint64_t rem = __ballot(valid);
        while (rem) {
            const int ld = __builtin_ctzll(rem);
            const uint32_t cc = static_cast<uint32_t>(__shfl(static_cast<int>(cell), ld, 64));
            const bool mine = valid && cell == cc;
            const uint64_t mm = __ballot(mine);
            int32_t lmin = mine ? rl : INT32_MAX, lmax = mine ? rl : INT32_MIN;
            int32_t mmin = mine && mok ? rm : INT32_MAX, mmax = mine && mok ? rm : INT32_MIN;
            for (int d = 32; d > 0; d >>= 1) {
                lmin = min(lmin, __shfl_xor(lmin, d, 64));
                lmax = max(lmax, __shfl_xor(lmax, d, 64));
                mmin = min(mmin, __shfl_xor(mmin, d, 64));
                mmax = max(mmax, __shfl_xor(mmax, d, 64));
            }
            if (cc != cur) {
                flush();
                cur = cc;
                ccnt = 0;
                clmin = INT32_MAX; clmax = INT32_MIN; cmmin = INT32_MAX; cmmax = INT32_MIN;
            }
            clmin = min(clmin, lmin);
            clmax = max(clmax, lmax);
            cmmin = min(cmmin, mmin);
            cmmax = max(cmmax, mmax);
            ccnt += static_cast<uint32_t>(__popcll(mm));
            rem &= ~mm;
        }
    }
    flush();
}

// One wave per model, lane m < 32 per piece: pick the kind with the smaller
// key-weighted window (a key sent down the tree counts 2 * max_window) and
// write the pieces the lookup reads.
template <class K>
__global__ __launch_bounds__(256) void k_choose(LiView<K> li, uint32_t M, uint32_t kind_pref, uint32_t max_window) {
    const uint32_t j = static_cast<uint32_t>(gid() / 64);
    const int lane = lane_id();
    if (j >= M) return;
    const ModelFit* f = li.fit + j;
    const bool mok = f->mlp_ok != 0;
    const uint64_t cell = static_cast<uint64_t>(j) * kSeg + lane;
    uint32_t c = 0;
    int32_t ll = 0, lh = 0, ml = 0, mh = 0;
    if (lane < kSeg) {
        c = li.cnt[cell];
        ll = li.bnd[4 * cell + 0]; lh = li.bnd[4 * cell + 1];
        ml = li.bnd[4 * cell + 2]; mh = li.bnd[4 * cell + 3];
    }
    auto fits = [&](int32_t lo, int32_t hi) {
        return lo <= hi && static_cast<int64_t>(hi) - lo + 1 <= static_cast<int64_t>(max_window) && lo >= -32768 &&
               hi <= 32767;
    };
    const double pen = 2.0 * max_window;
    double cl = 0.0, cm = 0.0;
    if (c) {
        cl = c * (fits(ll, lh) ? static_cast<double>(lh - ll + 1) : pen);
        cm = c * (mok && fits(ml, mh) ? static_cast<double>(mh - ml + 1) : pen);
    }
    uint32_t total = c;
    for (int d = 32; d > 0; d >>= 1) {
        cl += __shfl_xor(cl, d, 64);
        cm += __shfl_xor(cm, d, 64);
        total += __shfl_xor(total, d, 64);
    }
    bool use_mlp;
    if (kind_pref == 1) use_mlp = false;
    else if (kind_pref == 2) use_mlp = mok;
    else use_mlp = mok && cm < cl;
    const int32_t lo0 = use_mlp ? ml : ll, hi0 = use_mlp ? mh : lh;
    const bool keyed_out = c > 0 && !fits(lo0, hi0);
    const bool all_out = __ballot(c > 0 && !keyed_out) == 0 && total > 0;
    if (lane < kSeg) {
        Piece p;
        p.slope = use_mlp ? f->A[lane] : f->lin_s;
        p.icpt = use_mlp ? f->C[lane] : f->lin_t;
        p.base = f->base;
        int32_t lo = lo0, hi = hi0;
        if (c == 0) lo = hi = 0;          // no key here: the prediction alone
        else if (keyed_out) { lo = 1; hi = 0; }
        p.lo = static_cast<int16_t>(lo);
        p.hi = static_cast<int16_t>(hi);
        li.piece[cell] = p;
    }
    if (lane == 0) {
        li.fit[j].kind = all_out ? kKindTree : (use_mlp ? kKindMlp : kKindLinear);
        li.fit[j].n_keys = total;
    }
}

// Model quality over the trained keys (one workgroup): keys whose piece
// sends them down the tree, and the key-weighted window of the others.
constexpr int kQualityBlock = 1024;

template <class K>
__global__ __launch_bounds__(kQualityBlock) void k_quality(LiView<K> li, uint32_t cells) {
    __shared__ unsigned long long sh[3][kQualityBlock / 64];
    unsigned long long tree = 0, wsum = 0, wmax = 0;
    for (uint32_t c = threadIdx.x; c < cells; c += kQualityBlock) {
        const uint32_t n = li.cnt[c];
        const Piece p = li.piece[c];
        if (n == 0) continue;
        if (p.lo > p.hi) {
            tree += n;
        } else {
            const unsigned long long w = static_cast<unsigned long long>(p.hi - p.lo + 1);
            wsum += static_cast<unsigned long long>(n) * w;
            wmax = w > wmax ? w : wmax;
        }
    }
    for (int d = 32; d > 0; d >>= 1) {
        tree += __shfl_xor(tree, d, 64);
        wsum += __shfl_xor(wsum, d, 64);
        const unsigned long long o = __shfl_xor(wmax, d, 64);
        wmax = o > wmax ? o : wmax;
    }
    const int w = threadIdx.x / 64;
    if ((threadIdx.x & 63) == 0) {
        sh[0][w] = tree;
        sh[1][w] = wsum;
        sh[2][w] = wmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long a = 0, b = 0, m = 0;
        for (int i = 0; i < kQualityBlock / 64; ++i) {
            a += sh[0][i];
            b += sh[1][i];
            m = sh[2][i] > m ? sh[2][i] : m;
        }
        li.hdr->keys_tree = a;
        li.hdr->window_sum = b;
        li.hdr->max_win = static_cast<uint32_t>(m);
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

__global__ void k_set_bounds(Piece* piece, uint64_t cells, int32_t lo, int32_t hi) {
    for (uint64_t j = gid(); j < cells; j += gsz()) {
        if (piece[j].lo <= piece[j].hi) {
            piece[j].lo = static_cast<int16_t>(lo);
            piece[j].hi = static_cast<int16_t>(hi);
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

// A leaf's answer for one key: its value when the leaf holds it.
template <class K>
struct Hit {
    bool hit = false;
    K val = kmax<K>();
};

template <class K>
__device__ __forceinline__ void match_leaf(const typename Trav<K, kLiG>::KV& kv, const typename Trav<K, kLiG>::KV& vv,
                                           K key, int gbase, Hit<K>& v) {
    using T = Trav<K, kLiG>;
    const uint32_t slot = T::match_slot(kv, key, gbase);
    const K x = T::pick_value(vv, slot < kSlots ? slot : 0u, gbase);
    if (slot < kSlots) {
        v.hit = true;
        v.val = x;
    }
}

// A miss after the tree changed (or after li_set_bounds) resumes along the
// leaf chain from a candidate leaf: the last window leaf whose first key is
// <= key.  Chain order is key order, so the key lies in the candidate or in a
// leaf chained after it (a split moves the upper part of a leaf to new leaves
// chained right after it).  The walk goes on while the current leaf ends
// below the key; a walk longer than kWalkMax leaves, or no candidate, hands
// over to the root-to-leaf descent.  Trained leaf ids stay valid leaves
// because the tree never frees a leaf (it has no delete).  Returns false when
// the walk cannot decide.
template <class K>
__device__ __forceinline__ bool chain_walk(const TreeView<K>& t, K key, uint32_t cand, K cand_last, int gl,
                                           int gbase, Hit<K>& v) {
    using T = Trav<K, kLiG>;
    uint32_t cur = cand;
    K last = cand_last;
    for (int step = 0; step < kWalkMax; ++step) {
        if (last >= key) return true;           // the key's leaf was checked: absent
        const uint32_t nx = t.lmeta[cur].y;
        if (nx == kNone) return true;           // past the last leaf: absent
        const typename T::KV kv = T::load_keys(t.lkeys + static_cast<uint64_t>(nx) * kSlots, gl);
        const typename T::KV vv = T::load_keys(t.lvals + static_cast<uint64_t>(nx) * kSlots, gl);
        const K first = static_cast<K>(__shfl(kv.v[0], gbase, 64));
        if (first > key) return true;           // between two leaves: absent
        match_leaf<K>(kv, vv, key, gbase, v);
        if (v.hit) return true;
        last = static_cast<K>(__shfl(kv.v[T::KPL - 1], gbase + kLiG - 1, 64));
        cur = nx;
    }
    return last >= key;
}

// Learned lookup.  DIRECT: the trained directory is the identity (position
// = leaf id), so the window's leaves are read directly.  STALE: the tree may
// have changed since training or the bounds were overwritten; a miss then
// resumes along the leaf chain (chain_walk) before it falls back to the
// tree.  The host launches STALE = false while no insert was issued since
// training, so the common kernel carries none of that code.
template <class K, bool DIRECT, int BLK, bool STALE>
__global__ __launch_bounds__(BLK) void k_li_lookup(TreeView<K> t, LiView<K> li, LiArgs a, const K* __restrict__ q,
                                                   uint64_t B, K* __restrict__ vout, uint8_t* __restrict__ fout) {
    using T = Trav<K, kLiG>;
    // issued first, so the kernel's end does not wait for it
    if (gid() == 0) atomicAdd(&li.hdr->lookups, static_cast<unsigned long long>(B));
    const int lane = lane_id();
    const int gl = lane % kLiG, gbase = lane - gl;
    const uint64_t group = gid() / kLiG, ngroups = gsz() / kLiG;
    const int32_t last_pos = static_cast<int32_t>(a.L) - 1;
    // unchanged tree and trained bounds: the window holds every present key.
    // Read only when a miss needs it (-1: not read yet).
    int fresh = a.exact ? -1 : 0;
    for (uint64_t i = group; i < B; i += ngroups) {
        const K key = q[i];
        const Route r = route(a, static_cast<uint64_t>(key));
        const Piece e = load_piece(li.piece, r.j, r.m);
        Hit<K> v;
        bool fb = e.lo > e.hi;
        // where a stale miss resumes (STALE only)
        uint32_t cand = kNone;
        K cand_last = K(0);
        if (!fb) {
            const int32_t p = piece_pos(e.slope, e.icpt, e.base, r.x, a.L);
            const int32_t wl = max(p + e.lo, 0), wh = min(p + e.hi, last_pos);
            if constexpr (DIRECT) {
                // positions are leaf ids: read kDirect of the window's leaves at
                // once; each lane checks its own slots (no cross-lane work
                // until one lane holds the key)
                for (int32_t b0 = wl; b0 <= wh && !v.hit; b0 += kDirect) {
                    typename T::KV kv[kDirect], vv[kDirect];
#pragma unroll
                    for (int u = 0; u < kDirect; ++u) {
                        if (b0 + u <= wh) {
                            kv[u] = T::load_keys(t.lkeys + static_cast<uint64_t>(b0 + u) * kSlots, gl);
                            vv[u] = T::load_keys(t.lvals + static_cast<uint64_t>(b0 + u) * kSlots, gl);
                        }
                    }
                    // this lane's first slot holding the key (padding slots repeat
                    // a leaf's last key, so the first one is the real slot)
                    bool mine = false;
                    K mval = K(0);
#pragma unroll
                    for (int u = 0; u < kDirect; ++u) {
                        const bool in = b0 + u <= wh;
#pragma unroll
                        for (int x = 0; x < T::KPL; ++x) {
                            const bool m = in && !mine && kv[u].v[x] == key;
                            mval = m ? vv[u].v[x] : mval;
                            mine = mine || m;
                        }
                    }
                    const uint64_t hm = group_bits<kLiG>(__ballot(mine), gbase);
                    if (hm) {
                        v.hit = true;
                        v.val = static_cast<K>(__shfl(mval, gbase + __builtin_ctzll(hm), 64));
                    }
                }
                if constexpr (STALE) {
                    if (!v.hit) {
                        // the candidate from the window leaves' first and last
                        // keys, kLiG leaves at a time
                        for (int32_t b0 = wl; b0 <= wh; b0 += kLiG) {
                            const int32_t pp = b0 + gl;
                            const bool in = pp <= wh;
                            K first = K(0), last = K(0);
                            if (in) {
                                first = t.lkeys[static_cast<uint64_t>(pp) * kSlots];
                                last = t.lkeys[static_cast<uint64_t>(pp) * kSlots + kSlots - 1];
                            }
                            const uint64_t m = group_bits<kLiG>(__ballot(in && first <= key), gbase);
                            if (m) {
                                const int idx = 63 - __builtin_clzll(m);
                                cand = static_cast<uint32_t>(b0 + idx);
                                cand_last = static_cast<K>(__shfl(last, gbase + idx, 64));
                            }
                        }
                    }
                }
            } else {
                // the last fence <= key in the window picks the leaf; none: the
                // key lies before the window (absent while the tree is unchanged)
                uint32_t leaf = kNone;
                const int64_t c = window_search<K>(li.dir, wl, wh, key, gl, gbase, &leaf);
                if (c >= 0) {
                    const typename T::KV kv = T::load_keys(t.lkeys + static_cast<uint64_t>(leaf) * kSlots, gl);
                    const typename T::KV vv = T::load_keys(t.lvals + static_cast<uint64_t>(leaf) * kSlots, gl);
                    match_leaf<K>(kv, vv, key, gbase, v);
                    if constexpr (STALE) {
                        cand = leaf;
                        cand_last = static_cast<K>(__shfl(kv.v[T::KPL - 1], gbase + kLiG - 1, 64));
                    }
                }
            }
            // no hit: proof of absence on an unchanged tree, else the leaf
            // chain or the tree decides
            if (!v.hit) {
                if (fresh < 0) fresh = t.hdr->epoch == a.epoch ? 1 : 0;
                fb = fresh == 0;
            }
        }
        if constexpr (STALE) {
            if (fb && cand != kNone && chain_walk<K>(t, key, cand, cand_last, gl, gbase, v)) fb = false;
        }
        if (fb) {
            // the tree decides: plain root-to-leaf walk
            K kk[1] = {key};
            uint32_t lf[1];
            descend<K, kLiG, 1, false>(t, t.mirror, kMirrorMaxNodes, 0, kk, lf, gl, gbase);
            const typename T::KV kv = T::load_keys(t.lkeys + static_cast<uint64_t>(lf[0]) * kSlots, gl);
            const typename T::KV vv = T::load_keys(t.lvals + static_cast<uint64_t>(lf[0]) * kSlots, gl);
            v = Hit<K>();
            match_leaf<K>(kv, vv, key, gbase, v);
            // counted where it happens (rare): no reduction on the common path
            if (gl == 0) atomicAdd(&li.hdr->fallbacks, 1ull);
        }
        if (gl == 0) {
            vout[i] = v.hit ? v.val : kmax<K>();
            fout[i] = v.hit ? 1 : 0;
        }
    }
}

// Inference as the lookup runs it: piece id (model * 32 + piece), predicted
// position, the piece's bounds and the kind in use (2: down the tree).
template <class K>
__global__ __launch_bounds__(kLiBlock) void k_li_predict(LiView<K> li, LiArgs a, const K* __restrict__ q,
                                                         uint64_t B, uint32_t* mo, int32_t* po, int32_t* lo,
                                                         int32_t* hi, uint8_t* ko) {
    for (uint64_t i = gid(); i < B; i += gsz()) {
        const Route r = route(a, static_cast<uint64_t>(q[i]));
        const Piece e = load_piece(li.piece, r.j, r.m);
        const bool tree = e.lo > e.hi;
        mo[i] = r.j * kSeg + r.m;
        po[i] = tree ? 0 : piece_pos(e.slope, e.icpt, e.base, r.x, a.L);
        lo[i] = tree ? 0 : e.lo;
        hi[i] = tree ? 0 : e.hi;
        ko[i] = tree ? static_cast<uint8_t>(kKindTree)
                     : static_cast<uint8_t>(li.fit[r.j].kind == kKindMlp ? kKindMlp : kKindLinear);
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
    uint64_t off_fit, off_piece, off_dir, off_nxt0, off_nxt1, off_rank0, off_rank1, off_pos, off_start, off_bnd,
        off_cnt, off_partial, off_ident, off_lvl, off_scan;
    LiArgs args;
    bool declined = false;    // the quality gate sends lookups to the tree kernel
    uint32_t max_win = 0;     // widest window at training (leaves)
    uint64_t inserts_at_train = 0;  // the tree's insert count when trained
    uint64_t deletes_at_train = 0;  // and its delete count
    uint64_t generation = 0;  // bumped whenever the lookup's arguments or tables change
};

// The lookup launches a different kernel once the tree has changed since
// training (or the bounds were overwritten): that state is part of the
// generation, so a captured graph of the other state is captured again.
static bool li_stale(const gt_learned* li) {
    return !li->args.exact || li->t->inserts != li->inserts_at_train;
}

// After a delete batch the directory may name leaves the delete cleared or
// refilled, so lookups go down the tree until the next training.
static bool li_deleted(const gt_learned* li) { return li->t->deletes != li->deletes_at_train; }

uint64_t gt_li_generation(const gt_learned* li) {
    return 4 * li->generation + (li_deleted(li) ? 2 : 0) + (li_stale(li) ? 1 : 0);
}

namespace {

uint64_t al256(uint64_t x) { return (x + 255) / 256 * 256; }

uint32_t models_of(const gt_li_params* p) { return p && p->models ? p->models : 1024u; }

bool params_bad(const gt_li_params* p) {
    return p && (p->models > 4096 || p->kind > 2 || p->search > 2 || p->gate > 1 || p->reserved[0] ||
                 p->reserved[1]);
}

uint64_t layout_li(gt_learned* li, uint64_t leaf_cap, uint32_t M, int kb) {
    const uint64_t cells = static_cast<uint64_t>(M) * kSeg;
    uint64_t off = al256(sizeof(LiHeader));
    const uint64_t de = kb == 8 ? sizeof(DirEntry<uint64_t>) : sizeof(DirEntry<uint32_t>);
    uint64_t o_fit = off; off += al256(static_cast<uint64_t>(M) * sizeof(ModelFit));
    uint64_t o_piece = off; off += al256(cells * sizeof(Piece));
    uint64_t o_dir = off; off += al256((leaf_cap + 1) * de);
    uint64_t o_n0 = off; off += al256(leaf_cap * 4);
    uint64_t o_n1 = off; off += al256(leaf_cap * 4);
    uint64_t o_r0 = off; off += al256(leaf_cap * 4);
    uint64_t o_r1 = off; off += al256(leaf_cap * 4);
    uint64_t o_pos = off; off += al256(leaf_cap * 4);
    uint64_t o_start = off; off += al256((M + 1ull) * 4);
    uint64_t o_bnd = off; off += al256(4ull * cells * 4);
    uint64_t o_cnt = off; off += al256(cells * 4);
    uint64_t o_part = off; off += al256(kMaxPartials * 5ull * 8);
    uint64_t o_ident = off; off += 256;
    uint64_t o_lvl = off; off += al256(kMaxLevels * 4);
    uint64_t o_scan = off; off += al256(scan_tmp_bytes(leaf_cap + 1));
    if (li) {
        li->off_fit = o_fit; li->off_piece = o_piece; li->off_dir = o_dir; li->off_nxt0 = o_n0;
        li->off_nxt1 = o_n1; li->off_rank0 = o_r0; li->off_rank1 = o_r1; li->off_pos = o_pos;
        li->off_start = o_start; li->off_bnd = o_bnd; li->off_cnt = o_cnt; li->off_partial = o_part;
        li->off_ident = o_ident;
        li->off_lvl = o_lvl;
        li->off_scan = o_scan;
    }
    return off;
}

template <class K>
LiView<K> li_view(const gt_learned* li) {
    LiView<K> v;
    uint8_t* a = li->arena;
    v.hdr = reinterpret_cast<LiHeader*>(a);
    v.fit = reinterpret_cast<ModelFit*>(a + li->off_fit);
    v.piece = reinterpret_cast<Piece*>(a + li->off_piece);
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
    v.identity = reinterpret_cast<uint32_t*>(a + li->off_ident);
    v.lvl = reinterpret_cast<uint32_t*>(a + li->off_lvl);
    v.scan_tmp = a + li->off_scan;
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
        li->declined = false;
        li->inserts_at_train = t->inserts;
        li->deletes_at_train = t->deletes;
        li->generation++;
        return GT_OK;
    }
    const uint32_t ids = dh.leaf_used;  // leaf ids in use (a delete's merge can leave some unreached)
    if (ids > li->leaf_cap) return GT_ERR_CAPACITY;
    uint32_t n = 1;  // leaves in the tree: positions 0..n-1
    // leaf positions: expand the levels from the root (lists in nxt0/nxt1,
    // per-node child counts and their offsets in rank0/rank1)
    {
        const uint32_t h = dh.height;
        uint32_t* la = v.nxt0; uint32_t* lb = v.nxt1;
        uint32_t* lvl = v.lvl;  // lvl[l] = nodes of level l
        hipLaunchKernelGGL(k_pos_clear, dim3(grid_of(ids, 256)), dim3(256), 0, s, v.pos_of_leaf, ids);
        hipLaunchKernelGGL(k_bfs_init, dim3(1), dim3(64), 0, s, la, lvl, dh.root, v.pos_of_leaf, h <= 1 ? 1u : 0u);
        uint64_t bound = 1;  // nodes a level can have
        for (uint32_t l = 0; l + 1 < h; ++l) {
            const uint64_t g = grid_of(bound * kSlots, 256, 8192);
            hipLaunchKernelGGL(k_bfs_count, dim3(g), dim3(256), 0, s, t->ichild, la, lvl + l, v.rank0);
            scan_exclusive<uint32_t>(v.rank0, v.rank1, lvl + l + 1, lvl + l, bound, v.scan_tmp, s);
            hipLaunchKernelGGL(k_bfs_scatter, dim3(g), dim3(256), 0, s, t->ichild, la, lvl + l, v.rank0, v.rank1, lb,
                               v.pos_of_leaf, l + 2 == h ? 1u : 0u);
            uint32_t* x = la; la = lb; lb = x;
            bound = bound * kSlots < ids ? bound * kSlots : ids;
        }
        if (h > 1) {
            LI_HIP(hipMemcpyAsync(&n, lvl + (h - 1), 4, hipMemcpyDeviceToHost, s));
            LI_HIP(hipStreamSynchronize(s));
        }
    }
    if (n == 0 || n > ids) return GT_ERR_DEVICE;
    hipLaunchKernelGGL(k_directory<K>, dim3(grid_of(ids, 256)), dim3(256), 0, s, tv, v, ids, n);
    // root normalisation: smallest first key .. largest key of the tree
    DirEntry<K> d0, dl;
    LI_HIP(hipMemcpyAsync(&d0, v.dir, sizeof d0, hipMemcpyDeviceToHost, s));
    LI_HIP(hipMemcpyAsync(&dl, v.dir + (n - 1), sizeof dl, hipMemcpyDeviceToHost, s));
    LI_HIP(hipStreamSynchronize(s));
    K kmaxkey;
    LI_HIP(hipMemcpyAsync(&kmaxkey, tv.lkeys + static_cast<uint64_t>(dl.leaf) * kSlots + kSlots - 1, sizeof(K),
                          hipMemcpyDeviceToHost, s));
    LI_HIP(hipStreamSynchronize(s));
    const uint64_t kmin = static_cast<uint64_t>(d0.fence), kmx = static_cast<uint64_t>(kmaxkey);
    const double scale = kmx > kmin ? 1.0 / static_cast<double>(kmx - kmin) : 1.0;
    const uint32_t nb = n < static_cast<uint32_t>(kMaxPartials) ? n : kMaxPartials;
    const uint64_t cells = static_cast<uint64_t>(M) * kSeg;
    hipLaunchKernelGGL(k_root_partial<K>, dim3(nb), dim3(256), 0, s, v, n, M, kmin, scale);
    hipLaunchKernelGGL(k_root_final<K>, dim3(1), dim3(256), 0, s, v, nb, kmin, scale, n, M, dh.epoch);
    hipLaunchKernelGGL(k_ranges<K>, dim3(grid_of(n, 256)), dim3(256), 0, s, v, n, M);
    hipLaunchKernelGGL(k_fit<K>, dim3(M), dim3(256), 0, s, v, n, M);
    hipLaunchKernelGGL(k_bounds_init, dim3(grid_of(cells, 256)), dim3(256), 0, s, v.bnd, v.cnt,
                       static_cast<uint32_t>(cells));
    // over leaf ids: a leaf no longer in the tree holds no keys
    hipLaunchKernelGGL(k_bounds<K>, dim3(grid_of(static_cast<uint64_t>(ids) * kSlots, kLiBlock, 8192)),
                       dim3(kLiBlock), 0, s, tv, v, ids);
    uint32_t mw = li->p.max_window ? li->p.max_window : 64u;
    if (mw > 4096u) mw = 4096u;
    hipLaunchKernelGGL(k_choose<K>, dim3(grid_of(static_cast<uint64_t>(M) * 64, 256)), dim3(256), 0, s, v, M,
                       li->p.kind, mw);
    hipLaunchKernelGGL(k_li_finish<K>, dim3(1), dim3(64), 0, s, v, dh.n_keys);
    hipLaunchKernelGGL(k_quality<K>, dim3(1), dim3(kQualityBlock), 0, s, v, static_cast<uint32_t>(cells));
    const uint32_t one = 1;
    LI_HIP(hipMemcpyAsync(v.identity, &one, 4, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_identity, dim3(grid_of(ids, 256)), dim3(256), 0, s, v.pos_of_leaf, ids, v.identity);
    if (hipGetLastError() != hipSuccess) return GT_ERR_HIP;
    LiHeader h;
    uint32_t ident = 0;
    LI_HIP(hipMemcpyAsync(&h, v.hdr, sizeof h, hipMemcpyDeviceToHost, s));
    LI_HIP(hipMemcpyAsync(&ident, v.identity, 4, hipMemcpyDeviceToHost, s));
    LI_HIP(hipStreamSynchronize(s));
    li->args.kmin = h.kmin_root;
    li->args.a = h.root_a;
    li->args.c = h.root_c;
    li->args.L = h.L;
    li->args.M = h.M;
    li->args.epoch = h.epoch;
    li->args.identity = ident;
    li->args.exact = 1;
    li->args.pad = 0;
    li->trained = true;
    // quality gate: when many keys would go down the tree after the model
    // step, or the windows are wide, the model path costs more than the
    // tree's own descent; lookups then take the tree (same results)
    const double keys = static_cast<double>(h.n_keys);
    const double in_win = keys - static_cast<double>(h.keys_tree);
    const double mean_win = in_win > 0 ? static_cast<double>(h.window_sum) / in_win : 0.0;
    li->declined = li->p.gate == 0 &&
                   (static_cast<double>(h.keys_tree) > kGateTreeShare * keys || mean_win > kGateMeanWindow);
    li->max_win = h.max_win;
    li->inserts_at_train = t->inserts;
    li->deletes_at_train = t->deletes;
    li->generation++;
    return GT_OK;
}

template <class K, bool DIRECT, int BLK>
void launch_li_lookup_t(gt_learned* li, bool stale, const K* q, uint64_t B, K* vo, uint8_t* fo, hipStream_t stream) {
    const uint32_t grid = grid_of(B * kLiG, BLK, 8192);
    if (stale)
        hipLaunchKernelGGL((k_li_lookup<K, DIRECT, BLK, true>), dim3(grid), dim3(BLK), 0, stream, view<K>(li->t),
                           li_view<K>(li), li->args, q, B, vo, fo);
    else
        hipLaunchKernelGGL((k_li_lookup<K, DIRECT, BLK, false>), dim3(grid), dim3(BLK), 0, stream, view<K>(li->t),
                           li_view<K>(li), li->args, q, B, vo, fo);
}

// Small batches are latency-bound: 64-thread workgroups spread them over
// more CUs (fewer outstanding misses per CU).  Windows are read directly on
// a bulk-loaded tree (identity directory) for small batches when every
// window is narrow; otherwise the fence directory is searched.
template <class K>
void launch_li_lookup(gt_learned* li, const void* keys, uint64_t B, void* values_out, uint8_t* found_out,
                      hipStream_t stream) {
    const uint32_t mode = li->p.search;
    const bool direct = li->args.identity &&
                        (mode == 2 || (mode == 0 && B <= kDirectMaxBatch && li->max_win <= kDirectMaxWin));
    const bool small = B <= kSmallLookup;
    const bool stale = li_stale(li);
    const K* q = reinterpret_cast<const K*>(keys);
    K* vo = reinterpret_cast<K*>(values_out);
    if (direct) {
        if (small) launch_li_lookup_t<K, true, 64>(li, stale, q, B, vo, found_out, stream);
        else launch_li_lookup_t<K, true, kLiBlock>(li, stale, q, B, vo, found_out, stream);
    } else {
        if (small) launch_li_lookup_t<K, false, 64>(li, stale, q, B, vo, found_out, stream);
        else launch_li_lookup_t<K, false, kLiBlock>(li, stale, q, B, vo, found_out, stream);
    }
}

}  // namespace

extern "C" {

uint64_t li_arena_bytes(const gt_tree* t, const gt_li_params* p) {
    if (!t || t->wide || params_bad(p)) return 0;
    return layout_li(nullptr, t->leaf_cap, models_of(p), t->kb);
}

gt_status li_create(gt_tree* t, const gt_li_params* p, void* arena, uint64_t arena_bytes, gt_learned** out) {
    if (!t || t->wide || !arena || !out || params_bad(p)) return GT_ERR_INVALID;
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
    if (!li->trained || li->declined || li_deleted(li))
        return tree_lookup_batch(li->t, keys, B, values_out, found_out, stream);
    if (li->t->kb == 8) launch_li_lookup<uint64_t>(li, keys, B, values_out, found_out, stream);
    else launch_li_lookup<uint32_t>(li, keys, B, values_out, found_out, stream);
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status li_predict(gt_learned* li, const void* keys, uint64_t B, uint32_t* model_out, int32_t* pred_out,
                     int32_t* lo_out, int32_t* hi_out, uint8_t* kind_out, hipStream_t stream) {
    if (!li || (B && (!keys || !model_out || !pred_out || !lo_out || !hi_out || !kind_out))) return GT_ERR_INVALID;
    if (!li->trained) return GT_ERR_INVALID;
    if (B == 0) return GT_OK;
    const uint32_t grid = grid_of(B, kLiBlock, 4096);
    if (li->t->kb == 8)
        hipLaunchKernelGGL(k_li_predict<uint64_t>, dim3(grid), dim3(kLiBlock), 0, stream, li_view<uint64_t>(li),
                           li->args, reinterpret_cast<const uint64_t*>(keys), B, model_out, pred_out, lo_out, hi_out,
                           kind_out);
    else
        hipLaunchKernelGGL(k_li_predict<uint32_t>, dim3(grid), dim3(kLiBlock), 0, stream, li_view<uint32_t>(li),
                           li->args, reinterpret_cast<const uint32_t*>(keys), B, model_out, pred_out, lo_out, hi_out,
                           kind_out);
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status li_set_bounds(gt_learned* li, int32_t lo, int32_t hi, hipStream_t stream) {
    if (!li || lo > hi) return GT_ERR_INVALID;
    if (lo < -30000 || hi > 30000) return GT_ERR_INVALID;
    const uint64_t cells = static_cast<uint64_t>(li->M) * kSeg;
    li->args.exact = 0;  // windows no longer cover every key: misses need proof
    li->generation++;
    hipLaunchKernelGGL(k_set_bounds, dim3(grid_of(cells, 256)), dim3(256), 0, stream,
                       reinterpret_cast<Piece*>(li->arena + li->off_piece), cells, lo, hi);
    return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP;
}

gt_status li_stats(gt_learned* li, gt_li_stats* out, hipStream_t stream) {
    if (!li || !out) return GT_ERR_INVALID;
    const uint64_t cells = static_cast<uint64_t>(li->M) * kSeg;
    LiHeader h;
    std::vector<ModelFit> fs(li->M);
    std::vector<Piece> ps(cells);
    std::vector<uint32_t> cs(cells);
    LI_HIP(hipMemcpyAsync(&h, li->arena, sizeof h, hipMemcpyDeviceToHost, stream));
    LI_HIP(hipMemcpyAsync(fs.data(), li->arena + li->off_fit, fs.size() * sizeof(ModelFit), hipMemcpyDeviceToHost,
                          stream));
    LI_HIP(hipMemcpyAsync(ps.data(), li->arena + li->off_piece, ps.size() * sizeof(Piece), hipMemcpyDeviceToHost,
                          stream));
    LI_HIP(hipMemcpyAsync(cs.data(), li->arena + li->off_cnt, cs.size() * 4, hipMemcpyDeviceToHost, stream));
    LI_HIP(hipStreamSynchronize(stream));
    memset(out, 0, sizeof *out);
    out->models = li->M;
    if (!li->trained) return GT_OK;
    out->trained_leaves = h.L;
    out->trained_keys = h.n_keys;
    out->lookups = h.lookups;
    out->fallbacks = h.fallbacks;
    for (const ModelFit& f : fs) {
        if (f.kind == kKindLinear) out->linear_models++;
        else if (f.kind == kKindMlp) out->mlp_models++;
        else out->tree_models++;
    }
    double wsum = 0, ksum = 0;
    for (uint64_t c = 0; c < cells; ++c) {
        if (!cs[c] || ps[c].lo > ps[c].hi) continue;
        const uint32_t w = static_cast<uint32_t>(ps[c].hi - ps[c].lo + 1);
        wsum += static_cast<double>(w) * cs[c];
        ksum += cs[c];
        if (w > out->max_window) out->max_window = w;
    }
    out->mean_window = ksum > 0 ? wsum / ksum : 0.0;
    out->declined = li->declined ? 1u : 0u;
    return GT_OK;
}

gt_status li_destroy(gt_learned* li) {
    if (!li) return GT_ERR_INVALID;
    delete li;
    return GT_OK;
}

}  // extern "C"

// ------------------------------------------------- serving runtime support

uint64_t gt_li_arena_bytes_like(const gt_learned* li) { return layout_li(nullptr, li->leaf_cap, li->M, li->t->kb); }

gt_status gt_li_create_like(const gt_learned* li, void* arena, uint64_t arena_bytes, gt_learned** out) {
    return li_create(li->t, &li->p, arena, arena_bytes, out);
}

void gt_li_rebind(gt_learned* li, gt_tree* t, uint64_t inserts_at_train, uint64_t deletes_at_train) {
    li->t = t;
    li->inserts_at_train = inserts_at_train;
    li->deletes_at_train = deletes_at_train;
    li->generation++;
}

void* gt_li_arena(const gt_learned* li) { return li->arena; }

void gt_li_swap_arenas(gt_learned* a, gt_learned* b) {
    std::swap(a->arena, b->arena);
    a->generation++;
    b->generation++;
}

void gt_li_exchange(gt_learned* a, gt_learned* b) {
    std::swap(*a, *b);
    // each handle's generation only grows, so graphs captured against either
    // handle's previous state are captured again
    const uint64_t g = std::max(a->generation, b->generation) + 1;
    a->generation = g;
    b->generation = g;
}
