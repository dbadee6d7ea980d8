// Bulk build and the top-levels mirror.
//
// The paper builds its tree once on the host, flattens it breadth-first into
// equal-size nodes and copies it to device memory (Sections IV-B, V-B).
// Here the build runs on the device from sorted distinct keys: L leaves get
// the keys evenly (leaf j holds [j*n/L, (j+1)*n/L)), then each inner level
// is packed over the level below with the same even rule, bottom-up.  Inner
// ids are numbered top-down (root = 0), so the top levels are contiguous.
// The node counts follow from the packing rule: at fill 1.0 and 16^k keys
// the tree has sum_{i<h} 16^i nodes (Section III's N_max).
//
// The mirror holds up to three top inner levels in breadth-first order with,
// per node, its key line, its child line (real references) and the mirror
// index of its first child.  Search kernels copy it into LDS or read it from
// L2.  It is rebuilt (mirror.h) after an insert that rewrites a node of its
// levels or grows the root; inserts of up to 64 keys rebuild it in their own
// kernel.
#include "common.h"
#include "kernels.h"
#include "mirror.h"

namespace gt {

template <class K>
__global__ void k_gather(const K* __restrict__ src, const uint32_t* __restrict__ idx, K* __restrict__ dst,
                         uint64_t n) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        dst[i] = src[idx[i]];
}

template <class K>
__global__ void k_dup_check(const K* __restrict__ sk, uint64_t n, uint32_t* flag) {
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; i + 1 < n;
         i += static_cast<uint64_t>(gridDim.x) * blockDim.x)
        if (sk[i] == sk[i + 1]) atomicOr(flag, 1u);
}

template <class K>
__global__ void k_build_leaves(TreeView<K> t, const K* __restrict__ sk, const K* __restrict__ sv, uint64_t n,
                               uint64_t L, K* __restrict__ maxk) {
    for (uint64_t tid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; tid < L * kSlots;
         tid += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t j = tid / kSlots, s = tid % kSlots;
        const uint64_t b = part_start(j, n, L), e = part_start(j + 1, n, L);
        const uint64_t c = e - b;
        K key, val;
        if (s < c) { key = sk[b + s]; val = sv[b + s]; }
        else { key = c ? sk[e - 1] : kmax<K>(); val = kmax<K>(); }
        t.lkeys[tid] = key;
        t.lvals[tid] = val;
        if (s == 0) {
            t.lmeta[j] = make_uint2(static_cast<uint32_t>(c), j + 1 < L ? static_cast<uint32_t>(j + 1) : kNone);
            maxk[j] = c ? sk[e - 1] : kmax<K>();
        }
    }
}

template <class K>
__global__ void k_build_inner(TreeView<K> t, const K* __restrict__ cmax, uint64_t C, uint64_t P,
                              uint32_t child_base, int child_is_leaf, uint32_t node_base, K* __restrict__ nmax) {
    for (uint64_t tid = blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x; tid < P * kSlots;
         tid += static_cast<uint64_t>(gridDim.x) * blockDim.x) {
        const uint64_t j = tid / kSlots, s = tid % kSlots;
        const uint64_t b = part_start(j, C, P), e = part_start(j + 1, C, P);
        const uint64_t c = e - b;
        uint32_t ref = kNone;
        if (s < c) ref = child_is_leaf ? (kLeafTag | static_cast<uint32_t>(b + s)) : child_base + static_cast<uint32_t>(b + s);
        K sep = (s + 1 < c) ? cmax[b + s] : kmax<K>();
        // slot 15: the first child reference (children are consecutive)
        if (s == kFirstSlot) sep = static_cast<K>(child_is_leaf ? (kLeafTag | static_cast<uint32_t>(b))
                                                                : child_base + static_cast<uint32_t>(b));
        const uint64_t node = node_base + j;
        t.ikeys[node * kSlots + s] = sep;
        t.ichild[node * kSlots + s] = ref;
        if (s == 0) nmax[j] = cmax[e - 1];
    }
}

__global__ void k_set_header(DevHeader* h, uint32_t root, uint32_t height, uint64_t n_keys, uint32_t inner_used,
                             uint32_t leaf_used) {
    if (threadIdx.x == 0) {
        h->root = root;
        h->height = height;
        h->n_keys = n_keys;
        h->inner_used = inner_used;
        h->leaf_used = leaf_used;
        h->first_leaf = 0;
        h->error = 0;
        h->epoch = 0;
    }
}

// One workgroup of 256 threads.  With `dirty` given, nothing happens unless
// *dirty is set.
template <class K>
__global__ __launch_bounds__(256) void k_mirror_refresh(TreeView<K> t, const uint32_t* dirty) {
    if (dirty && *dirty == 0) return;
    mirror_refresh_body<K, 256>(t);
}

__global__ void k_clear_error(DevHeader* h) {
    if (threadIdx.x == 0) h->error = 0;
}

void launch_clear_error(DevHeader* h, hipStream_t s) {
    hipLaunchKernelGGL(k_clear_error, dim3(1), dim3(64), 0, s, h);
}

static uint32_t grid1d(uint64_t n, uint32_t block) {
    uint64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return static_cast<uint32_t>(g);
}

template <class K>
void launch_gather(const K* src, const uint32_t* idx, K* dst, uint64_t n, hipStream_t s) {
    if (!n) return;
    hipLaunchKernelGGL(k_gather<K>, dim3(grid1d(n, 256)), dim3(256), 0, s, src, idx, dst, n);
}

template <class K>
void launch_dup_check(const K* sk, uint64_t n, uint32_t* flag, hipStream_t s) {
    if (n < 2) return;
    hipLaunchKernelGGL(k_dup_check<K>, dim3(grid1d(n, 256)), dim3(256), 0, s, sk, n, flag);
}

template <class K>
void launch_mirror_refresh(const TreeView<K>& t, hipStream_t s) {
    hipLaunchKernelGGL(k_mirror_refresh<K>, dim3(1), dim3(256), 0, s, t, nullptr);
}

template <class K>
void launch_build(const TreeView<K>& t, const K* sk, const K* sv, uint64_t n, const uint64_t* level_sizes,
                  int levels, K* maxbuf, hipStream_t s) {
    const uint64_t L = level_sizes[0];
    uint64_t maxsz = 0;
    for (int i = 0; i < levels; ++i) maxsz = level_sizes[i] > maxsz ? level_sizes[i] : maxsz;
    K* cur = maxbuf;
    K* nxt = maxbuf + maxsz;
    hipLaunchKernelGGL(k_build_leaves<K>, dim3(grid1d(L * kSlots, 256)), dim3(256), 0, s, t, sk, sv, n, L, cur);
    // inner ids top-down: level i (i >= 1 above the leaves) starts after all
    // levels above it
    uint64_t base[kMaxLevels + 1] = {0};
    {
        uint64_t acc = 0;
        for (int i = levels - 1; i >= 1; --i) { base[i] = acc; acc += level_sizes[i]; }
    }
    for (int i = 1; i < levels; ++i) {
        const uint64_t C = level_sizes[i - 1], P = level_sizes[i];
        const uint32_t child_base = i == 1 ? 0u : static_cast<uint32_t>(base[i - 1]);
        hipLaunchKernelGGL(k_build_inner<K>, dim3(grid1d(P * kSlots, 256)), dim3(256), 0, s, t, cur, C, P,
                           child_base, i == 1 ? 1 : 0, static_cast<uint32_t>(base[i]), nxt);
        K* tk = cur; cur = nxt; nxt = tk;
    }
    uint64_t inner_total = 0;
    for (int i = 1; i < levels; ++i) inner_total += level_sizes[i];
    const uint32_t root = levels == 1 ? (kLeafTag | 0u) : 0u;
    hipLaunchKernelGGL(k_set_header, dim3(1), dim3(64), 0, s, t.hdr, root, static_cast<uint32_t>(levels), n,
                       static_cast<uint32_t>(inner_total), static_cast<uint32_t>(L));
    launch_mirror_refresh<K>(t, s);
}

template void launch_gather<uint32_t>(const uint32_t*, const uint32_t*, uint32_t*, uint64_t, hipStream_t);
template void launch_gather<uint64_t>(const uint64_t*, const uint32_t*, uint64_t*, uint64_t, hipStream_t);
template void launch_dup_check<uint32_t>(const uint32_t*, uint64_t, uint32_t*, hipStream_t);
template void launch_dup_check<uint64_t>(const uint64_t*, uint64_t, uint32_t*, hipStream_t);
template void launch_mirror_refresh<uint32_t>(const TreeView<uint32_t>&, hipStream_t);
template void launch_mirror_refresh<uint64_t>(const TreeView<uint64_t>&, hipStream_t);
template void launch_build<uint32_t>(const TreeView<uint32_t>&, const uint32_t*, const uint32_t*, uint64_t,
                                     const uint64_t*, int, uint32_t*, hipStream_t);
template void launch_build<uint64_t>(const TreeView<uint64_t>&, const uint64_t*, const uint64_t*, uint64_t,
                                     const uint64_t*, int, uint64_t*, hipStream_t);

}  // namespace gt
