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
// index of its first child.  Search kernels copy it into LDS.  It is rebuilt
// after every change to the tree.
#include "common.h"
#include "kernels.h"

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
        if (sk[i] == sk[i + 1]) *flag = 1u;
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
// *dirty is set.  Child references of a node fill its first slots, so a
// node's child count is the number of set bits of one ballot and a child's
// rank is its slot.
template <class K>
__global__ __launch_bounds__(256) void k_mirror_refresh(TreeView<K> t, const uint32_t* dirty) {
    if (dirty && *dirty == 0) return;
    using ML = MirrorLayout<K>;
    constexpr uint32_t full = kMirrorMaxNodes;
    constexpr int kCopyBatch = 6;  // node slots in flight per thread
    __shared__ uint32_t ids[kMirrorMaxNodes];
    __shared__ uint32_t cnt1[kSlots];
    __shared__ uint32_t pre1[kSlots + 1];
    __shared__ uint32_t counts[3];
    const uint32_t tid = threadIdx.x;
    const int lane = lane_id();
    const uint32_t height = t.hdr->height;
    const uint32_t root = t.hdr->root;
    const uint64_t n_keys = t.hdr->n_keys;
    const uint32_t levels = height >= 4 ? 3u : height - 1u;
    if (tid == 0) { counts[0] = levels >= 1 ? 1u : 0u; counts[1] = 0; counts[2] = 0; ids[0] = root; }
    if (levels >= 2 && tid < 64) {
        const uint32_t c = tid < kSlots ? t.ichild[static_cast<uint64_t>(root) * kSlots + tid] : kNone;
        if (tid < kSlots) ids[1 + tid] = c;
        const uint64_t m = __ballot(c != kNone);
        if (tid == 0) counts[1] = static_cast<uint32_t>(__popcll(m));
    }
    __syncthreads();
    if (levels >= 3) {
        const uint32_t n1 = counts[1];
        const uint32_t p = tid / kSlots, i = tid % kSlots;
        uint32_t c = kNone;
        if (p < n1) c = t.ichild[static_cast<uint64_t>(ids[1 + p]) * kSlots + i];
        const uint64_t m = __ballot(c != kNone);
        if (i == 0 && p < kSlots) cnt1[p] = static_cast<uint32_t>(__popcll((m >> (lane & ~15)) & 0xFFFFull));
        __syncthreads();
        if (tid <= n1) {
            uint32_t acc = 0;
            for (uint32_t q = 0; q < tid; ++q) acc += cnt1[q];
            pre1[tid] = acc;
            if (tid == n1) counts[2] = acc;
        }
        __syncthreads();
        if (c != kNone) ids[1 + n1 + pre1[p] + i] = c;
        __syncthreads();
    }
    const uint32_t n1 = counts[1], n2 = counts[2];
    const uint32_t nodes = counts[0] + n1 + n2;
    K* __restrict__ mkeys = reinterpret_cast<K*>(t.mirror + ML::keys_off());
    uint32_t* __restrict__ mchild = reinterpret_cast<uint32_t*>(t.mirror + ML::child_off(full));
    uint32_t* __restrict__ mfirst = reinterpret_cast<uint32_t*>(t.mirror + ML::first_off(full));
    const K* __restrict__ ikeys = t.ikeys;
    const uint32_t* __restrict__ ichild = t.ichild;
    const uint32_t slots = nodes * kSlots;
    for (uint32_t x0 = tid; x0 < slots; x0 += 256 * kCopyBatch) {
        K kk[kCopyBatch];
        uint32_t cc[kCopyBatch];
#pragma unroll
        for (int q = 0; q < kCopyBatch; ++q) {
            const uint32_t x = x0 + q * 256;
            if (x < slots) {
                const uint64_t at = static_cast<uint64_t>(ids[x / kSlots]) * kSlots + x % kSlots;
                kk[q] = ikeys[at];
                cc[q] = ichild[at];
            }
        }
#pragma unroll
        for (int q = 0; q < kCopyBatch; ++q) {
            const uint32_t x = x0 + q * 256;
            if (x < slots) {
                mkeys[x] = kk[q];
                mchild[x] = cc[q];
            }
        }
    }
    for (uint32_t m = tid; m < nodes; m += 256) {
        uint32_t f = 0;
        if (m == 0 && levels >= 2) f = 1;
        else if (m >= 1 && m < 1 + n1 && levels >= 3) f = 1 + n1 + pre1[m - 1];
        mfirst[m] = f;
    }
    // XCD splitters: the key space is cut into kXcds ranges of (nearly) equal
    // numbers of level-2 subtrees (level-1 subtrees for a 3-level tree); the
    // cut after subtree e is that subtree's upper bound, read from its
    // parent's separator or, for a last child, from the grandparent's.  One
    // thread per cut.
    K* sp = reinterpret_cast<K*>(t.mirror + ML::split_off());
    const K* rsep = ikeys + static_cast<uint64_t>(root) * kSlots;
    uint32_t nsplit = 0;
    if (levels >= 3 && n2 >= static_cast<uint32_t>(kXcds)) {
        nsplit = kXcds - 1;
        if (tid < nsplit) {
            const uint32_t e = static_cast<uint32_t>((tid + 1) * n2 / kXcds - 1);
            uint32_t p = 0;
            while (p + 1 < n1 && pre1[p + 1] <= e) ++p;
            const uint32_t i = e - pre1[p];
            const uint32_t cnt = pre1[p + 1] - pre1[p];
            K ub;
            if (i + 1 < cnt) ub = ikeys[static_cast<uint64_t>(ids[1 + p]) * kSlots + i];
            else ub = (p + 1 < n1) ? rsep[p] : kmax<K>();
            sp[tid] = ub;
        }
    } else if (levels >= 2 && n1 >= static_cast<uint32_t>(kXcds)) {
        nsplit = kXcds - 1;
        if (tid < nsplit) {
            const uint32_t e = static_cast<uint32_t>((tid + 1) * n1 / kXcds - 1);
            sp[tid] = (e + 1 < n1) ? rsep[e] : kmax<K>();
        }
    }
    if (tid == 0) {
        MirrorHeader* mh = reinterpret_cast<MirrorHeader*>(t.mirror);
        mh->height = height;
        mh->root = root;
        mh->n_keys = n_keys;
        mh->levels = levels;
        mh->nodes = nodes;
        mh->nsplit = nsplit;
    }
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
void launch_mirror_refresh_if(const TreeView<K>& t, const uint32_t* dirty, hipStream_t s) {
    hipLaunchKernelGGL(k_mirror_refresh<K>, dim3(1), dim3(256), 0, s, t, dirty);
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
template void launch_mirror_refresh_if<uint32_t>(const TreeView<uint32_t>&, const uint32_t*, hipStream_t);
template void launch_mirror_refresh_if<uint64_t>(const TreeView<uint64_t>&, const uint32_t*, hipStream_t);
template void launch_build<uint32_t>(const TreeView<uint32_t>&, const uint32_t*, const uint32_t*, uint64_t,
                                     const uint64_t*, int, uint32_t*, hipStream_t);
template void launch_build<uint64_t>(const TreeView<uint64_t>&, const uint64_t*, const uint64_t*, uint64_t,
                                     const uint64_t*, int, uint64_t*, hipStream_t);

}  // namespace gt
