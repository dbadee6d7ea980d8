// Top-levels mirror rebuild, shared by the refresh kernel and the
// small-batch insert kernel.
#pragma once
#include "common.h"

namespace gt {

// Rebuild of the top-levels mirror by one workgroup of NT >= 256 threads
// (every thread must call it).  Child references of a node fill its first
// slots, so a node's child count is the number of set bits of one ballot and
// a child's rank is its slot.
template <class K, int NT>
__device__ __forceinline__ void mirror_refresh_body(TreeView<K> t) {
    static_assert(NT >= 256 && NT % 64 == 0, "one thread per level-2 slot");
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
        if (p < n1 && p < kSlots) c = t.ichild[static_cast<uint64_t>(ids[1 + p]) * kSlots + i];
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
        if (c != kNone) ids[1 + n1 + pre1[p] + i] = c;  // c set only for p < n1
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
    for (uint32_t x0 = tid; x0 < slots; x0 += NT * kCopyBatch) {
        K kk[kCopyBatch];
        uint32_t cc[kCopyBatch];
#pragma unroll
        for (int q = 0; q < kCopyBatch; ++q) {
            const uint32_t x = x0 + q * NT;
            if (x < slots) {
                const uint64_t at = static_cast<uint64_t>(ids[x / kSlots]) * kSlots + x % kSlots;
                kk[q] = ikeys[at];
                cc[q] = ichild[at];
            }
        }
#pragma unroll
        for (int q = 0; q < kCopyBatch; ++q) {
            const uint32_t x = x0 + q * NT;
            if (x < slots) {
                mkeys[x] = kk[q];
                mchild[x] = cc[q];
            }
        }
    }
    for (uint32_t m = tid; m < nodes; m += NT) {
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

}  // namespace gt
