// Root-to-leaf traversal by groups of G lanes of a wave64 (G = 4, 8 or 16).
//
// A node line holds 16 entries; lane l of a group holds entries
// [l*KPL, (l+1)*KPL) with KPL = 16/G, loaded with one 8/16/32-byte vector
// load, so the group reads the 128-byte (u64) or 64-byte (u32) line once.
// The paper's comparison module (Section IV-E) compares the search key with
// every entry of the node in parallel and a priority encoder picks the first
// entry that is >= the key; here each lane compares its entries, a wave
// ballot per entry position collects the "entry < key" bits, and the popcount
// of the group's bits is the child index (entries past the last child hold
// the largest key, so they never count).  The child reference is taken from
// the lane that holds it with one cross-lane read.
//
// Each group walks QPG queries at once, level by level, so a wave keeps
// QPG independent node loads in flight per group (memory-level parallelism
// for the dependent chain of node loads).  All leaves are at the same depth,
// so every group of a wave runs the same number of levels and ballots stay
// wave-uniform.
#pragma once
#include "common.h"

namespace gt {

// Load n elements of T (n * sizeof(T) = 4, 8, 16 or 32 bytes, naturally
// aligned) with 4/8/16-byte vector loads into registers.
template <class T, int N>
__device__ __forceinline__ void load_vec(const T* p, T (&out)[N]) {
    constexpr int bytes = N * static_cast<int>(sizeof(T));
    if constexpr (bytes >= 16) {
#pragma unroll
        for (int c = 0; c < bytes / 16; ++c) {
            const uint4 x = reinterpret_cast<const uint4*>(p)[c];
            __builtin_memcpy(&out[c * (16 / sizeof(T))], &x, 16);
        }
    } else if constexpr (bytes == 8) {
        const uint2 x = *reinterpret_cast<const uint2*>(p);
        __builtin_memcpy(&out[0], &x, 8);
    } else {
        const uint32_t x = *reinterpret_cast<const uint32_t*>(p);
        __builtin_memcpy(&out[0], &x, 4);
    }
}

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));

// As load_vec, with non-temporal loads (streamed lines, low cache priority).
template <class T, int N>
__device__ __forceinline__ void load_vec_nt(const T* p, T (&out)[N]) {
    constexpr int bytes = N * static_cast<int>(sizeof(T));
    if constexpr (bytes >= 16) {
#pragma unroll
        for (int c = 0; c < bytes / 16; ++c) {
            const u32x4_t x = __builtin_nontemporal_load(reinterpret_cast<const u32x4_t*>(p) + c);
            __builtin_memcpy(&out[c * (16 / sizeof(T))], &x, 16);
        }
    } else {
        load_vec<T, N>(p, out);
    }
}

template <class K, int G>
struct Trav {
    static constexpr int KPL = kSlots / G;
    struct KV { K v[KPL]; };
    struct CV { uint32_t v[KPL]; };

    // child index = number of separators below `key` in the group's line
    // (slots 0..14; slot 15 is never a separator, see kFirstSlot)
    static __device__ __forceinline__ uint32_t child_index(const KV& kv, K key, int gbase) {
        uint32_t idx = 0;
#pragma unroll
        for (int e = 0; e < KPL; ++e) {
            uint64_t m = __ballot(kv.v[e] < key);
            if (e == KPL - 1) m &= ~(1ull << (gbase + G - 1));
            idx += static_cast<uint32_t>(__popcll(group_bits<G>(m, gbase)));
        }
        return idx;
    }

    // slot 15 of the group's line: the first child reference when the node's
    // children have consecutive references, else the largest key
    static __device__ __forceinline__ K first_slot(const KV& kv, int gbase) {
        return static_cast<K>(__shfl(kv.v[KPL - 1], gbase + G - 1, 64));
    }

    // children of an inner node from its key line: a node with C children
    // has C - 1 separators in slots 0..C-2 and the largest key in the other
    // slots below slot 15 (no separator is the largest key: that key can
    // only lie in the last child)
    static __device__ __forceinline__ uint32_t child_count(const KV& kv, int gl, int gbase) {
        uint32_t c = 1;
#pragma unroll
        for (int e = 0; e < KPL; ++e) {
            const bool sep = gl * KPL + e < kFirstSlot && kv.v[e] != kmax<K>();
            c += static_cast<uint32_t>(__popcll(group_bits<G>(__ballot(sep), gbase)));
        }
        return c;
    }

    // child reference for slot idx, read from the lane that holds it
    static __device__ __forceinline__ uint32_t pick_child(const CV& cv, uint32_t idx, int gbase) {
        uint32_t e = idx % KPL;
        uint32_t mine = cv.v[0];
#pragma unroll
        for (int j = 1; j < KPL; ++j)
            if (e == static_cast<uint32_t>(j)) mine = cv.v[j];
        return shfl_u32(mine, gbase + static_cast<int>(idx / KPL));
    }

    // value in slot `slot` of a line held KPL-per-lane by the group
    static __device__ __forceinline__ K pick_value(const KV& vv, uint32_t slot, int gbase) {
        uint32_t e = slot % KPL;
        K mine = vv.v[0];
#pragma unroll
        for (int j = 1; j < KPL; ++j)
            if (e == static_cast<uint32_t>(j)) mine = vv.v[j];
        return __shfl(mine, gbase + static_cast<int>(slot / KPL), 64);
    }

    // first slot whose key equals `key`, or 16 if none
    static __device__ __forceinline__ uint32_t match_slot(const KV& kv, K key, int gbase) {
        uint32_t best = kSlots;
#pragma unroll
        for (int e = 0; e < KPL; ++e) {
            uint64_t m = group_bits<G>(__ballot(kv.v[e] == key), gbase);
            if (m) {
                uint32_t s = static_cast<uint32_t>(__builtin_ctzll(m)) * KPL + e;
                best = s < best ? s : best;
            }
        }
        return best;
    }

    static __device__ __forceinline__ KV load_keys(const K* line, int gl) {
        KV r;
        load_vec<K, KPL>(line + gl * KPL, r.v);
        return r;
    }
    static __device__ __forceinline__ KV load_keys_nt(const K* line, int gl) {
        KV r;
        load_vec_nt<K, KPL>(line + gl * KPL, r.v);
        return r;
    }
    static __device__ __forceinline__ CV load_child(const uint32_t* line, int gl) {
        CV r;
        load_vec<uint32_t, KPL>(line + gl * KPL, r.v);
        return r;
    }
};

// Copy the first `nodes` mirror nodes (header, keys, children, first-child
// indices) from global memory into LDS.  Called by the whole workgroup.
template <class K>
__device__ __forceinline__ void stage_mirror(const uint8_t* mirror, uint8_t* lds, uint32_t nodes) {
    using ML = MirrorLayout<K>;
    constexpr uint32_t full = kMirrorMaxNodes;
    // header + keys prefix
    const uint32_t kbytes = ML::keys_off() + nodes * kSlots * sizeof(K);
    const uint32_t cbytes = nodes * kSlots * 4;
    const uint32_t fbytes = ((nodes * 4 + 15) / 16) * 16;
    const uint4* src0 = reinterpret_cast<const uint4*>(mirror);
    uint4* dst0 = reinterpret_cast<uint4*>(lds);
    for (uint32_t i = threadIdx.x; i < kbytes / 16; i += blockDim.x) dst0[i] = src0[i];
    const uint4* src1 = reinterpret_cast<const uint4*>(mirror + ML::child_off(full));
    uint4* dst1 = reinterpret_cast<uint4*>(lds + ML::child_off(nodes));
    for (uint32_t i = threadIdx.x; i < cbytes / 16; i += blockDim.x) dst1[i] = src1[i];
    const uint4* src2 = reinterpret_cast<const uint4*>(mirror + ML::first_off(full));
    uint4* dst2 = reinterpret_cast<uint4*>(lds + ML::first_off(nodes));
    for (uint32_t i = threadIdx.x; i < fbytes / 16; i += blockDim.x) dst2[i] = src2[i];
}

// Walk QPG keys from the root to their leaves.
//   mir      mirror (LDS copy holding `mnodes` nodes, or the global mirror
//            with mnodes = kMirrorMaxNodes)
//   use_lv   mirror levels to use (clamped to the levels the mirror holds)
// On return leaf[j] is the leaf index (tag removed) for key[j].
// If REC is set, path_node[l][j] / path_idx[l][j] receive the inner node and
// child slot taken at inner level l (0 = root level) for l < height-1, and
// path_cnt[l][j] (if given) that node's number of children.
template <class K, int G, int QPG, bool REC>
__device__ __forceinline__ void descend(const TreeView<K>& t, const uint8_t* mir, uint32_t mnodes, int use_lv,
                                        const K (&key)[QPG], uint32_t (&leaf)[QPG], int gl, int gbase,
                                        uint32_t* path_node = nullptr, uint8_t* path_idx = nullptr,
                                        uint64_t path_stride = 0, const uint64_t* qidx = nullptr,
                                        uint8_t* path_cnt = nullptr) {
    using T = Trav<K, G>;
    using ML = MirrorLayout<K>;
    const MirrorHeader* mh = reinterpret_cast<const MirrorHeader*>(mir);
    const int height = static_cast<int>(mh->height);
    const int inner_levels = height - 1;
    int lv = use_lv < static_cast<int>(mh->levels) ? use_lv : static_cast<int>(mh->levels);
    if (lv > inner_levels) lv = inner_levels;
    const K* mkeys = reinterpret_cast<const K*>(mir + ML::keys_off());
    const uint32_t* mchild = reinterpret_cast<const uint32_t*>(mir + ML::child_off(mnodes));
    const uint32_t* mfirst = reinterpret_cast<const uint32_t*>(mir + ML::first_off(mnodes));

    uint32_t node[QPG];
    const uint32_t root = mh->root;
#pragma unroll
    for (int j = 0; j < QPG; ++j) node[j] = root;

    int level = 0;
    if (lv > 0) {
        uint32_t m[QPG];
#pragma unroll
        for (int j = 0; j < QPG; ++j) m[j] = 0;
        for (; level < lv; ++level) {
            typename T::KV kv[QPG];
            typename T::CV cv[QPG];
#pragma unroll
            for (int j = 0; j < QPG; ++j) {
                kv[j] = T::load_keys(mkeys + m[j] * kSlots, gl);
                cv[j] = T::load_child(mchild + m[j] * kSlots, gl);
            }
#pragma unroll
            for (int j = 0; j < QPG; ++j) {
                uint32_t idx = T::child_index(kv[j], key[j], gbase);
                uint32_t c = T::pick_child(cv[j], idx, gbase);
                if constexpr (REC) {
                    const uint32_t nc = path_cnt ? T::child_count(kv[j], gl, gbase) : 0u;
                    if (gl == 0 && qidx[j] != ~0ull) {
                        path_node[level * path_stride + qidx[j]] = node[j];
                        path_idx[level * path_stride + qidx[j]] = static_cast<uint8_t>(idx);
                        if (path_cnt) path_cnt[level * path_stride + qidx[j]] = static_cast<uint8_t>(nc);
                    }
                }
                node[j] = c;
                if (level + 1 < lv) m[j] = mfirst[m[j]] + idx;
            }
        }
    }
    // HBM levels: a node whose children are consecutive gives its child
    // reference from the key line alone; only other nodes (rewritten by an
    // insert) cost a dependent read of the child line
    for (; level < inner_levels; ++level) {
        typename T::KV kv[QPG];
#pragma unroll
        for (int j = 0; j < QPG; ++j) kv[j] = T::load_keys(t.ikeys + static_cast<uint64_t>(node[j]) * kSlots, gl);
#pragma unroll
        for (int j = 0; j < QPG; ++j) {
            const uint32_t idx = T::child_index(kv[j], key[j], gbase);
            const K f = T::first_slot(kv[j], gbase);
            uint32_t c;
            if (f != kmax<K>()) {
                c = static_cast<uint32_t>(f) + idx;
            } else {
                const typename T::CV cv = T::load_child(t.ichild + static_cast<uint64_t>(node[j]) * kSlots, gl);
                c = T::pick_child(cv, idx, gbase);
            }
            if constexpr (REC) {
                const uint32_t nc = path_cnt ? T::child_count(kv[j], gl, gbase) : 0u;
                if (gl == 0 && qidx[j] != ~0ull) {
                    path_node[level * path_stride + qidx[j]] = node[j];
                    path_idx[level * path_stride + qidx[j]] = static_cast<uint8_t>(idx);
                    if (path_cnt) path_cnt[level * path_stride + qidx[j]] = static_cast<uint8_t>(nc);
                }
            }
            node[j] = c;
        }
    }
#pragma unroll
    for (int j = 0; j < QPG; ++j) leaf[j] = node[j] & ~kLeafTag;
}

}  // namespace gt
