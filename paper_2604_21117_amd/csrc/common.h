// Shared definitions of the HIP library: tree layout in the arena, the
// device header, the top-levels mirror and wave64 helpers.
//
// Layout (all in the caller's arena, 256-byte aligned regions):
//   DevHeader                      root, height, key count, pool cursors,
//                                  device error word
//   mirror                         copy of the top (up to three) inner levels
//                                  in breadth-first order, staged into LDS by
//                                  the search kernels
//   inner pool   ikeys[cap][16]    separators: entry i < c-1 is the largest key
//                                  below child i, entries from c-1 on hold the
//                                  largest key value (paper Section IV-E:
//                                  a key goes to the first child whose entry
//                                  is >= the key, so the child index is the
//                                  number of entries below the key)
//                                  -- except slot 15, which is never a
//                                  separator (at most 16 children): it holds
//                                  the first child reference when the node's
//                                  children have consecutive references (a
//                                  bulk-loaded node), so a search needs no
//                                  child line; a node an insert rewrites
//                                  gets the largest key there
//                ichild[cap][16]   child references, "none" from c on
//   leaf pool    lkeys[cap][16]    keys ascending; slots from count on repeat
//                                  the last key, so an equality ballot finds
//                                  a key without reading the count
//                lvals[cap][16]    values; slots from count on hold all ones
//                lmeta[cap]        {count, next leaf}
//   scratch                        per-batch work space of the insert path
//
// A u64 key line is 128 bytes and a u32 key line 64 bytes: one HBM line per
// node visit, read by 4, 8 or 16 lanes of a wavefront.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gt {

constexpr int kSlots = 16;                 // fanout = leaf capacity = entries per line
constexpr int kFirstSlot = kSlots - 1;     // inner key slot holding the first child reference
constexpr uint32_t kNone = 0xFFFFFFFFu;    // "no node"
constexpr uint32_t kLeafTag = 0x80000000u; // bit 31 marks a leaf reference
constexpr int kMirrorMaxNodes = 1 + 16 + 256;
constexpr int kMaxLevels = 16;             // height bound (>= 8 children per inner node)
constexpr uint32_t kErrCapacity = 0x1u;
constexpr uint32_t kErrInternal = 0x2u;
constexpr int kXcds = 8;                   // MI355X: 8 XCDs of 32 CUs, each with its own L2

template <class K>
__host__ __device__ constexpr K kmax() { return static_cast<K>(~static_cast<K>(0)); }

struct DevHeader {
    uint32_t root;       // node reference
    uint32_t height;     // levels, leaf level included
    uint64_t n_keys;
    uint32_t inner_used; // inner ids [0, inner_used) are allocated
    uint32_t leaf_used;
    uint32_t first_leaf;
    uint32_t error;      // kErr* bits, sticky until read by the host
    uint32_t epoch;      // applied insert batches
    uint32_t pad[7];
};
static_assert(sizeof(DevHeader) == 64, "DevHeader size");

// Mirror region: header, then node arrays sized for kMirrorMaxNodes.
struct MirrorHeader {
    uint32_t height;     // copy of DevHeader
    uint32_t root;
    uint64_t n_keys;
    uint32_t levels;     // inner levels held (0..3)
    uint32_t nodes;      // nodes held
    uint32_t nsplit;     // XCD splitter keys held (7, or 0 for a small tree)
    uint32_t pad[9];
};
static_assert(sizeof(MirrorHeader) == 64, "MirrorHeader size");

template <class K>
struct MirrorLayout {
    // byte offsets of the arrays for a mirror that holds `n` nodes
    static __host__ __device__ constexpr uint32_t keys_off() { return sizeof(MirrorHeader); }
    static __host__ __device__ constexpr uint32_t child_off(uint32_t n) { return keys_off() + n * kSlots * sizeof(K); }
    static __host__ __device__ constexpr uint32_t first_off(uint32_t n) { return child_off(n) + n * kSlots * 4; }
    static __host__ __device__ constexpr uint32_t bytes(uint32_t n) { return first_off(n) + ((n * 4 + 15) / 16) * 16; }
    // splitter keys live after the full-size arrays of the global mirror only
    static __host__ __device__ constexpr uint32_t split_off() { return bytes(kMirrorMaxNodes); }
    static __host__ __device__ constexpr uint32_t global_bytes() { return split_off() + 8 * sizeof(K); }
};

// nodes held by the first s levels of a full mirror (1, 17, 273)
__host__ __device__ constexpr uint32_t mirror_nodes_for_levels(int s) {
    return s <= 0 ? 0u : (s == 1 ? 1u : (s == 2 ? 17u : 273u));
}

template <class K>
struct TreeView {
    DevHeader* hdr;
    uint8_t* mirror;     // MirrorLayout<K> with kMirrorMaxNodes nodes
    K* ikeys;
    uint32_t* ichild;
    K* lkeys;
    K* lvals;
    uint2* lmeta;        // x = count, y = next
    uint32_t inner_cap;
    uint32_t leaf_cap;
};

// ----------------------------------------------------------- wave helpers

template <class T, int N>
struct alignas(sizeof(T) * N) VecN {
    T v[N];
};

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// bits of a wave ballot that belong to the G-lane group starting at gbase
template <int G>
__device__ __forceinline__ uint64_t group_bits(uint64_t m, int gbase) {
    if constexpr (G == 64) return m;
    else return (m >> gbase) & ((1ull << G) - 1ull);
}

__device__ __forceinline__ uint32_t shfl_u32(uint32_t v, int src) {
    return static_cast<uint32_t>(__shfl(static_cast<int>(v), src, 64));
}

// even split of `total` items into `parts`: part j holds [start(j), start(j+1))
__host__ __device__ __forceinline__ uint64_t part_start(uint64_t j, uint64_t total, uint64_t parts) {
    return j * total / parts;
}

// the part holding item `pos` under part_start
__host__ __device__ __forceinline__ uint64_t part_of(uint64_t pos, uint64_t total, uint64_t parts) {
    uint64_t j = pos * parts / total;
    while (j + 1 < parts && part_start(j + 1, total, parts) <= pos) ++j;
    while (j > 0 && part_start(j, total, parts) > pos) --j;
    return j;
}

// pieces an overfull node of `t` entries splits into (16 per node at most,
// at least 8 each when split)
__host__ __device__ __forceinline__ uint32_t split_pieces(uint64_t t) {
    return t <= kSlots ? 1u : static_cast<uint32_t>((t + kSlots - 1) / kSlots);
}

}  // namespace gt
