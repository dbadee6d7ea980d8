// Internal launch functions of the library (host side).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "common.h"
#include "../../include/gtree.h"

namespace gt {

struct LaunchCfg {
    int lanes;              // lanes per query: 4, 8, 16
    int queries_per_group;  // queries interleaved per lane group: 1, 2, 4
    int lds_levels;         // top inner levels read from LDS: 0..3
    int value_coload;       // read a leaf's value line together with its key line
    int xcd_split;          // 0 off, 1 on from kXcdMinBatch queries, 2 always
    int leaf_stream;        // non-temporal leaf loads: 0 value lines from kLargeBatch queries, 1 key and value lines, 2 none
    int large_qpg;          // queries per group from kLargeBatch queries on (0 = same)
    int shape_auto;         // lookup shape chosen by batch size: bit 0 lanes, 1 queries per group, 2 LDS levels
};

constexpr uint64_t kXcdMinBatch = 1u << 15;
constexpr uint64_t kLargeBatch = 1u << 15;
constexpr uint64_t kMidBatch = 1u << 13;

template <class K>
void launch_lookup(const TreeView<K>& t, const LaunchCfg& cfg, const K* q, uint64_t B, K* vout, uint8_t* fout,
                   hipStream_t s);

template <class K>
void launch_range(const TreeView<K>& t, const LaunchCfg& cfg, const K* lo, const K* hi, const uint32_t* mx,
                  const uint64_t* off, uint64_t B, K* ok, K* ov, uint32_t* cnt, hipStream_t s);

// Bulk build from sorted distinct keys (sk, sv): writes leaves, inner levels,
// header and mirror.  level_sizes[0] = leaves, level_sizes[i] = nodes of the
// i-th inner level above the leaves; `levels` entries, the last being 1.
// maxbuf needs room for max(level_sizes) keys, twice.
template <class K>
void launch_build(const TreeView<K>& t, const K* sk, const K* sv, uint64_t n, const uint64_t* level_sizes,
                  int levels, K* maxbuf, hipStream_t s);

template <class K>
void launch_gather(const K* src, const uint32_t* idx, K* dst, uint64_t n, hipStream_t s);

template <class K>
void launch_dup_check(const K* sk, uint64_t n, uint32_t* flag, hipStream_t s);

template <class K>
void launch_mirror_refresh(const TreeView<K>& t, hipStream_t s);


// Clear the device error word with a kernel (safe inside a captured graph).
void launch_clear_error(DevHeader* h, hipStream_t s);

// Workspace of a level-wise lookup batch: byte offsets of the two FIFOs
// (per 64-query window a run-start mask, per query a node reference) and,
// unless the batch arrives sorted, the sort buffers.
struct LwLayout {
    uint64_t ha, hb, ra, rb, sk, si, sk2, si2, tmp, total;
};
LwLayout lw_layout(uint64_t B, int key_bytes, bool presorted);

// Size of the fixed scratch array of the allocation-free level-wise lookup
// (per device), and its address on the current device (resolved once per
// device, then cached).
constexpr uint64_t kLwScratchBytes = GT_LW_NOALLOC_SCRATCH_BYTES;
hipError_t lw_scratch(void** out);

// Level-wise lookup: sort the batch (unless presorted), then one kernel per
// level for `levels` levels (at least the tree's height).
template <class K>
void launch_lookup_levelwise(const TreeView<K>& t, const K* keys, uint64_t B, bool presorted, uint32_t levels,
                             K* vout, uint8_t* fout, void* ws, hipStream_t s);

}  // namespace gt
