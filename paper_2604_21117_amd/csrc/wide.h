// The paper's key and node variants: 32-byte keys (Section IV-C) compared
// byte by byte with the most significant byte deciding (Section IV-E), and
// tree orders m = 16, 32 and 64 (Section V-C) -- a static tree, built once
// and searched (the paper's setting, Section V-B), beside the dynamic
// fanout-16 tree of the rest of the library.
//
// Layout in the caller's arena (256-byte aligned regions):
//   WideHeader                     root, height, key count, node counts
//   ikeys[inner][kw][m]            word-sliced 8-byte words: word w of
//                                  entry i (w = 0 most significant; a
//                                  32-byte key's words as big-endian
//                                  numbers).  Entry i < c-1: the largest key
//                                  below child i; entries from c-1 on: the
//                                  largest key value (all bytes 0xFF)
//   imeta[inner]                   {first child, children, tie mask (2 x
//                                  32 bits, low first)}: a bulk-loaded
//                                  node's children are consecutive ids of
//                                  the level below; bit i of the mask: entry
//                                  i's leading word equals that of the next
//                                  key in key order (the first key of child
//                                  i+1).  One 16-byte record per node, read
//                                  in one load
//   leaves of 8-byte keys: lkeys[leaves][m] up to m-1 keys ascending (the
//     paper's k_max = m - 1), slots from count on repeating the last key;
//     lvals[leaves][m] 8-byte values, all ones from count on
//   leaves of 32-byte keys (lkeys only, 40 bytes per entry): per leaf the
//     m leading words, then m 32-byte records {words 1..3, value}, words as
//     big-endian numbers; the same ordering and padding
//   lmeta[leaves]                  {count, next leaf}
// A key is kb = 8 * kw bytes: kw = 1 holds an 8-byte unsigned integer in
// native (little-endian) order, compared as an integer; kw = 4 holds the
// caller's 32 bytes as given, compared as a byte string.  Inner ids number
// the levels top-down (root 0), leaf ids follow key order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/gtree.h"

namespace gt {

struct WideHeader {
    uint32_t root;        // inner id 0, or leaf id 0 for a one-leaf tree
    uint32_t height;      // levels, leaf level included
    uint64_t n_keys;
    uint32_t n_inner;
    uint32_t n_leaves;
    uint32_t error;
    uint32_t pad[9];
};
static_assert(sizeof(WideHeader) == 64, "WideHeader size");

struct WideView {
    const WideHeader* hdr;
    const uint8_t* ikeys;
    const uint4* imeta;
    const uint8_t* lkeys;
    const uint64_t* lvals;
    const uint2* lmeta;
};

// Host record of a wide tree inside a gt_tree handle.
struct WideTree {
    int kw;               // 64-bit words per key: 1 or 4
    int m;                // order: children per inner node at most
    double fill;
    WideHeader* hdr;
    uint8_t* ikeys;
    uint4* imeta;
    uint8_t* lkeys;
    uint64_t* lvals;
    uint2* lmeta;
    uint64_t inner_cap, leaf_cap;
    uint64_t arena_bytes;
    uint32_t height;      // exact: the tree never changes after the build
};

// The parameter set selects the wide tree: key_bytes 32 with fanout 0
// (16), 16, 32 or 64, or key_bytes 8 with fanout 32 or 64.
bool wide_selected(const gt_params* p);
bool wide_params_ok(const gt_params* p);
uint64_t wide_arena_bytes(const gt_params* p, uint64_t n);
gt_status wide_build(const gt_params* p, const void* keys, const void* values, uint64_t n, void* arena,
                     uint64_t arena_bytes, hipStream_t s, WideTree** out);
gt_status wide_lookup(const WideTree* w, const void* keys, uint64_t B, void* values_out, uint8_t* found_out,
                      hipStream_t s);
gt_status wide_range(const WideTree* w, const void* lo, const void* hi, const uint32_t* max_out,
                     const uint64_t* out_offsets, uint64_t B, void* out_keys, void* out_values, uint32_t* count_out,
                     hipStream_t s);
gt_status wide_export(const WideTree* w, void* host_buf, uint64_t* bytes, hipStream_t s);
gt_status wide_stats(const WideTree* w, gt_tree_stats* out, hipStream_t s);
gt_status wide_device_error(const WideTree* w, hipStream_t s);

}  // namespace gt
