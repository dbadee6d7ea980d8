// The tree handle (host memory) shared by the library's host-side files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/gtree.h"
#include "common.h"
#include "kernels.h"
#include "wide.h"

// Changes whenever li_train or li_set_bounds changes what a learned lookup
// launch captures (kernel arguments, tables); a cached graph of an older
// generation must be captured again.
uint64_t gt_li_generation(const gt_learned* li);

struct gt_tree {
    gt_params p;
    int kb;
    uint8_t* arena;
    uint64_t arena_bytes;   // bytes used
    gt::DevHeader* hdr;
    uint8_t* mirror;
    void* ikeys;
    uint32_t* ichild;
    void* lkeys;
    void* lvals;
    uint2* lmeta;
    uint64_t inner_cap, leaf_cap;
    uint8_t* scratch;
    uint64_t scratch_bytes;
    uint64_t max_batch;
    gt::LaunchCfg cfg;
    uint32_t h_bound;       // the tree's height or more (exact after the build;
                            // after an insert, the most the pool sizes allow)
    uint64_t inserts = 0;   // insert batches enqueued on this tree
    uint64_t deletes = 0;   // delete batches applied to this tree
    uint32_t* h_flag = nullptr;  // pinned host word a delete reads its rebuild flag into
    gt::WideTree* wide = nullptr;  // set for a tree of 32-byte keys or order 32/64:
                                   // static, searched by wide.hip; the fields
                                   // above are then unused
};


namespace gt {

template <class K>
inline TreeView<K> view(const gt_tree* t) {
    TreeView<K> v;
    v.hdr = t->hdr;
    v.mirror = t->mirror;
    v.ikeys = reinterpret_cast<K*>(t->ikeys);
    v.ichild = t->ichild;
    v.lkeys = reinterpret_cast<K*>(t->lkeys);
    v.lvals = reinterpret_cast<K*>(t->lvals);
    v.lmeta = t->lmeta;
    v.inner_cap = static_cast<uint32_t>(t->inner_cap);
    v.leaf_cap = static_cast<uint32_t>(t->leaf_cap);
    return v;
}


}  // namespace gt
