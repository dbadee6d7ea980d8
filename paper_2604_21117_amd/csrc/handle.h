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

// Serving-runtime support for retraining beside the serving index.
// Arena bytes of an index like `li` (same tree, parameters and models).
uint64_t gt_li_arena_bytes_like(const gt_learned* li);
// A new, untrained index over li's tree with li's parameters.
gt_status gt_li_create_like(const gt_learned* li, void* arena, uint64_t arena_bytes, gt_learned** out);
// Point `li` at tree handle `t` (another handle of the same layout, e.g. over
// a copy of the arena) and record the insert and delete counts of `t` that
// its training reflects: lookups then read `t`, and treat any later insert
// or delete as a change since training.
void gt_li_rebind(gt_learned* li, gt_tree* t, uint64_t inserts_at_train, uint64_t deletes_at_train);
// Exchange the whole states (arena, models, arguments) of two indexes over
// the same tree; launches already enqueued keep the state they captured.
void gt_li_exchange(gt_learned* a, gt_learned* b);
// The arena an index's state lives in, and the exchange of two indexes'
// arenas alone (for handing a state back into its owner's arena after a
// byte copy: the two arenas must then hold the same bytes).
void* gt_li_arena(const gt_learned* li);
void gt_li_swap_arenas(gt_learned* a, gt_learned* b);
// A handle over `arena`, a byte copy of t's arena: the same layout and
// parameters, no inserts or deletes counted.
struct gt_tree* gt_tree_clone_handle(const struct gt_tree* t, uint8_t* arena);
// Enqueue on `s` a copy of what training reads (header, child references of
// the inner nodes in use, keys and metadata of the leaves in use) from t's
// arena into the arena of `dst`, a clone handle of t.
gt_status gt_tree_copy_for_training(const struct gt_tree* t, struct gt_tree* dst, hipStream_t s);

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
    // pinned host word a delete reads its rebuild flag into (low half), with
    // the number of the delete call that stored it (high half)
    uint64_t* h_flag = nullptr;
    uint64_t* d_flag = nullptr;  // the same word's device address
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
