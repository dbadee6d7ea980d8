// Insert path (sort, merge, split, parent-split propagation) and delete path
// (remove in place, merges under the parent and the grandparent, rebuild).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include "common.h"
#include "kernels.h"

namespace gt {

struct InsertCtx {
    uint8_t* scratch;
    uint64_t scratch_bytes;
    uint64_t max_batch;
    uint64_t inner_cap, leaf_cap;
    LaunchCfg cfg;
};

// Arena scratch bytes the insert path needs for batches up to max_batch on
// node pools of the given capacities.
uint64_t insert_scratch_bytes(uint64_t max_batch, int key_bytes, uint64_t leaf_cap, uint64_t inner_cap);

// Testing switches of the one-key insert kernel and the one-launch insert
// and delete of small batches; each returns the previous setting.
int set_single_key_insert(int on);
int set_one_launch_insert(int on);
int set_one_launch_delete(int on);

template <class K>
void launch_insert(const TreeView<K>& t, const InsertCtx& c, const K* keys, const K* vals, uint64_t B,
                   uint8_t* status, hipStream_t s);

// Delete batch on the same scratch; returns the device word that is nonzero
// when the tree must be rebuilt from its keys (read after the stream ends).
// host_word (optional) is the device address of a pinned host word: the
// batch's last kernel then also stores (seq << 32 | flag) there itself, and
// *flag_on_host says so (the caller needs no copy and may wait for that word
// instead of the stream).
template <class K>
const uint32_t* launch_delete(const TreeView<K>& t, const InsertCtx& c, const K* keys, uint64_t B, uint8_t* status,
                              uint64_t* host_word, uint32_t seq, bool* flag_on_host, hipStream_t s);

// Every pair of the leaves that hold keys, appended at *n (device counter);
// past `cap` pairs nothing is written, the counter still counts.
template <class K>
void launch_delete_collect(const TreeView<K>& t, uint32_t leaves, K* ok, K* ov, uint64_t cap,
                           unsigned long long* n, hipStream_t s);

}  // namespace gt
