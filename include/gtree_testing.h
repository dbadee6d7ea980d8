/*
 * gtree_testing.h -- testing hooks of libgtree.so.
 *
 * Not needed to use the library: these calls let tests drive failure paths
 * that cannot be provoked from the inputs.  Declarations of gtree.h apply.
 */
#ifndef GTREE_TESTING_H
#define GTREE_TESTING_H

#include <stdint.h>
#include "gtree.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Testing hook for the failure path of the device radix sort (inputs above
 * 2048 keys: tree_build, tree_insert_batch, tree_delete_batch,
 * tree_lookup_levelwise).  A
 * workgroup of a sort pass waits on the published counts of earlier ones;
 * `limit` is how many look-back steps that find nothing new it takes
 * before it gives up (default 1 << 20, never reached in practice).  0 makes
 * every workgroup but the first of a pass give up at once, so any sort of
 * more than 4096 keys fails.  A failed sort reports GT_ERR_DEVICE from
 * tree_build; in an insert, delete or level-wise lookup it sets
 * GT_DEVERR_INTERNAL in the tree's error word, an insert or delete batch is
 * refused with the tree unchanged, and the lookup's outputs are
 * unspecified.  Process-wide, read
 * when a sort is launched (a captured graph keeps the value in force when
 * it was captured); not meant to be changed while other threads launch
 * work.  Returns the previous value.
 */
uint32_t gt_set_sort_spin_limit(uint32_t limit);

/*
 * Testing switch of the one-key insert: a batch of B = 1 runs in one kernel
 * (descent, leaf and parent rewrites, header, mirror) instead of the batch
 * path's kernels, with the same resulting tree.  enable = 0 sends B = 1
 * through the batch path, so that tests can compare the two; any other
 * value restores the default (on).  Process-wide, read when an insert is
 * launched (a captured graph keeps the path it was captured with).
 * Returns the previous setting (1 on, 0 off).
 */
int gt_set_single_key_insert(int enable);

/*
 * Testing switch of the one-launch insert: a batch of 2 to 64 keys runs in
 * one launch (the small-batch path's phases in one workgroup: ranking and
 * deduplication, locate, plan, leaf and parent rebuilds, root growth, commit
 * and mirror) instead of that path's four kernels, with the same resulting
 * tree and statuses.  enable = 0 sends such batches through the four
 * kernels; any other value restores the default (on).  Process-wide, read
 * when an insert is launched.  Returns the previous setting (1 on, 0 off).
 */
int gt_set_one_launch_insert(int enable);

/*
 * Testing switch of the one-launch delete: a batch of at most 64 keys runs
 * in one launch (the batch path's phases in one workgroup: ranking and
 * deduplication, locate, leaf removal, the parent and grandparent merges,
 * commit and mirror) instead of the batch path's eight, with the same
 * resulting tree.  enable = 0 sends such batches through the batch path;
 * any other value restores the default (on).  Process-wide, read when a
 * delete is launched.  Returns the previous setting (1 on, 0 off).
 */
int gt_set_one_launch_delete(int enable);

#ifdef __cplusplus
}
#endif
#endif /* GTREE_TESTING_H */
