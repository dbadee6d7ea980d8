/*
 * gtree.h -- C ABI of the MI355X batched B+-tree library (libgtree.so).
 *
 * The library keeps a B+-tree (paper Section III: order m, data only in the
 * leaves, leaves linked left to right) resident in device memory and runs
 * batches of operations on it with hand-written gfx950 kernels:
 *
 *   tree_build         bulk load from (key, value) pairs      (Section V-B: the
 *                      one-time build and transfer of the tree)
 *   tree_lookup_batch  root-to-leaf search of a key batch     (Section IV-A,
 *                      IV-E, IV-F: batch search, routing by key-vs-entry compare,
 *                      -1 for a key that is not found)
 *   tree_lookup_levelwise  the same results by the paper's level-by-level
 *                      walk of a sorted batch (Sections IV-A, IV-F)
 *   tree_insert_batch  sort / merge / split insert of a batch with parent
 *                      split propagation (keeps the Section III invariants)
 *   tree_range_batch   range scans over the linked leaves (Section III)
 *
 * Conventions shared by every call:
 *  - Pointers are DEVICE pointers unless the comment says "host".
 *  - Keys and values have the same width, key_bytes = 4 or 8; keys compare
 *    as unsigned integers (the static tree of 32-byte keys or order 32/64
 *    described at gt_params has 8-byte values).  A NOT-FOUND value is all ones at that width (the
 *    paper's -1) and the matching found flag is 0; the flag is authoritative
 *    because all ones is also a legal value.
 *  - Every call is asynchronous on `stream`.  Errors that the host can see
 *    (null pointers, bad sizes, a batch above the tree's max_batch, an arena
 *    that is too small) are returned synchronously and nothing is enqueued.
 *    Errors found on the device set bits of the tree's device error word;
 *    tree_device_error() synchronises the stream and reports them.
 *  - Results are written in caller order.  B = 0 is a no-op returning GT_OK.
 *  - Calls that modify a tree must be ordered on one stream by the caller;
 *    reads may run on several streams only while no write is in flight.
 *
 * Ownership: the caller owns every input and output buffer and the arena.
 * The library places all tree state (header, node pools, a copy of the top
 * tree levels, per-batch scratch) inside the arena and allocates no device
 * memory on the lookup, range or insert paths.  tree_build alone allocates
 * temporary sort buffers, released before it returns.  The arena must stay
 * allocated until tree_destroy.
 */
#ifndef GTREE_H
#define GTREE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gt_tree gt_tree; /* opaque handle, host memory */

typedef enum {
    GT_OK = 0,
    GT_ERR_INVALID = 1,   /* bad argument                                     */
    GT_ERR_DUPLICATE = 2, /* tree_build input holds a key twice               */
    GT_ERR_CAPACITY = 3,  /* arena or node pool too small for the request     */
    GT_ERR_ADMISSION = 4, /* serving runtime refused a request                */
    GT_ERR_HIP = 5,       /* a HIP runtime call failed                        */
    GT_ERR_DEVICE = 6     /* device error word set (other than capacity)      */
} gt_status;

/*
 * Tree parameters (host struct).  Zero fields take the default.
 *
 * Two kinds of tree share this ABI:
 *  - the dynamic tree: key_bytes 4 or 8, fanout 16, 16 keys per leaf;
 *    every call below applies;
 *  - the paper's key and node variants (Sections IV-B, IV-C, V-C), a
 *    static tree built once and searched: key_bytes 32 with fanout 16, 32
 *    or 64, or key_bytes 8 with fanout 32 or 64.  A node of order m has at
 *    most m children and, below the root, at least m/2; a leaf holds at
 *    most m - 1 keys (the paper's k_max) and, when there are two or more
 *    leaves, at least m/2.  32-byte keys are byte strings compared byte by
 *    byte, byte 0 most significant, each byte unsigned (the order of the
 *    paper's bytewise comparators with the cascading priority rule,
 *    Section IV-E); 8-byte keys are unsigned integers.  Values are 8 bytes
 *    (the paper's data).  Buffers of 32-byte keys (keys, lo, hi, out_keys)
 *    and the arena must be 16-byte aligned, else GT_ERR_INVALID.
 *    tree_build, tree_lookup_batch, tree_range_batch,
 *    tree_stats, tree_export, tree_device_error and tree_destroy apply, with
 *    key arrays of key_bytes per key and value arrays of 8 bytes per value;
 *    tree_insert_batch, tree_delete_batch, the level-wise lookups, li_* and
 *    srv_create return GT_ERR_INVALID (tree_lookup_levelwise_workspace_bytes
 *    and li_arena_bytes return 0).  Only key_bytes, fanout, leaf_cap (0 or
 *    fanout - 1) and fill may be set; tree_arena_bytes ignores leaf_slack.
 */
typedef struct {
    uint32_t key_bytes;       /* 4, 8 or 32 (no default)                      */
    uint32_t fanout;          /* inner order m: 16 (default), or 32 / 64 for
                                 the static tree (above)                      */
    uint32_t leaf_cap;        /* keys per leaf: 16 for the dynamic tree,
                                 fanout - 1 for the static one; 0 = that     */
    float fill;               /* bulk-load fill in [0.5, 1]; default 1.0      */
    uint32_t lanes_per_query; /* lookup lanes per query: 4, 8 or 16; 0 = by
                                 batch size (16 below 2^13 queries, else 8);
                                 ranges and insert location use 8            */
    uint32_t lds_levels;      /* top inner levels read from an LDS copy: 1..3,
                                 4 = none; 0 = by batch size (none below 2^15
                                 queries, else 2; ranges and insert location
                                 use 2)                                       */
    uint32_t sorted_mode;     /* reserved, must be 0                          */
    uint32_t queries_per_group; /* queries a lane group walks at once: 1, 2
                                   or 4 for every batch; 0 = by batch size
                                   (1 below 2^15 queries, else 2)             */
    uint64_t max_batch;       /* largest insert batch; default 2^20           */
    uint32_t value_coload;    /* 1: a lookup reads the leaf's value line with
                                 its key line (one dependent load fewer);
                                 2: it reads the one value after the match;
                                 0 = default (1)                              */
    uint32_t xcd_split;       /* 1: large lookup batches are split by key
                                 range over the 8 XCDs so that each XCD's L2
                                 holds the inner nodes of its own subtrees;
                                 2: off; 0 = default (off)                  */
    uint32_t leaf_stream;     /* non-temporal loads of leaf lines in lookups
                                 (lines that stream should not evict the
                                 inner nodes other queries reuse from L2):
                                 1: key and value lines, every batch; 2:
                                 none; 0 = default: the value line from
                                 2^15 queries on                            */
    uint32_t reserved;        /* must be 0                                    */
} gt_params;

typedef struct {
    uint64_t n_keys;
    uint32_t height;          /* levels including the leaf level              */
    uint32_t root;            /* node reference of the root                   */
    uint64_t inner_used, inner_cap;
    uint64_t leaf_used, leaf_cap;
    uint64_t arena_bytes;     /* bytes of the arena the tree uses             */
    uint64_t max_batch;
    uint32_t error_word;      /* device error bits (see GT_DEVERR_*)          */
    uint32_t key_bytes;
} gt_tree_stats;

/* device error word bits */
#define GT_DEVERR_CAPACITY 0x1u  /* an insert batch did not fit; it was not applied */
#define GT_DEVERR_INTERNAL 0x2u  /* an internal consistency check failed          */

/* Bytes of arena needed for n keys plus `leaf_slack` extra leaves of
 * headroom for inserts, with the given params (host).  Returns 0 for bad
 * params. */
uint64_t tree_arena_bytes(const gt_params* p /*host*/, uint64_t n, uint64_t leaf_slack);

/*
 * Bulk load (Section V-B's one-time build, done on the device).
 * keys[n], values[n]: any order; duplicate keys give GT_ERR_DUPLICATE.
 * Leaves are filled evenly to `fill` (at least half full when there are two
 * or more), inner levels are built bottom-up with the same rule, and the
 * leaves are chained in key order.  n = 0 builds an empty tree.
 * This call synchronises `stream` before it returns.  On success *out
 * receives a new handle; GT_ERR_DEVICE if the device sort of the keys
 * failed (a bounded wait between its workgroups gave up: not expected).
 */
gt_status tree_build(const gt_params* p /*host*/, const void* keys, const void* values, uint64_t n,
                     void* arena, uint64_t arena_bytes, hipStream_t stream, gt_tree** out /*host*/);

/*
 * Lookup batch (Sections IV-A to IV-F).  For each i < B: if keys[i] is in
 * the tree, values_out[i] = its value and found_out[i] = 1; otherwise
 * values_out[i] = all ones and found_out[i] = 0.  keys: B entries of
 * key_bytes; values_out: B entries of key_bytes; found_out: B bytes.
 */
gt_status tree_lookup_batch(gt_tree* t, const void* keys, uint64_t B, void* values_out,
                            uint8_t* found_out, hipStream_t stream);

/*
 * Level-wise lookup batch: the paper's own traversal (Sections IV-A and
 * IV-F).  The batch is sorted, then walks the tree one level at a time: a
 * FIFO of (node, first query, count) entries, each node read once and
 * compared with the whole run of sorted queries that passes through it,
 * the run cut into the next level's entries where the child changes.  The
 * results are those of tree_lookup_batch, in caller order.
 *
 * flags: 0, or GT_LW_PRESORTED when the caller's keys are already in
 * ascending order: no sort is made and the runs come straight from the
 * caller's order.  Keys that are not in order still get correct results
 * (the runs are only shorter).
 *
 * workspace: device memory of at least
 * tree_lookup_levelwise_workspace_bytes(t, B, flags) bytes, owned by the
 * caller; its contents on entry are ignored.  A call uses it until the call
 * completes on `stream`, so calls that may overlap need separate
 * workspaces.  B < 2^31.  Errors: GT_ERR_INVALID for null pointers, unknown
 * flags or B too large; GT_ERR_CAPACITY when workspace_bytes is too small.
 * Nothing is enqueued on an error.  No memory is allocated; the call is
 * graph-capturable.  Should the device sort of a batch above 2048 keys fail
 * (a bounded wait between its workgroups gives up: not expected) the tree's
 * device error word gets the internal bit (tree_device_error: GT_ERR_DEVICE)
 * and the results are not valid.
 */
#define GT_LW_PRESORTED 1u
uint64_t tree_lookup_levelwise_workspace_bytes(const gt_tree* t, uint64_t B, uint32_t flags);
gt_status tree_lookup_levelwise(gt_tree* t, const void* keys, uint64_t B, uint32_t flags, void* values_out,
                                uint8_t* found_out, void* workspace, uint64_t workspace_bytes,
                                hipStream_t stream);

/*
 * Level-wise lookup that allocates nothing, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc).  Same arguments, results and
 * errors as tree_lookup_levelwise, without the workspace: the library keeps
 * a fixed scratch array of GT_LW_NOALLOC_SCRATCH_BYTES in device memory,
 * one per GPU it runs on, held until the process ends, and uses it as the
 * workspace.  A batch is accepted when
 * tree_lookup_levelwise_workspace_bytes(t, B, flags) fits that size (8-byte
 * keys: any B <= 2^18 with the library sort, B <= 2^20 presorted; 4-byte
 * keys: B <= 2^19 and B <= 2^20); a larger one returns GT_ERR_CAPACITY with
 * nothing enqueued.  The call makes no hipMalloc, hipFree or other
 * allocating call; the first call on a device resolves that device's array
 * (the tree's device must be current, as for every call).  Every call on a
 * GPU shares its one array, whatever the tree or stream: calls that may
 * overlap on one GPU race and must be ordered by the caller (one stream, or
 * events).  The array keeps the last call's contents; a call needs none of
 * them (it clears what it uses with kernels, no memset), so it is
 * graph-capturable like tree_lookup_levelwise.
 */
#define GT_LW_NOALLOC_SCRATCH_BYTES (16ull << 20)
gt_status tree_lookup_levelwise_noalloc(gt_tree* t, const void* keys, uint64_t B, uint32_t flags,
                                        void* values_out, uint8_t* found_out, hipStream_t stream);

/*
 * Insert batch.  Equivalent to inserting (keys[i], values[i]) one at a time
 * for i = 0..B-1: a present key gets its value overwritten.  status_out[i]
 * = 0 (INSERTED) when keys[i] was absent before the batch and not earlier in
 * the batch, else 1 (UPDATED).  Leaves that overflow split evenly into
 * ceil(t/16) leaves, inner nodes that overflow split the same way, and the
 * root grows when it splits; every node but the root stays at least half
 * full (Section III).  B <= max_batch.  The batch is applied whole or not
 * at all: if the node pools cannot hold it, the device error word gets
 * GT_DEVERR_CAPACITY, the tree is left unchanged and status_out is
 * unspecified.  A batch is not applied either while the word holds
 * GT_DEVERR_INTERNAL (set, for one, when the device sort of a batch above
 * 2048 keys gives up a bounded wait between its workgroups: not expected);
 * tree_device_error clears the word.
 */
gt_status tree_insert_batch(gt_tree* t, const void* keys, const void* values, uint64_t B,
                            uint8_t* status_out, hipStream_t stream);

/*
 * Delete batch.  Equivalent to deleting keys[i] one at a time for
 * i = 0..B-1: status_out[i] = 1 (DELETED) when keys[i] was present before
 * the batch and not earlier in the batch, else 0 (ABSENT).  Every node but
 * the root stays at least half full (Section III): a leaf left with fewer
 * than 8 keys is merged with its siblings (the parent's keys are spread
 * evenly over as few of its leaves as hold them at least half full, at
 * least 8 of them), a parent that would itself fall below half full is
 * merged with its siblings (the grandparent's keys, at most 4096, laid out
 * again over as few of its parents and leaves as keep both at least half
 * full), the root loses levels when few keys remain (one parent, then one
 * leaf), and when a grandparent would fall below half full the tree is
 * rebuilt in place from its keys (as tree_build, bulk load, height
 * recomputed).  Leaves and inner nodes a merge gives up are not reused by
 * later inserts (the pools only grow until the next tree_build).  Like an
 * insert, a batch is not applied while the device error word holds
 * GT_DEVERR_INTERNAL.  keys: B keys; status_out: B bytes; B <= max_batch.
 * Waits once on the host, to learn whether a rebuild is needed: for the
 * flag the batch's last kernel stores into pinned host memory (that kernel
 * may still be finishing its last writes when the call returns; later work
 * on `stream` is ordered after it).
 * The rebuild allocates and frees temporary device memory.  A learned index
 * over the tree answers through the tree after a delete until li_train.
 */
gt_status tree_delete_batch(gt_tree* t, const void* keys, uint64_t B, uint8_t* status_out, hipStream_t stream);

/*
 * Range batch over the linked leaves (Section III).  For each i < B, the
 * pairs with lo[i] <= key <= hi[i], ascending, cut to the first max_out[i],
 * are written to out_keys/out_values starting at out_offsets[i];
 * count_out[i] receives how many.  The caller sizes the outputs so that
 * out_offsets[i] + max_out[i] entries fit.  lo > hi yields no pairs.
 * lo, hi: B keys; max_out: B u32; out_offsets: B u64.
 */
gt_status tree_range_batch(gt_tree* t, const void* lo, const void* hi, const uint32_t* max_out,
                           const uint64_t* out_offsets, uint64_t B, void* out_keys,
                           void* out_values, uint32_t* count_out, hipStream_t stream);

/* Release the handle (host memory only; the arena stays the caller's). */
gt_status tree_destroy(gt_tree* t);

/* Synchronise `stream` and fill *out (host) from the device header. */
gt_status tree_stats(gt_tree* t, gt_tree_stats* out /*host*/, hipStream_t stream);

/*
 * Synchronise `stream`, read and clear the device error word.  Returns
 * GT_OK, GT_ERR_CAPACITY (an insert batch was refused) or GT_ERR_DEVICE.
 */
gt_status tree_device_error(gt_tree* t, hipStream_t stream);

/*
 * Copy the tree into host memory in the flat export format (synchronises):
 *   header, 48 bytes little endian:
 *     u32 magic 0x58455447, key_bytes, fanout, leaf_cap, height, root,
 *     first_leaf, n_inner, n_leaves, value_bytes;  u64 n_keys
 *     (value_bytes is 0 for the dynamic tree, meaning key_bytes; the static
 *     tree writes 8)
 *   n_inner inner records:  key[fanout] (key_bytes each), child[fanout] (u32)
 *   n_leaves leaf records:  key[leaf_cap] (key_bytes each),
 *                           value[leaf_cap] (value_bytes each),
 *                           u32 count, u32 next
 * A node reference with bit 31 set is a leaf (index in the low bits),
 * otherwise an inner node index; 0xFFFFFFFF is "none".  Inner entry i < c-1
 * is the largest key below child i; entries from c-1 on hold the largest
 * key and child slots from c on hold "none".  Leaf key slots from count on
 * repeat the last key (the largest key in an empty leaf).
 * With host_buf = NULL, *bytes (host) receives the size needed.
 */
gt_status tree_export(gt_tree* t, void* host_buf, uint64_t* bytes /*host*/, hipStream_t stream);

/* A constant, human-readable name for a status code (host). */
const char* gt_status_str(gt_status s);

/* The testing hook of the device sort's failure path is declared in
 * gtree_testing.h (same library). */

/* ------------------------------------------------------------------------
 * Learned index over a tree (an addition to the paper's tree search).
 *
 * A two-stage model maps a key to its leaf's position in key order.  The
 * root is linear (evaluated in FP64); its output picks one of `models`
 * leaf models and its fractional part is that model's input.  Each leaf
 * model is FP32: a line, or a one-hidden-layer ReLU network with 32 units
 * whose knots sit on a uniform grid, which makes it linear on 32 pieces;
 * it is stored as 32 (slope, intercept) pieces, chosen per model by the
 * smaller error window.  The models are trained on the device from the
 * tree's own (key, leaf position) pairs, and every piece gets exact error
 * bounds lo <= pos - pred <= hi over all keys routed to it, computed by the
 * same evaluation the lookup runs.  A lookup predicts, reads the leaves of
 * [pred + lo, pred + hi] (directly on a bulk-loaded tree, else through the
 * directory of leaf fence keys) and answers when a leaf holds the key; while
 * the tree is unchanged since training a window without the key proves it
 * absent, and otherwise (inserts since training, overwritten bounds, a piece
 * without bounds) such a query goes down the tree.  Results are always
 * exactly those of tree_lookup_batch; the models only change the speed.
 * ---------------------------------------------------------------------- */
typedef struct gt_learned gt_learned; /* opaque handle, host memory */

typedef struct {
    uint32_t models;      /* leaf models, 1..4096; 0 = default 1024          */
    uint32_t kind;        /* 0 = per model, the kind with the smaller window;
                             1 = linear only; 2 = network only                */
    uint32_t max_window;  /* a piece whose window spans more leaves sends its
                             keys down the tree; 0 = default 64               */
    uint32_t search;      /* window search: 1 = through the fence directory;
                             2 = read the window's leaves directly when the
                             trained directory is the identity (a bulk-loaded
                             tree); 0 = default: direct for batches up to
                             2^13 keys on such a tree when no window spans
                             more than 16 leaves, else the directory          */
    uint32_t gate;        /* 0 = default: after training, if more than a
                             quarter of the keys go down the tree or the
                             key-weighted mean window exceeds 16 leaves, the
                             models cannot beat the tree's descent and
                             li_lookup_batch runs tree_lookup_batch instead
                             (same results; li_stats reports `declined`);
                             1 = always take the model path                  */
    uint32_t reserved[2]; /* must be 0                                        */
} gt_li_params;

typedef struct {
    uint64_t trained_leaves;  /* leaves in the directory at training         */
    uint64_t trained_keys;
    uint64_t lookups;         /* queries answered since training             */
    uint64_t fallbacks;       /* of which went down the tree                 */
    uint32_t models, linear_models, mlp_models, tree_models;
                              /* tree_models: every key goes down the tree   */
    uint32_t max_window;      /* widest window (leaves) of a piece in use    */
    uint32_t declined;        /* 1: the quality gate sends lookups to the
                                 tree (see gt_li_params.gate)                */
    double mean_window;       /* window per trained key, averaged over keys  */
} gt_li_stats;

/* Arena bytes a learned index over tree t needs (host). */
uint64_t li_arena_bytes(const gt_tree* t, const gt_li_params* p /*host*/);

/* Create an (untrained) learned index over t in `arena` (device memory the
 * caller owns and keeps until li_destroy).  Lookups before li_train go
 * down the tree. */
gt_status li_create(gt_tree* t, const gt_li_params* p /*host*/, void* arena, uint64_t arena_bytes,
                    gt_learned** out /*host*/);

/* (Re)train from the tree's current leaves: leaf positions in key order
 * (the tree expanded level by level from the root), the fence directory,
 * root and leaf model fits, exact bounds over every key.  Synchronises
 * `stream`. */
gt_status li_train(gt_learned* li, hipStream_t stream);

/* Same contract as tree_lookup_batch.  The launch passes the index's current
 * parameters by value: a graph that captured it must be captured again after
 * li_train or li_set_bounds, and after the first tree_insert_batch on its
 * tree since training (from then on a miss resumes along the leaf chain,
 * which another kernel does; a graph captured before still answers
 * correctly, through the tree). */
gt_status li_lookup_batch(gt_learned* li, const void* keys, uint64_t B, void* values_out,
                          uint8_t* found_out, hipStream_t stream);

/* Inference as the lookup runs it, for checking bounds: per key the piece
 * (model * 32 + piece, the unit that owns bounds), the predicted leaf
 * position and that piece's bounds (lo, hi), and the kind in use (0 line,
 * 1 network; 2, with pred, lo and hi 0, when the piece sends keys down the
 * tree).  Outputs: B entries each (u32, i32, i32, i32, u8). */
gt_status li_predict(gt_learned* li, const void* keys, uint64_t B, uint32_t* model_out, int32_t* pred_out,
                     int32_t* lo_out, int32_t* hi_out, uint8_t* model_kind_out, hipStream_t stream);

/* Test hook: overwrite every piece's bounds with [lo, hi] (a wrong window
 * must only cost fallbacks, never a wrong result). */
gt_status li_set_bounds(gt_learned* li, int32_t lo, int32_t hi, hipStream_t stream);

/* Counters and model summary (synchronises). */
gt_status li_stats(gt_learned* li, gt_li_stats* out /*host*/, hipStream_t stream);

/* Release the handle (host memory only; the caller frees the arena after
 * work that uses it has completed). */
gt_status li_destroy(gt_learned* li);

/* ------------------------------------------------------------------------
 * Serving runtime (an addition to the paper's batch search; its closest
 * analogue is the host/device overlap of Section V-B).
 *
 * Lookup, insert and range batches of uneven sizes arrive from host
 * threads and are admitted in arrival order when a slot is free and the
 * bytes in flight stay under the memory cap (a batch that can never fit is
 * refused).  Admission order is the linearization order: a batch sees every
 * insert admitted before it and none after.  Reads run concurrently on
 * several HIP streams; an insert waits for the reads admitted before it and
 * the reads after it wait for the insert.  Each batch is padded to a power
 * of two with entries that leave the result unchanged (repeats of the last
 * lookup key, insert pair or delete key; empty ranges) and, once its
 * (slot, op, size) shape has been seen, replayed from a captured hipGraph
 * (input copy, kernels, output copy).  Inputs and outputs live in the
 * caller's host memory; the runtime stages them through pinned buffers.
 * ---------------------------------------------------------------------- */
typedef struct gt_server gt_server;

typedef struct {
    uint32_t read_streams;   /* streams for reads; 0 = default 4            */
    uint32_t slots;          /* batches in flight at once; 0 = default 16   */
    uint64_t mem_cap;        /* cap on staged bytes in flight; 0 = 32 GiB   */
    uint32_t max_batch;      /* largest batch; 0 = default 1024             */
    uint32_t max_range;      /* largest per-query range length; 0 = 128     */
    uint32_t use_graphs;     /* 1 = replay captured graphs, 2 = direct
                                launches; 0 = default (1)                   */
    uint32_t retrain_log2;   /* with a learned index: after 2^retrain_log2
                                inserted (or deleted) keys the server copies
                                the tree's arena between the writes admitted
                                before and after that point, trains a second
                                index on the copy on a thread and stream of
                                its own while admission goes on, and then
                                exchanges the two indexes' states (batches
                                admitted from then on use the new one; a
                                write after the copy counts as a change since
                                its training, as for any stale index);
                                0 = never; at most 40.  The copy and the
                                second index are allocated by srv_create     */
} gt_srv_params;

enum { GT_OP_LOOKUP = 0, GT_OP_INSERT = 1, GT_OP_RANGE = 2, GT_OP_DELETE = 3 };
enum { GT_REQ_QUEUED = 0, GT_REQ_INFLIGHT = 1, GT_REQ_DONE = 2, GT_REQ_REFUSED = 3 };

/* One batch; every pointer is HOST memory owned by the caller until the
 * request is done.  lookup: keys -> out0 (values), out1 (found, u8);
 * insert: keys, values -> out0 (status, u8); range: keys (lo), values (hi),
 * max_out -> out0 (keys), out1 (values) in CSR order of max_out, count_out;
 * delete: keys -> out0 (status, u8).  Inserts and deletes are writes: each
 * sees every batch admitted before it.  A delete batch runs outside the
 * captured graphs (tree_delete_batch waits on the host). */
typedef struct {
    uint32_t op;
    uint32_t B;
    const void* keys;
    const void* values;
    const uint32_t* max_out;
    void* out0;
    void* out1;
    uint32_t* count_out;
    double arrival_s;        /* srv_replay: arrival time after the start    */
} gt_request;

typedef struct {
    uint64_t done[4];        /* batches completed per op (GT_OP_*)          */
    uint64_t ops[4];         /* keys (lookup, insert, delete) / ranges done */
    uint64_t refused;
    uint64_t graph_launches, direct_launches;
    double wall_s;           /* first arrival to last completion            */
    double p50_us, p99_us;   /* arrival -> completion latency, all batches  */
    double p50_us_op[4], p99_us_op[4];  /* per op, indexed by GT_OP_*   */
    double busy_frac;        /* share of wall_s in which the device worked on
                                at least one batch (copies included), from
                                timing events around each batch              */
    uint64_t retrains;       /* learned-index retrainings since creation     */
    double retrain_s;        /* their total time (copy to exchange)          */
    uint64_t captures;       /* graphs the worker captured since creation    */
    double capture_s;        /* worker time spent capturing them             */
    uint64_t precaptured;    /* lookup graphs captured by the trainer for a
                                retrained index and installed at the
                                exchange                                     */
} gt_srv_stats;

/* Create a server over tree t (and learned index li for lookups, or NULL).
 * Allocates its staging buffers (pinned host, device) here, not later; with
 * retrain_log2 also a copy of t's arena and a second index like li.
 * li_train / li_set_bounds on li are allowed while no request is in flight
 * and no retraining runs (srv_replay returns after the retrainings its
 * batches started); the server then captures its lookup graphs again.  At
 * srv_destroy li holds the most recent training, in its own arena. */
gt_status srv_create(gt_tree* t, gt_learned* li, const gt_srv_params* p /*host*/, gt_server** out);
/* Queue a batch (non-blocking); *ticket identifies it. */
gt_status srv_submit(gt_server* s, const gt_request* r /*host*/, uint64_t* ticket /*host*/);
/* State of a ticket (GT_REQ_*). */
gt_status srv_poll(gt_server* s, uint64_t ticket, uint32_t* state /*host*/);
/* Block until the ticket is done or refused. */
gt_status srv_wait(gt_server* s, uint64_t ticket);
/* Submit reqs[i] at reqs[i].arrival_s after the call starts (open loop),
 * then wait for all of them; statistics cover exactly these requests. */
gt_status srv_replay(gt_server* s, const gt_request* reqs /*host*/, uint64_t n);
/* Statistics of the last srv_replay's requests (host). */
gt_status srv_stats(gt_server* s, gt_srv_stats* out /*host*/);
/* Arrival-to-completion latency in microseconds of the last srv_replay's
 * requests, in their order (host array of n). */
gt_status srv_latencies(gt_server* s, double* out /*host*/, uint64_t n);
/* Drain every admitted request, stop the worker and free the staging
 * buffers, streams and captured graphs. */
gt_status srv_destroy(gt_server* s);

#ifdef __cplusplus
}
#endif
#endif /* GTREE_H */
