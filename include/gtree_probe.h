/*
 * gtree_probe.h -- memory-system probes of libgtree.so (diagnostics).
 *
 * Small kernels that measure what bounds the search kernels on the GPU they
 * run on: the cost of a launch, the latency of a dependent load, the rate of
 * random 128-byte line reads, and a lookup-shaped batch whose chain of
 * dependent rounds is chosen by the caller.  They compute nothing of the
 * tree; bench.py --probe times them (HIP events) and reports the figures.
 * Every pointer is a device pointer; every call is asynchronous on
 * `stream`; GT_ERR_INVALID for a null pointer or a zero size, GT_ERR_HIP
 * when the launch fails.
 */
#ifndef GTREE_PROBE_H
#define GTREE_PROBE_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>
#include "gtree.h"

#ifdef __cplusplus
extern "C" {
#endif

/* An empty kernel: one workgroup of 64 threads that returns at once. */
gt_status gt_probe_empty(hipStream_t stream);

/*
 * Where workgroups run: `workgroups` workgroups of 256 threads; workgroup w
 * writes to out[w] the XCC (XCD) it runs on, read from the XCC_ID hardware
 * register (0..7 on MI355X).  Checks the dealing of workgroups to XCDs in
 * turn that XCD-aware launches assume (w and w + 8 on one XCD).
 */
gt_status gt_probe_xcc(uint32_t* out, uint32_t workgroups, hipStream_t stream);

/*
 * Dependent loads: one lane starts at element `start` of `next` and reads
 * x = next[x] `steps` times, then writes x to out[0].  next holds element
 * indices (u64); the caller lays out a cycle whose elements sit in distinct
 * 128-byte lines, so every step is one line that depends on the last.
 */
gt_status gt_probe_chase(const uint64_t* next, uint64_t steps, uint64_t start, uint64_t* out,
                         hipStream_t stream);

/*
 * Random line reads: n reads of 128-byte lines of `region` (lines lines),
 * each by 8 lanes with 16-byte loads, the line index a hash of the read's
 * number and `seed`; `per_group` independent reads in flight per 8-lane
 * group.  `lines` is a power of two.  The xor of everything read goes to out[0] (so no read is dead).
 */
gt_status gt_probe_gather(const uint64_t* region, uint64_t lines, uint64_t n, uint32_t per_group, uint64_t seed,
                          uint64_t* out, hipStream_t stream);

/*
 * A lookup-shaped batch: B queries, 8 lanes each.  A query reads q[i], then
 * makes `table_rounds` dependent 16-byte reads from `table` (table_lines
 * 128-byte lines, meant to stay in L2), then `region_rounds` dependent
 * rounds of `lines_per_round` independent 128-byte line reads from `region`
 * (region_lines lines), each index a hash of the previous round's data and
 * the query, and writes one u64 to out[i].  Rounds of zero are skipped.
 * table_lines and region_lines are powers of two; lines_per_round <= 8
 * (the round's reads are issued together).
 */
gt_status gt_probe_batch(const uint64_t* q, uint64_t B, const uint64_t* table, uint64_t table_lines,
                         uint32_t table_rounds, const uint64_t* region, uint64_t region_lines, uint32_t region_rounds,
                         uint32_t lines_per_round, uint64_t* out, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* GTREE_PROBE_H */
