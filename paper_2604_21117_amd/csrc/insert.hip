// Insert path: placeholder until the sort-merge-split kernels land.
#include "insert.h"

namespace gt {

uint64_t insert_scratch_bytes(uint64_t max_batch, int key_bytes) { return 256; }

__global__ void k_insert_unavailable(DevHeader* h) {
    if (threadIdx.x == 0) atomicOr(&h->error, kErrInternal);
}

template <class K>
void launch_insert(const TreeView<K>& t, const InsertCtx&, const K*, const K*, uint64_t, uint8_t*, hipStream_t s) {
    hipLaunchKernelGGL(k_insert_unavailable, dim3(1), dim3(64), 0, s, t.hdr);
}

template void launch_insert<uint32_t>(const TreeView<uint32_t>&, const InsertCtx&, const uint32_t*,
                                      const uint32_t*, uint64_t, uint8_t*, hipStream_t);
template void launch_insert<uint64_t>(const TreeView<uint64_t>&, const InsertCtx&, const uint64_t*,
                                      const uint64_t*, uint64_t, uint8_t*, hipStream_t);

}  // namespace gt
