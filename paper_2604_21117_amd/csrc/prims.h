// Device-wide primitives used by the build and insert paths: exclusive scans
// and a stable (key, index) sort.  Wave64 block helpers live here too.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gt {

template <class T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive scan across the block (blockDim.x a multiple of 64, <= 2048).
// `sh` needs 33 entries of shared memory.  All threads must call it.
template <class T>
__device__ __forceinline__ T block_excl_scan(T v, T* sh, T* total) {
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = blockDim.x >> 6;
    T inc = wave_incl_scan(v);
    if (lane == 63) sh[w] = inc;
    __syncthreads();
    if (w == 0) {
        T s = lane < nw ? sh[lane] : T(0);
        T si = wave_incl_scan(s);
        if (lane < nw) sh[lane] = si - s;
        if (lane == nw - 1) sh[32] = si;
    }
    __syncthreads();
    T res = inc - v + sh[w];
    *total = sh[32];
    __syncthreads();
    return res;
}

// ------------------------------------------------------------ host side

// Scratch bytes needed by scan_exclusive for up to n elements.
uint64_t scan_tmp_bytes(uint64_t n);

// out[i] = sum of in[0..i) for i < n, where n = *n_dev if n_dev is given
// (n_max is then an upper bound used to size the grid), else n_max.  If
// `total` is non-null it receives the sum of all n inputs.  in == out is
// allowed.
template <class T>
void scan_exclusive(const T* in, T* out, T* total, const uint32_t* n_dev, uint64_t n_max,
                    void* tmp, hipStream_t s);

// Scratch bytes needed by sort_pairs for n elements.
uint64_t sort_tmp_bytes(uint64_t n, int key_bytes);

// Stable sort of (keys[i], idx[i]) by key, n host-known.  keys_alt/idx_alt
// are ping-pong buffers of n entries.  The result ends in keys/idx.
template <class K>
void sort_pairs(K* keys, uint32_t* idx, K* keys_alt, uint32_t* idx_alt, uint64_t n, void* tmp,
                hipStream_t s);

}  // namespace gt
