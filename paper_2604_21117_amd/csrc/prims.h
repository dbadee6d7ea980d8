// Device-wide primitives used by the build and insert paths: exclusive scans
// and a stable (key, index) sort.  Wave64 block helpers live here too.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gt {

// Inclusive scan over the 64 lanes of a wave (every lane active).  32-bit
// integers use DPP moves, which stay in the vector ALU: within each row of
// 16 lanes, steps adding the value 1, 2, 4 and 8 lanes below (a lane whose
// source lies outside its row adds 0), then row 0's total into row 1 and
// row 2's into row 3 (row broadcast of lane 15), then the total of rows 0-1
// into rows 2 and 3 (row broadcast of lane 31).  Other types shift with
// cross-lane reads, one LDS-path round trip per step, in the same order as
// before for floating point.
template <class T>
__device__ __forceinline__ T wave_incl_scan(T x) {
    if constexpr (sizeof(T) == 4 && static_cast<T>(-1) > static_cast<T>(0)) {
        int v = static_cast<int>(x);
        v += __builtin_amdgcn_update_dpp(0, v, 0x111, 0xf, 0xf, true);   // row_shr:1
        v += __builtin_amdgcn_update_dpp(0, v, 0x112, 0xf, 0xf, true);   // row_shr:2
        v += __builtin_amdgcn_update_dpp(0, v, 0x114, 0xf, 0xf, true);   // row_shr:4
        v += __builtin_amdgcn_update_dpp(0, v, 0x118, 0xf, 0xf, true);   // row_shr:8
        v += __builtin_amdgcn_update_dpp(0, v, 0x142, 0xa, 0xf, false);  // row_bcast:15, rows 1 and 3
        v += __builtin_amdgcn_update_dpp(0, v, 0x143, 0xc, 0xf, false);  // row_bcast:31, rows 2 and 3
        return static_cast<T>(v);
    } else {
        const int lane = threadIdx.x & 63;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            T y = __shfl_up(x, d, 64);
            if (lane >= d) x += y;
        }
        return x;
    }
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

// Bitonic sort of (key, index) pairs held in LDS, n2 a power of two, by the
// whole workgroup; pairs compare by key then index, so equal keys keep their
// index order.
template <class K>
__device__ __forceinline__ void bitonic_lds(K* sk, uint32_t* si, uint32_t n2) {
    const uint32_t half = n2 >> 1;
    for (uint32_t k = 2; k <= n2; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            // pair q compares slots t and t + j, where t has bit j clear
            for (uint32_t q = threadIdx.x; q < half; q += blockDim.x) {
                const uint32_t t = ((q & ~(j - 1)) << 1) | (q & (j - 1));
                const uint32_t p = t | j;
                const K a = sk[t], b = sk[p];
                const uint32_t ia = si[t], ib = si[p];
                const bool gt = (a > b) || (a == b && ia > ib);
                const bool up = (t & k) == 0;
                if (gt == up) {
                    sk[t] = b; sk[p] = a;
                    si[t] = ib; si[p] = ia;
                }
            }
            __syncthreads();
        }
    }
}

// ------------------------------------------------------------ host side

// Largest batch rank_sort_small takes (all keys sit in each workgroup's LDS).
constexpr uint32_t kRankSortMax = 2048;

// Stable sort of B <= kRankSortMax keys by rank: sk[r] = keys[i] and
// si[r] = i, where r is the number of pairs (keys[j], j) before (keys[i], i)
// in (key, index) order.  If `zero` is given, its first `zero_words` words
// are cleared by the first workgroup (a free ride for the caller's counters).
template <class K>
void rank_sort_small(const K* keys, uint32_t B, K* sk, uint32_t* si, uint32_t* zero, uint32_t zero_words,
                     hipStream_t s);

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
// are ping-pong buffers of n entries.  The result ends in keys/idx.  If a
// tile's look-back wait gives up (never expected: it waits only on running
// tiles), err_bit is or-ed into *err (a device word; by default one in tmp)
// and the order is not valid.
template <class K>
void sort_pairs(K* keys, uint32_t* idx, K* keys_alt, uint32_t* idx_alt, uint64_t n, void* tmp,
                hipStream_t s, uint32_t* err = nullptr, uint32_t err_bit = 1u);

// The same sort of (src[i], i): src is read, keys/idx receive the result,
// keys_alt/idx_alt are ping-pong buffers.  Saves staging the pairs.
template <class K>
void sort_from(const K* src, K* keys, uint32_t* idx, K* keys_alt, uint32_t* idx_alt, uint64_t n, void* tmp,
               hipStream_t s, uint32_t* err = nullptr, uint32_t err_bit = 1u);

// Empty look-back steps after which a sort gives up (process-wide; 0 makes
// every tile after the first give up at once).  Returns the previous value.
uint32_t set_sort_spin_limit(uint32_t limit);

}  // namespace gt
