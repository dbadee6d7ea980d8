// Scans and the stable key sort (hand-written for gfx950, wave64).
//
// scan_exclusive: one workgroup of 1024 threads for up to 16 Ki elements
// (it walks the input in 4096-element rounds with a running carry), else
// reduce-then-scan over 4096-element tiles (tile sums, one-workgroup scan of
// the sums, tile scans plus offsets).
//
// sort_pairs: up to 2048 elements sort inside one workgroup with a bitonic
// network on (key, index) pairs, which orders equal keys by index and so is
// stable.  Larger inputs use LSD radix sort with 8-bit digits: per pass a
// per-tile digit histogram, an exclusive scan of the histograms in
// digit-major order, and a stable scatter in which each wave ranks its
// lanes by digit with eight ballots (lanes whose digit bits all agree are
// peers) and waves are offset by a per-digit prefix in LDS.
#include "prims.h"
#include "common.h"

namespace gt {

constexpr int kScanBlock = 1024;
constexpr int kScanItems = 4;
constexpr uint64_t kScanTile = kScanBlock * kScanItems;  // 4096
constexpr uint64_t kScanSmallMax = 1 << 14;  // one workgroup up to four tiles

static uint32_t ntiles_for(uint64_t n) { return static_cast<uint32_t>((n + kScanTile - 1) / kScanTile); }

uint64_t scan_tmp_bytes(uint64_t n) {
    uint64_t t = ntiles_for(n) + 1;
    return ((t * 8 + 255) / 256) * 256 + 256;
}

template <class T>
__device__ __forceinline__ uint64_t resolve_n(const uint32_t* n_dev, uint64_t n_max) {
    return n_dev ? static_cast<uint64_t>(*n_dev) : n_max;
}

// One workgroup walks the whole input with a carry.
template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_single(const T* in, T* out, T* total,
                                                             const uint32_t* n_dev, uint64_t n_max) {
    __shared__ T sh[33];
    const uint64_t n = resolve_n<T>(n_dev, n_max);
    T carry = 0;
    for (uint64_t base = 0; base < n; base += kScanTile) {
        T v[kScanItems];
        T sum = 0;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            uint64_t i = base + threadIdx.x * kScanItems + j;
            v[j] = i < n ? in[i] : T(0);
            sum += v[j];
        }
        T tot;
        T off = block_excl_scan<T>(sum, sh, &tot) + carry;
#pragma unroll
        for (int j = 0; j < kScanItems; ++j) {
            uint64_t i = base + threadIdx.x * kScanItems + j;
            if (i < n) out[i] = off;
            off += v[j];
        }
        carry += tot;
    }
    if (total && threadIdx.x == 0) *total = carry;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_tile_sums(const T* in, T* sums, const uint32_t* n_dev,
                                                                uint64_t n_max) {
    __shared__ T sh[33];
    const uint64_t n = resolve_n<T>(n_dev, n_max);
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile;
    if (base >= n) {
        if (threadIdx.x == 0) sums[blockIdx.x] = 0;
        return;
    }
    T s = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        uint64_t i = base + threadIdx.x * kScanItems + j;
        if (i < n) s += in[i];
    }
    T tot;
    block_excl_scan<T>(s, sh, &tot);
    if (threadIdx.x == 0) sums[blockIdx.x] = tot;
}

template <class T>
__global__ __launch_bounds__(kScanBlock) void k_scan_tiles(const T* in, T* out, const T* offs,
                                                            const uint32_t* n_dev, uint64_t n_max) {
    __shared__ T sh[33];
    const uint64_t n = resolve_n<T>(n_dev, n_max);
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kScanTile;
    if (base >= n) return;
    T v[kScanItems];
    T sum = 0;
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        uint64_t i = base + threadIdx.x * kScanItems + j;
        v[j] = i < n ? in[i] : T(0);
        sum += v[j];
    }
    T tot;
    T off = block_excl_scan<T>(sum, sh, &tot) + offs[blockIdx.x];
#pragma unroll
    for (int j = 0; j < kScanItems; ++j) {
        uint64_t i = base + threadIdx.x * kScanItems + j;
        if (i < n) out[i] = off;
        off += v[j];
    }
}

template <class T>
void scan_exclusive(const T* in, T* out, T* total, const uint32_t* n_dev, uint64_t n_max, void* tmp,
                    hipStream_t s) {
    if (n_max <= kScanSmallMax) {
        hipLaunchKernelGGL(k_scan_single<T>, dim3(1), dim3(kScanBlock), 0, s, in, out, total, n_dev, n_max);
        return;
    }
    uint32_t nt = ntiles_for(n_max);
    T* sums = reinterpret_cast<T*>(tmp);
    hipLaunchKernelGGL(k_scan_tile_sums<T>, dim3(nt), dim3(kScanBlock), 0, s, in, sums, n_dev, n_max);
    hipLaunchKernelGGL(k_scan_single<T>, dim3(1), dim3(kScanBlock), 0, s, sums, sums, total, nullptr,
                       static_cast<uint64_t>(nt));
    hipLaunchKernelGGL(k_scan_tiles<T>, dim3(nt), dim3(kScanBlock), 0, s, in, out, sums, n_dev, n_max);
}

template void scan_exclusive<uint32_t>(const uint32_t*, uint32_t*, uint32_t*, const uint32_t*, uint64_t,
                                       void*, hipStream_t);
template void scan_exclusive<uint64_t>(const uint64_t*, uint64_t*, uint64_t*, const uint32_t*, uint64_t,
                                       void*, hipStream_t);

// ------------------------------------------------------------------ sort

constexpr int kSortBlock = 1024;
constexpr int kSortRounds = 4;
constexpr uint64_t kSortTile = kSortBlock * kSortRounds;  // 4096
constexpr uint64_t kBitonicMax = 2048;

static uint32_t sort_tiles(uint64_t n) { return static_cast<uint32_t>((n + kSortTile - 1) / kSortTile); }

uint64_t sort_tmp_bytes(uint64_t n, int) {
    uint64_t nt = sort_tiles(n);
    uint64_t hist = nt * 256 * 4;
    return ((hist + 255) / 256) * 256 + scan_tmp_bytes(nt * 256);
}

template <class K>
__global__ __launch_bounds__(kSortBlock) void k_bitonic(K* keys, uint32_t* idx, uint32_t n, uint32_t n2) {
    __shared__ K sk[kBitonicMax];
    __shared__ uint32_t si[kBitonicMax];
    for (uint32_t t = threadIdx.x; t < n2; t += kSortBlock) {
        sk[t] = t < n ? keys[t] : kmax<K>();
        si[t] = t < n ? idx[t] : 0xFFFFFFFFu;
    }
    __syncthreads();
    bitonic_lds<K>(sk, si, n2);
    for (uint32_t t = threadIdx.x; t < n; t += kSortBlock) {
        keys[t] = sk[t];
        idx[t] = si[t];
    }
}

template <class K>
__global__ __launch_bounds__(kSortBlock) void k_radix_hist(const K* keys, uint64_t n, int shift, uint32_t* gh,
                                                            uint32_t ntiles) {
    __shared__ uint32_t h[256];
    if (threadIdx.x < 256) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kSortTile;
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        uint64_t i = base + r * kSortBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[static_cast<uint32_t>(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (threadIdx.x < 256) gh[static_cast<uint64_t>(threadIdx.x) * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter of one tile for one digit.  The tile's elements are first
// placed in LDS in (digit, original order) order, then written out in that
// order, so consecutive threads store consecutive positions of one digit's
// run (coalesced lines instead of one line per lane).
template <class K>
__global__ __launch_bounds__(kSortBlock) void k_radix_scatter(const K* kin, const uint32_t* iin, K* kout,
                                                               uint32_t* iout, uint64_t n, int shift,
                                                               const uint32_t* gofs, uint32_t ntiles) {
    __shared__ uint32_t wcnt[kSortBlock / 64][256];
    __shared__ uint32_t run[256];
    __shared__ uint32_t base[256];   // global position of this tile's run of digit d
    __shared__ uint32_t lstart[256]; // position of that run inside the tile
    __shared__ uint32_t sh[33];
    __shared__ K tk[kSortTile];
    __shared__ uint32_t ti[kSortTile];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const uint64_t tbase = static_cast<uint64_t>(blockIdx.x) * kSortTile;
    if (tid < 256) {
        run[tid] = 0;
        const uint64_t at = static_cast<uint64_t>(tid) * ntiles + blockIdx.x;
        base[tid] = gofs[at];
    }
    __syncthreads();
    // this tile's count of digit d: the next offset in digit-major order
    // (the next tile's for d, or the next digit's first tile) minus its own
    {
        uint32_t c = 0;
        if (tid < 256) {
            const uint64_t at = static_cast<uint64_t>(tid) * ntiles + blockIdx.x;
            const uint64_t nxt = at + 1 < static_cast<uint64_t>(ntiles) * 256 ? gofs[at + 1] : n;
            c = static_cast<uint32_t>(nxt - base[tid]);
        }
        uint32_t tot;
        const uint32_t st = block_excl_scan<uint32_t>(c, sh, &tot);
        if (tid < 256) lstart[tid] = st;
    }
    __syncthreads();
    const uint64_t lt = (1ull << lane) - 1ull;
    for (int r = 0; r < kSortRounds; ++r) {
        uint32_t* flat = &wcnt[0][0];
        for (int j = tid; j < (kSortBlock / 64) * 256; j += kSortBlock) flat[j] = 0;
        __syncthreads();
        const uint64_t i = tbase + r * kSortBlock + tid;
        const bool valid = i < n;
        K k = valid ? kin[i] : K(0);
        uint32_t d = static_cast<uint32_t>(k >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t rank = static_cast<uint32_t>(__popcll(peers & lt));
        if (valid && rank == 0) wcnt[w][d] = static_cast<uint32_t>(__popcll(peers));
        __syncthreads();
        if (tid < 256) {
            uint32_t acc = run[tid];
#pragma unroll
            for (int ww = 0; ww < kSortBlock / 64; ++ww) {
                uint32_t c = wcnt[ww][tid];
                wcnt[ww][tid] = acc;
                acc += c;
            }
            run[tid] = acc;
        }
        __syncthreads();
        if (valid) {
            const uint32_t p = lstart[d] + wcnt[w][d] + rank;  // place in the tile
            tk[p] = k;
            ti[p] = iin[i];
        }
        __syncthreads();
    }
    const uint64_t cnt = n - tbase < kSortTile ? n - tbase : kSortTile;
    for (uint32_t p = tid; p < cnt; p += kSortBlock) {
        const K k = tk[p];
        const uint32_t d = static_cast<uint32_t>(k >> shift) & 255u;
        const uint64_t dst = static_cast<uint64_t>(base[d]) + (p - lstart[d]);
        kout[dst] = k;
        iout[dst] = ti[p];
    }
}

template <class K>
void sort_pairs(K* keys, uint32_t* idx, K* keys_alt, uint32_t* idx_alt, uint64_t n, void* tmp, hipStream_t s) {
    if (n <= 1) return;
    if (n <= kBitonicMax) {
        uint32_t n2 = 2;
        while (n2 < n) n2 <<= 1;
        hipLaunchKernelGGL(k_bitonic<K>, dim3(1), dim3(kSortBlock), 0, s, keys, idx, static_cast<uint32_t>(n), n2);
        return;
    }
    const uint32_t nt = sort_tiles(n);
    uint32_t* gh = reinterpret_cast<uint32_t*>(tmp);
    void* stmp = reinterpret_cast<uint8_t*>(tmp) + ((static_cast<uint64_t>(nt) * 256 * 4 + 255) / 256) * 256;
    K* ka = keys; uint32_t* ia = idx;
    K* kb = keys_alt; uint32_t* ib = idx_alt;
    for (int shift = 0; shift < static_cast<int>(sizeof(K) * 8); shift += 8) {
        hipLaunchKernelGGL(k_radix_hist<K>, dim3(nt), dim3(kSortBlock), 0, s, ka, n, shift, gh, nt);
        scan_exclusive<uint32_t>(gh, gh, nullptr, nullptr, static_cast<uint64_t>(nt) * 256, stmp, s);
        hipLaunchKernelGGL(k_radix_scatter<K>, dim3(nt), dim3(kSortBlock), 0, s, ka, ia, kb, ib, n, shift, gh, nt);
        K* tk = ka; ka = kb; kb = tk;
        uint32_t* ti = ia; ia = ib; ib = ti;
    }
    // sizeof(K) passes is even, so the result is back in keys/idx
}

// ------------------------------------------------------------ rank sort
//
// Every workgroup holds all B keys in LDS and 16 lanes share one element's
// count, so the B^2 comparisons spread over B / 16 CUs instead of the one
// CU a workgroup-local sort would use.
constexpr uint32_t kRankLanes = 16;  // lanes sharing one element's count

template <class K>
__global__ __launch_bounds__(256) void k_rank_sort(const K* __restrict__ keys, uint32_t B, K* __restrict__ osk,
                                                   uint32_t* __restrict__ osi, uint32_t* zero, uint32_t zero_words) {
    __shared__ K sk[kRankSortMax];
    if (zero && blockIdx.x == 0)
        for (uint32_t i = threadIdx.x; i < zero_words; i += blockDim.x) zero[i] = 0;
    for (uint32_t i = threadIdx.x; i < B; i += blockDim.x) sk[i] = keys[i];
    __syncthreads();
    const uint32_t e = (blockIdx.x * blockDim.x + threadIdx.x) / kRankLanes, l = threadIdx.x % kRankLanes;
    if (e >= B) return;  // whole groups of lanes leave together
    const K ke = sk[e];
    uint32_t c = 0;
    // lane l takes keys l, l + 16, ...: neighbouring lanes read neighbouring
    // LDS words (no bank conflicts); eight reads in flight per batch
    constexpr uint32_t R = 8;
    uint32_t j = l;
    for (; j + kRankLanes * (R - 1) < B; j += kRankLanes * R) {
        K kj[R];
#pragma unroll
        for (uint32_t u = 0; u < R; ++u) kj[u] = sk[j + kRankLanes * u];
#pragma unroll
        for (uint32_t u = 0; u < R; ++u) {
            const uint32_t jj = j + kRankLanes * u;
            c += (kj[u] < ke || (kj[u] == ke && jj < e)) ? 1u : 0u;
        }
    }
    for (; j < B; j += kRankLanes) {
        const K kj = sk[j];
        c += (kj < ke || (kj == ke && j < e)) ? 1u : 0u;
    }
#pragma unroll
    for (uint32_t m = 1; m < kRankLanes; m <<= 1) c += __shfl_xor(c, static_cast<int>(m), 64);
    if (l == 0) {
        osk[c] = ke;
        osi[c] = e;
    }
}

template <class K>
void rank_sort_small(const K* keys, uint32_t B, K* sk, uint32_t* si, uint32_t* zero, uint32_t zero_words,
                     hipStream_t s) {
    const uint32_t grid = (B * kRankLanes + 255) / 256;
    hipLaunchKernelGGL(k_rank_sort<K>, dim3(grid < 1 ? 1 : grid), dim3(256), 0, s, keys, B, sk, si, zero,
                       zero_words);
}

template void rank_sort_small<uint32_t>(const uint32_t*, uint32_t, uint32_t*, uint32_t*, uint32_t*, uint32_t,
                                        hipStream_t);
template void rank_sort_small<uint64_t>(const uint64_t*, uint32_t, uint64_t*, uint32_t*, uint32_t*, uint32_t,
                                        hipStream_t);

template void sort_pairs<uint32_t>(uint32_t*, uint32_t*, uint32_t*, uint32_t*, uint64_t, void*, hipStream_t);
template void sort_pairs<uint64_t>(uint64_t*, uint32_t*, uint64_t*, uint32_t*, uint64_t, void*, hipStream_t);

}  // namespace gt
