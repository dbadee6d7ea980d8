// Scans and the stable key sort (hand-written for gfx950, wave64).
//
// scan_exclusive: one workgroup of 1024 threads for up to 16 Ki elements
// (it walks the input in 4096-element rounds with a running carry), else
// reduce-then-scan over 4096-element tiles (tile sums, one-workgroup scan of
// the sums, tile scans plus offsets).
//
// sort_pairs: up to 2048 elements sort inside one workgroup with a bitonic
// network on (key, index) pairs, which orders equal keys by index and so is
// stable.  Larger inputs use LSD radix sort with 8-bit digits, one stable
// scatter kernel per pass whose tiles find their output offsets by
// decoupled look-back (below).
#include <atomic>

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
//
// For n > kBitonicMax: LSD radix sort with 8-bit digits, one scatter kernel
// per pass (the decoupled look-back of single-pass prefix scans, Merrill and
// Garland, "Single-pass Parallel Prefix Scan with Decoupled Look-back",
// NVIDIA technical report NVR-2016-002, 2016; written here for wave64 tiles).
// One kernel clears the pass tickets and tile words, one counts the digits
// of every pass over the whole input.  In a pass, each workgroup takes the
// next 4096-element tile from an atomic ticket, ranks its elements by digit
// (eight ballots per wave, per-digit prefixes over the waves in LDS),
// publishes its per-digit counts, and sums the counts of earlier tiles by
// walking back over their published words until one carries an inclusive
// prefix; it then publishes its own inclusive prefix, reorders the tile in
// LDS and writes each digit's run contiguously.  A tile waits only on tiles
// with smaller tickets, which are already running and publish their counts
// before they wait, so every wait ends; the spin is bounded all the same.
// A tile that gives up sums only part of the earlier counts, so its writes
// stay inside its digits' ranges; it marks the sort failed, later passes
// then rank and publish but write nothing, and a last kernel replaces the
// failed result by a valid sorted one (every key 0, index i at position i)
// so that whatever consumes it stays in bounds while the error is reported.

constexpr int kSortBlock = 1024;
constexpr int kSortRounds = 4;
constexpr uint64_t kSortTile = kSortBlock * kSortRounds;  // 4096
constexpr uint64_t kBitonicMax = 2048;
constexpr uint32_t kSpinMax = 1u << 20;       // a look-back that waits longer gives up
static std::atomic<uint32_t> g_spin_max{kSpinMax};  // set by the testing hook (0: give up at once)

uint32_t set_sort_spin_limit(uint32_t limit) { return g_spin_max.exchange(limit, std::memory_order_relaxed); }
constexpr uint64_t kNarrowMax = 1ull << 30;   // counts fit the 30 bits of a 32-bit tile word

static uint32_t sort_tiles(uint64_t n) { return static_cast<uint32_t>((n + kSortTile - 1) / kSortTile); }

struct SortLayout {
    uint64_t totals, tickets, fail, flags, bytes;
};

static SortLayout sort_layout(uint64_t n, int key_bytes) {
    const uint64_t nt = sort_tiles(n), w = n < kNarrowMax ? 4 : 8;
    auto al = [](uint64_t x) { return (x + 255) / 256 * 256; };
    SortLayout L{};
    uint64_t o = 0;
    L.totals = o;  o += al(static_cast<uint64_t>(key_bytes) * 256 * 4);
    L.tickets = o; o += al(static_cast<uint64_t>(key_bytes) * 4);
    L.fail = o;    o += al(4);
    L.flags = o;   o += al(static_cast<uint64_t>(key_bytes) * nt * 256 * w);
    L.bytes = o;
    return L;
}

uint64_t sort_tmp_bytes(uint64_t n, int key_bytes) { return sort_layout(n, key_bytes).bytes; }

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
__global__ __launch_bounds__(256) void k_sort_stage(const K* __restrict__ src, uint64_t n, K* __restrict__ keys,
                                                    uint32_t* __restrict__ idx) {
    const uint64_t i = blockIdx.x * 256ull + threadIdx.x;
    if (i < n) {
        keys[i] = src[i];
        idx[i] = static_cast<uint32_t>(i);
    }
}

__global__ __launch_bounds__(256) void k_sort_clear(uint32_t* w, uint64_t words) {
    for (uint64_t i = blockIdx.x * 256ull + threadIdx.x; i < words; i += gridDim.x * 256ull) w[i] = 0;
}

// Digit counts of every pass over the whole input.
template <class K>
__global__ __launch_bounds__(kSortBlock) void k_sort_hist(const K* __restrict__ keys, uint64_t n,
                                                           uint32_t* __restrict__ totals) {
    constexpr int P = sizeof(K);
    __shared__ uint32_t h[P * 256];
    for (int i = threadIdx.x; i < P * 256; i += kSortBlock) h[i] = 0;
    __syncthreads();
    for (uint64_t i = blockIdx.x * static_cast<uint64_t>(kSortBlock) + threadIdx.x; i < n;
         i += static_cast<uint64_t>(gridDim.x) * kSortBlock) {
        const K k = keys[i];
#pragma unroll
        for (int p = 0; p < P; ++p) atomicAdd(&h[p * 256 + (static_cast<uint32_t>(k >> (8 * p)) & 255u)], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < P * 256; i += kSortBlock)
        if (h[i]) atomicAdd(&totals[i], h[i]);
}

// One pass over the digit at `shift`; `totals` are this pass's digit counts,
// `flags` its tile words (2 flag bits: 1 = tile count, 2 = inclusive prefix).
// Without `iin` the element at position i carries index i.
template <class K, class W>
__global__ __launch_bounds__(kSortBlock) void k_sort_pass(const K* __restrict__ kin, const uint32_t* __restrict__ iin,
                                                           K* __restrict__ kout, uint32_t* __restrict__ iout, uint64_t n,
                                                           int shift, const uint32_t* __restrict__ totals,
                                                           uint32_t* ticket, W* flags, uint32_t* fail,
                                                           uint32_t* err, uint32_t err_bit, uint32_t spin_max) {
    constexpr int kSh = static_cast<int>(sizeof(W)) * 8 - 2;
    constexpr W kAgg = W(1) << kSh, kIncl = W(2) << kSh, kVal = (W(1) << kSh) - 1;
    __shared__ uint32_t wcnt[kSortBlock / 64][256];
    __shared__ uint32_t part[4][256];  // per digit: counts of four waves each
    __shared__ uint32_t run[256];
    __shared__ uint32_t lstart[256];  // this tile's run of digit d inside the tile
    __shared__ uint64_t gbase[256];   // and in the output
    __shared__ uint32_t sh[33];
    __shared__ uint32_t s_tile, s_failed;
    __shared__ K tk[kSortTile];
    __shared__ uint32_t ti[kSortTile];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    if (tid == 0) {
        s_tile = atomicAdd(ticket, 1u);
        s_failed = __hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const uint32_t tile = s_tile;
    const bool failed = s_failed != 0;  // an earlier tile gave up: write nothing
    const uint64_t tbase = static_cast<uint64_t>(tile) * kSortTile;
    // rank the tile's elements by digit, in input order.  Wave w ranks the
    // tile's w-th block of 256 elements, four 64-element chunks in order,
    // against its own per-digit running count in LDS (one wave's LDS
    // operations take effect in order, so the chunks need no barrier); a
    // prefix over the waves then offsets each wave's runs.  Every chunk's
    // key and index are loaded up front.
    constexpr int kPerWave = kSortTile / (kSortBlock / 64);  // 256
    const uint64_t lt = (1ull << lane) - 1ull;
    K kr[kSortRounds];
    uint32_t dr[kSortRounds], rr[kSortRounds], ir[kSortRounds];
    bool vr[kSortRounds];
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const uint64_t i = tbase + static_cast<uint64_t>(w) * kPerWave + r * 64 + lane;
        vr[r] = i < n;
        kr[r] = vr[r] ? kin[i] : K(0);
        ir[r] = vr[r] ? (iin ? iin[i] : static_cast<uint32_t>(i)) : 0u;
    }
    {
        uint32_t* flat = &wcnt[0][0];
        for (int j = tid; j < (kSortBlock / 64) * 256; j += kSortBlock) flat[j] = 0;
    }
    // where each digit starts in the output: scan of the pass's totals (its
    // barriers also order the clearing above before the counting below)
    uint32_t tot;
    const uint32_t dstart = block_excl_scan<uint32_t>(tid < 256 ? totals[tid] : 0u, sh, &tot);
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        const bool valid = vr[r];
        const uint32_t d = static_cast<uint32_t>(kr[r] >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const uint64_t m = __ballot((d >> b) & 1u);
            peers &= ((d >> b) & 1u) ? m : ~m;
        }
        const uint32_t base = wcnt[w][d];
        const uint32_t rank = static_cast<uint32_t>(__popcll(peers & lt));
        __builtin_amdgcn_wave_barrier();
        if (valid && rank == 0) wcnt[w][d] = base + static_cast<uint32_t>(__popcll(peers));
        __builtin_amdgcn_wave_barrier();
        dr[r] = d;
        rr[r] = base + rank;  // rank among this wave's elements of digit d
    }
    __syncthreads();
    // per digit, offsets of the waves' runs: thread (digit, q) sums waves
    // 4q..4q+3, then adds the earlier quarters
    {
        static_assert(kSortBlock == 1024, "four threads per digit, four waves each");
        const int dd = tid & 255, q = tid >> 8;
        const uint32_t c0 = wcnt[4 * q][dd], c1 = wcnt[4 * q + 1][dd];
        const uint32_t c2 = wcnt[4 * q + 2][dd], c3 = wcnt[4 * q + 3][dd];
        part[q][dd] = c0 + c1 + c2 + c3;
        __syncthreads();
        uint32_t b0 = 0;
        for (int qq = 0; qq < q; ++qq) b0 += part[qq][dd];
        wcnt[4 * q][dd] = b0;
        wcnt[4 * q + 1][dd] = b0 + c0;
        wcnt[4 * q + 2][dd] = b0 + c0 + c1;
        wcnt[4 * q + 3][dd] = b0 + c0 + c1 + c2;
        if (q == 3) run[dd] = b0 + c0 + c1 + c2 + c3;
        __syncthreads();
    }
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) rr[r] += vr[r] ? wcnt[w][dr[r]] : 0u;

    // publish this tile's counts, look back for the earlier tiles' sums
    if (tid < 256) {
        const uint32_t cnt = run[tid];
        W* mine = flags + static_cast<uint64_t>(tile) * 256 + tid;
        uint64_t excl = 0;
        if (tile == 0) {
            __hip_atomic_store(mine, kIncl | static_cast<W>(cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else if (spin_max == 0) {
            // forced from the host (testing): give up without waiting, still
            // publishing a prefix so that no later tile waits either
            atomicOr(fail, 1u);
            if (err) atomicOr(err, err_bit);
            __hip_atomic_store(mine, kIncl | static_cast<W>(cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        } else {
            __hip_atomic_store(mine, kAgg | static_cast<W>(cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            // eight earlier tiles per step, their words read together; sum
            // counts until an inclusive prefix, resume at a tile not yet
            // published
            constexpr int kLook = 8;
            int64_t j = static_cast<int64_t>(tile) - 1;
            uint32_t spins = 0;
            bool done = false;
            while (!done) {
                W x[kLook];
#pragma unroll
                for (int q = 0; q < kLook; ++q)
                    x[q] = j - q >= 0 ? __hip_atomic_load(flags + static_cast<uint64_t>(j - q) * 256 + tid,
                                                          __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                      : kIncl;  // never reached: tile 0 publishes an inclusive prefix
                int used = 0;
#pragma unroll
                for (int q = 0; q < kLook; ++q) {
                    if (done || used < q) continue;  // stopped at an earlier word
                    const W f = x[q] >> kSh;
                    if (f == 0) continue;  // not yet published
                    excl += x[q] & kVal;
                    ++used;
                    if (f == 2) done = true;
                }
                j -= used;
                if (!done && used == 0 && ++spins > spin_max) {
                    atomicOr(fail, 1u);
                    if (err) atomicOr(err, err_bit);
                    break;
                }
            }
            __hip_atomic_store(mine, kIncl | static_cast<W>(excl + cnt), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        gbase[tid] = static_cast<uint64_t>(dstart) + excl;
    }
    {
        uint32_t t2;
        const uint32_t st = block_excl_scan<uint32_t>(tid < 256 ? run[tid] : 0u, sh, &t2);
        if (tid < 256) lstart[tid] = st;
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kSortRounds; ++r) {
        if (vr[r]) {
            const uint32_t p = lstart[dr[r]] + rr[r];
            tk[p] = kr[r];
            ti[p] = ir[r];
        }
    }
    __syncthreads();
    if (failed) return;  // the same for the whole workgroup, after its last barrier
    const uint64_t cnt = n - tbase < kSortTile ? n - tbase : kSortTile;
    for (uint32_t p = tid; p < cnt; p += kSortBlock) {
        const K k = tk[p];
        const uint32_t d = static_cast<uint32_t>(k >> shift) & 255u;
        const uint64_t dst = gbase[d] + (p - lstart[d]);
        kout[dst] = k;
        iout[dst] = ti[p];
    }
}

// After the passes: a failed sort's result becomes every key 0, index i at
// position i (sorted, and a valid permutation).  One workgroup: the check
// costs one small dispatch, and the rewrite happens only after a failure.
template <class K>
__global__ __launch_bounds__(1024) void k_sort_fix(K* __restrict__ keys, uint32_t* __restrict__ idx, uint64_t n,
                                                   const uint32_t* fail) {
    if (__hip_atomic_load(fail, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) return;
    for (uint64_t i = threadIdx.x; i < n; i += 1024) {
        keys[i] = K(0);
        idx[i] = static_cast<uint32_t>(i);
    }
}

template <class K, class W>
static void sort_onesweep(const K* src, K* keys, uint32_t* idx, K* keys_alt, uint32_t* idx_alt, uint64_t n,
                          void* tmp, hipStream_t s, uint32_t* err_out, uint32_t err_bit) {
    constexpr int P = sizeof(K);
    const uint32_t nt = sort_tiles(n);
    const SortLayout L = sort_layout(n, P);
    uint8_t* b = reinterpret_cast<uint8_t*>(tmp);
    uint32_t* totals = reinterpret_cast<uint32_t*>(b + L.totals);
    uint32_t* tickets = reinterpret_cast<uint32_t*>(b + L.tickets);
    uint32_t* fail = reinterpret_cast<uint32_t*>(b + L.fail);
    W* flags = reinterpret_cast<W*>(b + L.flags);
    const uint64_t words = L.bytes / 4;
    const uint64_t cg = (words + 255) / 256;
    hipLaunchKernelGGL(k_sort_clear, dim3(static_cast<uint32_t>(cg < 4096 ? cg : 4096)), dim3(256), 0, s,
                       reinterpret_cast<uint32_t*>(b), words);
    const uint32_t hg = nt < 512 ? nt : 512;
    hipLaunchKernelGGL(k_sort_hist<K>, dim3(hg), dim3(kSortBlock), 0, s, src ? src : keys, n, totals);
    // pass 0 reads the source (indices 0..n-1) or keys/idx and writes the
    // alternates; sizeof(K) passes is even, so the result ends in keys/idx
    const K* ka = src ? src : keys;
    const uint32_t* ia = src ? nullptr : idx;
    K* kb = keys_alt; uint32_t* ib = idx_alt;
    for (int p = 0; p < P; ++p) {
        hipLaunchKernelGGL((k_sort_pass<K, W>), dim3(nt), dim3(kSortBlock), 0, s, ka, ia, kb, ib, n, 8 * p,
                           totals + p * 256, tickets + p, flags + static_cast<uint64_t>(p) * nt * 256, fail,
                           err_out, err_bit, g_spin_max.load(std::memory_order_relaxed));
        ka = kb;
        ia = ib;
        kb = (p & 1) ? keys_alt : keys;
        ib = (p & 1) ? idx_alt : idx;
    }
    hipLaunchKernelGGL(k_sort_fix<K>, dim3(1), dim3(1024), 0, s, keys, idx, n, fail);
}

template <class K>
void sort_pairs(K* keys, uint32_t* idx, K* keys_alt, uint32_t* idx_alt, uint64_t n, void* tmp, hipStream_t s,
                uint32_t* err, uint32_t err_bit) {
    if (n <= 1) return;
    if (n <= kBitonicMax) {
        uint32_t n2 = 2;
        while (n2 < n) n2 <<= 1;
        hipLaunchKernelGGL(k_bitonic<K>, dim3(1), dim3(kSortBlock), 0, s, keys, idx, static_cast<uint32_t>(n), n2);
        return;
    }
    if (n < kNarrowMax) sort_onesweep<K, uint32_t>(nullptr, keys, idx, keys_alt, idx_alt, n, tmp, s, err, err_bit);
    else sort_onesweep<K, uint64_t>(nullptr, keys, idx, keys_alt, idx_alt, n, tmp, s, err, err_bit);
}

template <class K>
void sort_from(const K* src, K* keys, uint32_t* idx, K* keys_alt, uint32_t* idx_alt, uint64_t n, void* tmp,
               hipStream_t s, uint32_t* err, uint32_t err_bit) {
    if (n <= kBitonicMax) {
        // stage (key, position) pairs, then the in-workgroup sort
        hipLaunchKernelGGL(k_sort_stage<K>, dim3(static_cast<uint32_t>((n + 255) / 256 ? (n + 255) / 256 : 1)),
                           dim3(256), 0, s, src, n, keys, idx);
        sort_pairs<K>(keys, idx, keys_alt, idx_alt, n, tmp, s, err, err_bit);
        return;
    }
    if (n < kNarrowMax) sort_onesweep<K, uint32_t>(src, keys, idx, keys_alt, idx_alt, n, tmp, s, err, err_bit);
    else sort_onesweep<K, uint64_t>(src, keys, idx, keys_alt, idx_alt, n, tmp, s, err, err_bit);
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

template void sort_pairs<uint32_t>(uint32_t*, uint32_t*, uint32_t*, uint32_t*, uint64_t, void*, hipStream_t,
                                   uint32_t*, uint32_t);
template void sort_from<uint32_t>(const uint32_t*, uint32_t*, uint32_t*, uint32_t*, uint32_t*, uint64_t, void*,
                                  hipStream_t, uint32_t*, uint32_t);
template void sort_from<uint64_t>(const uint64_t*, uint64_t*, uint32_t*, uint64_t*, uint32_t*, uint64_t, void*,
                                  hipStream_t, uint32_t*, uint32_t);
template void sort_pairs<uint64_t>(uint64_t*, uint32_t*, uint64_t*, uint32_t*, uint64_t, void*, hipStream_t,
                                   uint32_t*, uint32_t);

}  // namespace gt
