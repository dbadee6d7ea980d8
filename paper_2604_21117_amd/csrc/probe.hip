// Memory-system probes (gtree_probe.h): diagnostics that measure the
// launch cost, dependent-load latency, random line-read rate and the
// dependent-round chain of a lookup-shaped batch on the GPU they run on.
// They share nothing with the tree but the wave helpers.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/gtree_probe.h"
#include "common.h"

namespace gt {
namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    // splitmix64's output mixer (Steele, Lea and Flood, 2014)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t shfl_u64p(uint64_t v, int src) {
    const uint32_t lo = shfl_u32(static_cast<uint32_t>(v), src);
    const uint32_t hi = shfl_u32(static_cast<uint32_t>(v >> 32), src);
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

__global__ void k_probe_empty() {}

// each workgroup's XCC (bits 3:0 of the XCC_ID hardware register)
__global__ void k_probe_xcc(uint32_t* out, uint32_t n) {
    if (threadIdx.x == 0 && blockIdx.x < n) out[blockIdx.x] = __builtin_amdgcn_s_getreg((15 << 11) | 20) & 0xFu;
}

__global__ void k_probe_chase(const uint64_t* __restrict__ next, uint64_t steps, uint64_t start,
                              uint64_t* __restrict__ out) {
    if (threadIdx.x != 0) return;
    uint64_t x = start;
    for (uint64_t s = 0; s < steps; ++s) x = next[x];
    out[0] = x;
}

constexpr int kG = 8;              // lanes per line: 8 x 16 bytes
constexpr uint32_t kMaxLines = 8;  // reads per round of a probe batch

bool pow2(uint64_t x) { return x && !(x & (x - 1)); }

__global__ __launch_bounds__(256) void k_probe_gather(const uint64_t* __restrict__ region, uint64_t lines, uint64_t n,
                                                      uint32_t per_group, uint64_t seed, uint64_t* __restrict__ out) {
    const int lane = threadIdx.x & 63, gl = lane % kG;
    const uint64_t group = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kG;
    const uint64_t groups = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kG;
    uint64_t acc = 0;
    for (uint64_t r0 = group * per_group; r0 < n; r0 += groups * per_group) {
#pragma unroll 8
        for (uint32_t u = 0; u < per_group; ++u) {
            const uint64_t r = r0 + u;
            if (r < n) {
                const uint64_t line = mix64(r ^ seed) & (lines - 1);
                const uint4 v = *reinterpret_cast<const uint4*>(region + line * 16 + gl * 2);
                acc ^= (static_cast<uint64_t>(v.y) << 32 | v.x) ^ (static_cast<uint64_t>(v.w) << 32 | v.z);
            }
        }
    }
    if (acc == 0x5EED5EED5EED5EEDull) out[0] = acc;  // practically never; keeps the reads live
}

__global__ void k_probe_batch(const uint64_t* __restrict__ q, uint64_t B, const uint64_t* __restrict__ table,
                              uint64_t table_lines, uint32_t table_rounds, const uint64_t* __restrict__ region,
                              uint64_t region_lines, uint32_t region_rounds, uint32_t lines_per_round,
                              uint64_t* __restrict__ out) {
    const int lane = threadIdx.x & 63, gl = lane % kG, gbase = lane - gl;
    const uint64_t group = (blockIdx.x * static_cast<uint64_t>(blockDim.x) + threadIdx.x) / kG;
    const uint64_t groups = (static_cast<uint64_t>(gridDim.x) * blockDim.x) / kG;
    for (uint64_t i = group; i < B; i += groups) {
        uint64_t x = q[i];
        for (uint32_t r = 0; r < table_rounds; ++r) {
            const uint64_t line = mix64(x + r) & (table_lines - 1);
            const uint4 v = *reinterpret_cast<const uint4*>(table + line * 16 + gl * 2);
            x = shfl_u64p(x ^ (static_cast<uint64_t>(v.y) << 32 | v.x), gbase);
        }
        for (uint32_t r = 0; r < region_rounds; ++r) {
            // the round's reads are issued together, then combined
            uint4 v[kMaxLines];
#pragma unroll
            for (uint32_t l = 0; l < kMaxLines; ++l)
                if (l < lines_per_round) {
                    const uint64_t line = mix64(x + 977 * l + r) & (region_lines - 1);
                    v[l] = *reinterpret_cast<const uint4*>(region + line * 16 + gl * 2);
                }
            uint64_t acc = 0;
#pragma unroll
            for (uint32_t l = 0; l < kMaxLines; ++l)
                if (l < lines_per_round) acc ^= static_cast<uint64_t>(v[l].y) << 32 | v[l].x;
            x = shfl_u64p(x ^ acc, gbase);
        }
        if (gl == 0) out[i] = x;
    }
}

uint32_t grid_of_probe(uint64_t threads, int block, uint64_t cap) {
    uint64_t g = (threads + block - 1) / block;
    if (g > cap) g = cap;
    return static_cast<uint32_t>(g ? g : 1);
}

gt_status done() { return hipGetLastError() == hipSuccess ? GT_OK : GT_ERR_HIP; }

}  // namespace
}  // namespace gt

using namespace gt;

extern "C" {

gt_status gt_probe_empty(hipStream_t stream) {
    hipLaunchKernelGGL(k_probe_empty, dim3(1), dim3(64), 0, stream);
    return done();
}

gt_status gt_probe_xcc(uint32_t* out, uint32_t workgroups, hipStream_t stream) {
    if (!out || !workgroups) return GT_ERR_INVALID;
    hipLaunchKernelGGL(k_probe_xcc, dim3(workgroups), dim3(256), 0, stream, out, workgroups);
    return done();
}

gt_status gt_probe_chase(const uint64_t* next, uint64_t steps, uint64_t start, uint64_t* out, hipStream_t stream) {
    if (!next || !out || !steps) return GT_ERR_INVALID;
    hipLaunchKernelGGL(k_probe_chase, dim3(1), dim3(64), 0, stream, next, steps, start, out);
    return done();
}

gt_status gt_probe_gather(const uint64_t* region, uint64_t lines, uint64_t n, uint32_t per_group, uint64_t seed,
                          uint64_t* out, hipStream_t stream) {
    if (!region || !out || !pow2(lines) || !n || !per_group) return GT_ERR_INVALID;
    const uint64_t groups = (n + per_group - 1) / per_group;
    hipLaunchKernelGGL(k_probe_gather, dim3(grid_of_probe(groups * kG, 256, 1u << 16)), dim3(256), 0, stream, region,
                       lines, n, per_group, seed, out);
    return done();
}

gt_status gt_probe_batch(const uint64_t* q, uint64_t B, const uint64_t* table, uint64_t table_lines,
                         uint32_t table_rounds, const uint64_t* region, uint64_t region_lines, uint32_t region_rounds,
                         uint32_t lines_per_round, uint64_t* out, hipStream_t stream) {
    if (!q || !out || !B) return GT_ERR_INVALID;
    if (table_rounds && (!table || !pow2(table_lines))) return GT_ERR_INVALID;
    if (region_rounds && (!region || !pow2(region_lines) || !lines_per_round || lines_per_round > kMaxLines))
        return GT_ERR_INVALID;
    // 64-thread workgroups: a small batch spreads over as many CUs as it can
    hipLaunchKernelGGL(k_probe_batch, dim3(grid_of_probe(B * kG, 64, 8192)), dim3(64), 0, stream, q, B, table,
                       table_lines, table_rounds, region, region_lines, region_rounds, lines_per_round, out);
    return done();
}

}  // extern "C"
