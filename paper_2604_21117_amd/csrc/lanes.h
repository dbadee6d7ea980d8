// Cross-lane moves within a row of 16 lanes (DPP), for lane groups that
// are whole rows: the lane to read from is part of the instruction, so a
// value moves in one vector-ALU operation instead of an LDS-path round trip.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <type_traits>

namespace gt {

// The value x holds in lane S of this lane's row of 16 lanes: a DPP row
// broadcast (row_newbcast), one vector-ALU move where a cross-lane read
// would make an LDS-path round trip.  The source lane must be active.
template <int S>
__device__ __forceinline__ uint32_t row_lane(uint32_t x) {
    static_assert(S >= 0 && S < 16, "a lane of the row");
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(x), 0x150 + S, 0xf, 0xf, false));
}
template <int S>
__device__ __forceinline__ uint64_t row_lane(uint64_t x) {
    const uint32_t lo = row_lane<S>(static_cast<uint32_t>(x));
    const uint32_t hi = row_lane<S>(static_cast<uint32_t>(x >> 32));
    return (static_cast<uint64_t>(hi) << 32) | lo;
}

// f(std::integral_constant<int, I>) for I = B .. E-1, unrolled at compile
// time (for cross-lane moves whose lane is part of the instruction).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

}  // namespace gt
