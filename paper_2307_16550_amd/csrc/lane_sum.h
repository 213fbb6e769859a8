// Sums over groups of lanes of a wave, shared by the refinement and the
// Block-OMP right-hand side.
#pragma once

#include "gh_internal.h"

namespace gh {

// Sums over aligned groups of n lanes (n a power of two, at most 64) into each
// group's first lane; the other lanes are left with partial sums.  Within a
// row of 16 lanes, lane i adds lane i + K read by a DPP row shift (lanes past
// the row's end read zero); across rows, lane shuffles.
template <int K>
__device__ __forceinline__ float from_lane_above(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x100 + K, 0xf, 0xf, true));
}
template <int K>
__device__ __forceinline__ double from_lane_above(double v) {
    const long long b = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(unsigned)b, 0x100 + K, 0xf, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x100 + K, 0xf, 0xf, true);
    return __longlong_as_double((long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
}
template <int K, typename T, int N>
__device__ __forceinline__ void add_lane_above(T (&v)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += from_lane_above<K>(v[i]);
}
template <typename T, int N>
__device__ __forceinline__ void group_sum_to_first(T (&v)[N], int n) {
    if (n > 1) add_lane_above<1>(v);
    if (n > 2) add_lane_above<2>(v);
    if (n > 4) add_lane_above<4>(v);
    if (n > 8) add_lane_above<8>(v);
    if (n > 16) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] += __shfl_down(v[i], 16, 64);
    }
    if (n > 32) {
#pragma unroll
        for (int i = 0; i < N; ++i) v[i] += __shfl_down(v[i], 32, 64);
    }
}

}  // namespace gh
