// Device helpers shared by the register-tiled 2-D sweeps: the complex vector
// type of a field precision and the DPP lane shifts that give a lane its x-1
// and x+1 neighbours.
#pragma once

#include <hip/hip_runtime.h>

namespace tdp {

template <typename T>
struct V2t;
template <>
struct V2t<double> {
    using type = double2;
};
template <>
struct V2t<float> {
    using type = float2;
};

// Cross-lane neighbours of a row held one node per lane (lane = tile column):
// the value of the lane to the left (x-1) or right (x+1), 0 past the wave's
// ends, which is the tile's zero pad.  DPP wave shifts by one lane (VALU
// moves; no LDS traffic).
__device__ __forceinline__ int dpp_from_left(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x138 /* wave_shr:1 */, 0xF, 0xF, true);
}
__device__ __forceinline__ int dpp_from_right(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, 0x130 /* wave_shl:1 */, 0xF, 0xF, true);
}
__device__ __forceinline__ float lane_west(float v)
{
    return __int_as_float(dpp_from_left(__float_as_int(v)));
}
__device__ __forceinline__ float lane_east(float v)
{
    return __int_as_float(dpp_from_right(__float_as_int(v)));
}
__device__ __forceinline__ double lane_west(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)dpp_from_left((int)b);
    const unsigned hi = (unsigned)dpp_from_left((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ double lane_east(double v)
{
    const long long b = __double_as_longlong(v);
    const unsigned lo = (unsigned)dpp_from_right((int)b);
    const unsigned hi = (unsigned)dpp_from_right((int)(b >> 32));
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

}  // namespace tdp
