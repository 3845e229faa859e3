// Device helpers shared by the register-tiled 2-D sweeps: the complex vector
// type of a field precision, the DPP lane shifts that give a lane its x-1
// and x+1 neighbours, and the per-node fold of the cell slowness into the
// step's stencil coefficients.
#pragma once

#include <hip/hip_runtime.h>

#include "tdp_internal.h"

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

// Per-node coefficients of the step from the four cells around a node (SW,
// SE, NW, NE) and its damping factor dd: centre, W, E, S, N, then the corner
// weights (four with corner mass terms, one shared weight without).
template <typename T, int SC, int MC, int NCO>
__device__ __forceinline__ void fold_node(const Stencil<T> &st, T dd, T mSW, T mSE, T mNW, T mNE,
                                          T (&c)[NCO])
{
    c[0] = dd * (st.c0 + st.m[0] * ((mSW + mSE) + (mNW + mNE)));
    c[1] = dd * (st.s[1] + st.m[1] * (mSW + mNW));   // W
    c[2] = dd * (st.s[1] + st.m[1] * (mSE + mNE));   // E
    c[3] = dd * (st.s[1] + st.m[1] * (mSW + mSE));   // S
    c[4] = dd * (st.s[1] + st.m[1] * (mNW + mNE));   // N
    if (MC > 2) {
        c[5] = dd * (st.s[2] + st.m[2] * mSW);
        c[6] = dd * (st.s[2] + st.m[2] * mSE);
        c[7] = dd * (st.s[2] + st.m[2] * mNW);
        c[8] = dd * (st.s[2] + st.m[2] * mNE);
    } else if (SC > 2) {
        c[5] = dd * st.s[2];   // the four corners share one weight
    }
}

}  // namespace tdp
