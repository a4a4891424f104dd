// Cross-lane moves of a double between adjacent lanes of a 64-wide wave (the
// i -+ 1 neighbours of a spatial stencil), shared by the matvec kernels: a DPP
// wave shift when DPP is set, else ds_bpermute.  Lane 0 (from the left) and lane
// 63 (from the right) receive no wave neighbour; callers supply those values.
#pragma once
#include <hip/hip_runtime.h>

namespace aao {

template <bool DPP>
__device__ __forceinline__ double lane_from_left(double v)
{
    if constexpr (DPP) {
        // wave_shr:1 -- lane j receives lane j-1
        const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x138, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x138, 0xf, 0xf, false);
        return __hiloint2double(hi, lo);
    } else {
        return __shfl_up(v, 1, 64);
    }
}
template <bool DPP>
__device__ __forceinline__ double lane_from_right(double v)
{
    if constexpr (DPP) {
        // wave_shl:1 -- lane j receives lane j+1
        const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
        const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
        return __hiloint2double(hi, lo);
    } else {
        return __shfl_down(v, 1, 64);
    }
}

}  // namespace aao
