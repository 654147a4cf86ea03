// Wavefront-wide FP64 sums by DPP lane moves (device code only).
#pragma once

#include <hip/hip_runtime.h>

namespace mbem {

// One DPP step on a double: quad swaps, half-row and row mirrors, each
// pairing a lane with a lane of the other group within its row of 16.
__device__ __forceinline__ double dpp_move(double v, int ctrl_sel) {
    const int lo = __double2loint(v), hi = __double2hiint(v);
    int l2, h2;
    switch (ctrl_sel) {
        case 0: l2 = __builtin_amdgcn_update_dpp(0, lo, 0xB1, 0xF, 0xF, false);   // quad_perm [1,0,3,2]
                h2 = __builtin_amdgcn_update_dpp(0, hi, 0xB1, 0xF, 0xF, false); break;
        case 1: l2 = __builtin_amdgcn_update_dpp(0, lo, 0x4E, 0xF, 0xF, false);   // quad_perm [2,3,0,1]
                h2 = __builtin_amdgcn_update_dpp(0, hi, 0x4E, 0xF, 0xF, false); break;
        case 2: l2 = __builtin_amdgcn_update_dpp(0, lo, 0x141, 0xF, 0xF, false);  // row_half_mirror
                h2 = __builtin_amdgcn_update_dpp(0, hi, 0x141, 0xF, 0xF, false); break;
        default: l2 = __builtin_amdgcn_update_dpp(0, lo, 0x140, 0xF, 0xF, false); // row_mirror
                 h2 = __builtin_amdgcn_update_dpp(0, hi, 0x140, 0xF, 0xF, false); break;
    }
    return __hiloint2double(h2, l2);
}
__device__ __forceinline__ double lane_value(double v, int lane) {
    return __hiloint2double(__builtin_amdgcn_readlane(__double2hiint(v), lane),
                            __builtin_amdgcn_readlane(__double2loint(v), lane));
}
// Sum over the 64 lanes, returned to every lane; all lanes must be active.
// Four dependent DPP steps give each row of 16 its sum, then the four row
// sums are read from lanes 0, 16, 32, 48 as wavefront-uniform values (a
// fixed order, so every wavefront that sums the same values gets the same
// result).
__device__ __forceinline__ double wsum_all(double v) {
    v += dpp_move(v, 0);
    v += dpp_move(v, 1);
    v += dpp_move(v, 2);
    v += dpp_move(v, 3);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

}  // namespace mbem
