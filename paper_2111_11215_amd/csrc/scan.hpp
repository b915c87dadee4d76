// Wavefront-wide float scans shared by the per-ray kernels (compositing
// and its adjoint, the coarse stage).
#pragma once
#include <hip/hip_runtime.h>

namespace dvgo_dev {

// Wavefront scans on DPP lane shifts (VALU operands, no LDS round trip):
// a Hillis-Steele scan inside each row of 16 lanes (row_shr / row_shl by 1,
// 2, 4, 8; a lane whose source is outside its row reads 0), then each row
// adds the totals of the rows before (prefix) or after (suffix) it, read
// from one lane of each row.
template <int kCtrl>
__device__ __forceinline__ float dpp_in_row(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl, 0xf, 0xf, true));
}
// whole-wavefront shift by one lane (wave_shr:1 / wave_shl:1); the lane
// without a source reads 0
template <int kCtrl>
__device__ __forceinline__ float dpp_wave(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), kCtrl, 0xf, 0xf, true));
}
__device__ __forceinline__ float lane_value(float v, int l) {
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}

// inclusive prefix sum: sum over lanes <= lane
__device__ __forceinline__ float wave_incl_scan(float v, int lane) {
    v += dpp_in_row<0x111>(v);   // row_shr:1
    v += dpp_in_row<0x112>(v);   // row_shr:2
    v += dpp_in_row<0x114>(v);   // row_shr:4
    v += dpp_in_row<0x118>(v);   // row_shr:8
    const float t0 = lane_value(v, 15), t1 = lane_value(v, 31), t2 = lane_value(v, 47);
    const int row = lane >> 4;
    return v + (row == 0 ? 0.0f : row == 1 ? t0 : row == 2 ? t0 + t1 : (t0 + t1) + t2);
}
// inclusive suffix sum: sum over lanes >= lane
__device__ __forceinline__ float wave_incl_suffix(float v, int lane) {
    v += dpp_in_row<0x101>(v);   // row_shl:1
    v += dpp_in_row<0x102>(v);   // row_shl:2
    v += dpp_in_row<0x104>(v);   // row_shl:4
    v += dpp_in_row<0x108>(v);   // row_shl:8
    const float s1 = lane_value(v, 16), s2 = lane_value(v, 32), s3 = lane_value(v, 48);
    const int row = lane >> 4;
    return v + (row == 3 ? 0.0f : row == 2 ? s3 : row == 1 ? s2 + s3 : s1 + (s2 + s3));
}
__device__ __forceinline__ float wave_sum(float v) {
    return lane_value(wave_incl_scan(v, static_cast<int>(threadIdx.x & 63)), 63);
}

}  // namespace dvgo_dev
