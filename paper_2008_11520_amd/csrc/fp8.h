// OCP FP8 E4M3 conversion on gfx950 (kernel sources only).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dnnmg {

// Four FP32 values to E4M3 codes (round to nearest even), byte 0 = a.  The
// hardware conversion gives NaN above 464, so inputs are clamped to the
// largest finite value first: the quantisers only pass values within an FP32
// rounding of 448.
__device__ inline float clamp_e4m3(float x) { return fminf(fmaxf(x, -448.0f), 448.0f); }
__device__ inline uint32_t pack4_e4m3(float a, float b, float c, float d)
{
    int w = __builtin_amdgcn_cvt_pk_fp8_f32(clamp_e4m3(a), clamp_e4m3(b), 0, false);
    w = __builtin_amdgcn_cvt_pk_fp8_f32(clamp_e4m3(c), clamp_e4m3(d), w, true);
    return (uint32_t)w;
}

// One E4M3 code of an FP32 value.
__device__ inline uint8_t to_e4m3(float a)
{
    return (uint8_t)(__builtin_amdgcn_cvt_pk_fp8_f32(clamp_e4m3(a), 0.0f, 0, false) & 0xff);
}

}  // namespace dnnmg
