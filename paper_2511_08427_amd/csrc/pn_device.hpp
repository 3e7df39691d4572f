// Device-side storage types shared by the gfx950 kernel files of the CT
// projector library: BF16/FP16 storage elements, their widening to FP32 and
// the round-to-nearest-even stores.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace pn {

// ------------------------------------------------------------ dtypes ----

struct bf16 {
    uint16_t bits;
};
using f16 = _Float16;

__device__ __forceinline__ float to_f32(float v) { return v; }
__device__ __forceinline__ float to_f32(bf16 v) { return __uint_as_float(static_cast<uint32_t>(v.bits) << 16); }
__device__ __forceinline__ float to_f32(f16 v) { return static_cast<float>(v); }

template <typename T>
__device__ __forceinline__ T from_f32(float f);
template <>
__device__ __forceinline__ float from_f32<float>(float f) { return f; }
template <>
__device__ __forceinline__ bf16 from_f32<bf16>(float f)
{
    // round to nearest, ties to even; NaN stays a (quiet) NaN
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return bf16{static_cast<uint16_t>((u >> 16) | 0x40u)};
    u += 0x7fffu + ((u >> 16) & 1u);
    return bf16{static_cast<uint16_t>(u >> 16)};
}
template <>
__device__ __forceinline__ f16 from_f32<f16>(float f)
{
    // the empty asm pins the FP32 value, so the store is the RNE rounding of
    // the FP32 result (without it the compiler may fuse the producing
    // multiply into a mixed-precision instruction that rounds only once)
    asm volatile("" : "+v"(f));
    return static_cast<f16>(f);  // v_cvt_f16_f32, round to nearest even
}

}  // namespace pn
