// Cross-lane exchanges of a 64-wide wavefront: lane l receives the value of
// lane l ^ 2^k.  Each must be called with the whole wave active (DPP reads 0
// from an inactive lane).  xor1/xor2 are quad permutes, xor8 is a row rotate
// by 8 (the partner in a 16-lane row), xor4/xor16 are LDS swizzles and xor32
// a backwards permute through the LDS crossbar.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace halo {

__device__ __forceinline__ uint32_t lane_xor1(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0xB1, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t lane_xor2(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x4E, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t lane_xor4(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x101F);
}
__device__ __forceinline__ uint32_t lane_xor8(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x128, 0xF, 0xF, false);
}
__device__ __forceinline__ uint32_t lane_xor16(uint32_t x) {
  return (uint32_t)__builtin_amdgcn_ds_swizzle((int)x, 0x401F);
}
__device__ __forceinline__ uint32_t lane_xor32(uint32_t x) {
  const int l = (int)(threadIdx.x & 63u);
  return (uint32_t)__builtin_amdgcn_ds_bpermute((l ^ 32) << 2, (int)x);
}

// The same exchanges on FP64 / FP32 values (moved as 32-bit words).
template <uint32_t (*X)(uint32_t)>
__device__ __forceinline__ double lane_xor_f64(double v) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(v);
  const uint32_t lo = X((uint32_t)u), hi = X((uint32_t)(u >> 32));
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
template <uint32_t (*X)(uint32_t)>
__device__ __forceinline__ float lane_xor_f32(float v) {
  return __uint_as_float(X(__float_as_uint(v)));
}

}  // namespace halo
