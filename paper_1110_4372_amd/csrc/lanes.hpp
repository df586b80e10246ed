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

// Lane-half swaps (gfx950): swap_halves32 exchanges the upper 32 lanes of x
// with the lower 32 lanes of y (x keeps its lower half and takes y's lower
// half above it; y takes x's upper half below its own upper half);
// swap_halves16 does the same for the odd 16-lane rows of x and the even rows
// of y.  Combining x and y after a swap reduces lanes l and l ^ 32 (l ^ 16) of
// one value in one half and of the other value in the other half.
__device__ __forceinline__ void swap_halves32(uint32_t& x, uint32_t& y) {
  const auto r = __builtin_amdgcn_permlane32_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}
__device__ __forceinline__ void swap_halves16(uint32_t& x, uint32_t& y) {
  const auto r = __builtin_amdgcn_permlane16_swap(x, y, false, false);
  x = r[0];
  y = r[1];
}

// After a transposed 8-value reduction built from swap_halves32, swap_halves16,
// an l ^ 8 keep/send exchange and the l ^ 1, 2, 4 exchanges, lane l with
// l & 7 == 0 holds value u = 4 b3 + 2 b4 + b5 (b3..b5 bits 3..5 of l).
__device__ __forceinline__ uint32_t swap8_index() {
  const uint32_t l = threadIdx.x & 63u;
  return (((l >> 3) & 1u) << 2) | (((l >> 4) & 1u) << 1) | ((l >> 5) & 1u);
}

}  // namespace halo
