// Split-BF16 operands: x = hi + lo with hi = bf16(x) and lo = bf16(x - hi),
// both rounded to nearest even (finite inputs).  The matrix cores then form
// a b as hi_a hi_b + hi_a lo_b + lo_a hi_b with FP32 accumulation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sefase {

__device__ inline uint16_t bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

__device__ inline void bf16_split(float v, uint16_t& hi, uint16_t& lo) {
  hi = bf16_rne(v);
  lo = bf16_rne(v - bf16_to_f32(hi));
}

}  // namespace sefase
