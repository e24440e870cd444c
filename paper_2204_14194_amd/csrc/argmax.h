// Wave-level selection of the largest |R| with the lowest index among exact
// ties, shared by the iteration-loop kernels.  A candidate is packed into a
// 64-bit key
//     |R| bits << 32  |  (0xFFFF - k) << 16  |  sign << 15
// (|R| >= 0, so its float bits order like integers); the maximum key over
// the wave is found with DPP lane permutations (no LDS traffic).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sefase {

// DPP controls (gfx9 encoding)
constexpr int kQuadXor1 = 0xB1;       // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;       // quad_perm [2,3,0,1]
constexpr int kRowHalfMirror = 0x141;
constexpr int kRowMirror = 0x140;
constexpr int kRowBcast15 = 0x142;
constexpr int kRowBcast31 = 0x143;

template <int CTRL, int ROWMASK>
__device__ __forceinline__ void key_step(uint32_t& hi, uint32_t& lo) {
  const uint32_t ohi = (uint32_t)__builtin_amdgcn_update_dpp((int)hi, (int)hi, CTRL, ROWMASK, 0xF, false);
  const uint32_t olo = (uint32_t)__builtin_amdgcn_update_dpp((int)lo, (int)lo, CTRL, ROWMASK, 0xF, false);
  const uint64_t a = ((uint64_t)ohi << 32) | olo;
  const uint64_t b = ((uint64_t)hi << 32) | lo;
  if (a > b) {
    hi = ohi;
    lo = olo;
  }
}

// Maximum 64-bit key over the wave, returned wave-uniform.
__device__ __forceinline__ uint64_t wave_max_key(uint32_t hi, uint32_t lo) {
  key_step<kQuadXor1, 0xF>(hi, lo);
  key_step<kQuadXor2, 0xF>(hi, lo);
  key_step<kRowHalfMirror, 0xF>(hi, lo);
  key_step<kRowMirror, 0xF>(hi, lo);          // every row of 16 lanes now uniform
  key_step<kRowBcast15, 0xA>(hi, lo);         // rows 1, 3 take rows 0, 2
  key_step<kRowBcast31, 0xC>(hi, lo);         // rows 2, 3 take row 1 -> lane 63 holds the max
  const uint32_t h = (uint32_t)__builtin_amdgcn_readlane((int)hi, 63);
  const uint32_t l = (uint32_t)__builtin_amdgcn_readlane((int)lo, 63);
  return ((uint64_t)h << 32) | l;
}

// Maximum 64-bit key over each aligned group of G lanes (G a power of two up
// to 16), returned wave-uniform: every group must hold the same G keys (as
// when lane i holds item i mod G), so each group's maximum is the maximum.
template <int G>
__device__ __forceinline__ uint64_t group_max_key(uint32_t hi, uint32_t lo) {
  static_assert(G >= 1 && G <= 16 && (G & (G - 1)) == 0, "groups within a row of 16 lanes");
  if constexpr (G >= 2) key_step<kQuadXor1, 0xF>(hi, lo);
  if constexpr (G >= 4) key_step<kQuadXor2, 0xF>(hi, lo);
  if constexpr (G >= 8) key_step<kRowHalfMirror, 0xF>(hi, lo);
  if constexpr (G >= 16) key_step<kRowMirror, 0xF>(hi, lo);
  const uint32_t h = (uint32_t)__builtin_amdgcn_readfirstlane((int)hi);
  const uint32_t l = (uint32_t)__builtin_amdgcn_readfirstlane((int)lo);
  return ((uint64_t)h << 32) | l;
}

__device__ __forceinline__ uint64_t make_key(float v, int idx) {
  const uint32_t bits = __float_as_uint(v);
  const uint32_t hi = bits & 0x7FFFFFFFu;
  const uint32_t lo = ((uint32_t)(0xFFFF - idx) << 16) | ((bits >> 31) << 15);
  return ((uint64_t)hi << 32) | lo;
}


// Maximum over the wave of a non-negative float, returned wave-uniform.
// Non-negative floats order like their bit patterns, so the reduction runs
// on unsigned integers: with 0 (the identity of unsigned max) as the value
// of lanes a step does not write, each step folds into one v_max_u32 with a
// DPP operand.  Lanes outside rows 1 and 3 hold partial values after the
// broadcast steps; lane 63 holds the maximum.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ uint32_t umax_step(uint32_t v) {
  const uint32_t o = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xF, false);
  return v > o ? v : o;
}

__device__ __forceinline__ float wave_max_f32(float x) {
  uint32_t v = __float_as_uint(x);
  v = umax_step<kQuadXor1, 0xF>(v);
  v = umax_step<kQuadXor2, 0xF>(v);
  v = umax_step<kRowHalfMirror, 0xF>(v);
  v = umax_step<kRowMirror, 0xF>(v);
  v = umax_step<kRowBcast15, 0xA>(v);
  v = umax_step<kRowBcast31, 0xC>(v);
  return __uint_as_float((uint32_t)__builtin_amdgcn_readlane((int)v, 63));
}

// Decode the winner of a key: index and signed value; an all-zero key (no
// positive score anywhere) decodes to atom 0 with value 0.
__device__ __forceinline__ void decode_key(uint64_t key, int K, int& u, float& rv) {
  const uint32_t khi = (uint32_t)(key >> 32), klo = (uint32_t)key;
  u = 0xFFFF - (int)(klo >> 16);
  rv = __uint_as_float(khi | ((klo & 0x8000u) << 16));
  if (khi == 0u || u < 0 || u >= K) {
    u = 0;
    rv = 0.0f;
  }
}

// Keys of the class form of the loop, whose positions follow the atom order
// inside a class but not across classes: an exact tie is decided on the
// original atom index, and the position travels in the low bits,
//     |R| bits << 32  |  (0xFFFF - atom) << 16  |  sign << 15  |  position
// (positions below 2^15).
__device__ __forceinline__ uint64_t make_class_key(uint32_t vbits, int atom, int pos) {
  return ((uint64_t)(vbits & 0x7FFFFFFFu) << 32) | ((uint32_t)(0xFFFF - atom) << 16) |
         ((vbits >> 31) << 15) | (uint32_t)pos;
}

__device__ __forceinline__ void decode_class_key(uint64_t key, int& pos, float& rv) {
  const uint32_t khi = (uint32_t)(key >> 32), klo = (uint32_t)key;
  pos = (int)(klo & 0x7FFFu);
  rv = __uint_as_float(khi | ((klo & 0x8000u) << 16));
  if (khi == 0u) {
    pos = 0;
    rv = 0.0f;
  }
}

}  // namespace sefase
