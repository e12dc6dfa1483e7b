// Device helpers shared by the libfinger kernels (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#define FINGER_WAVE 64

namespace finger {

// Compiler fence for LDS traffic between lanes of one wavefront: keeps the
// compiler from moving LDS accesses across it and waits for issued LDS ops.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc64(uint64_t x) { return __popcll(x); }

// number of set bits of mask below this lane
__device__ __forceinline__ int mask_rank(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0));
}

__device__ __forceinline__ float shfl_xor_f(float v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ int shfl_i(int v, int src) { return __shfl(v, src, 64); }
__device__ __forceinline__ float shfl_f(float v, int src) { return __shfl(v, src, 64); }

// DPP lane moves inside rows of 16 lanes (no LDS traffic): quad_perm
// [1,0,3,2] and [2,3,0,1] swap neighbours and pairs, row_half_mirror maps
// lane i to 7 - i within 8, row_mirror i to 15 - i within 16.
constexpr int kDppXor1 = 0xB1, kDppXor2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float readlane_f(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}

// sum over aligned groups of G lanes (G a power of two <= 64); every lane of
// the group gets the total.  Within 16 lanes each step adds a DPP-moved copy
// (after the quad steps every lane holds its quad's sum, so the mirrors pair
// whole quads and then whole 8-lane halves); wider groups add 16- and
// 32-lane swaps.
template <int G>
__device__ __forceinline__ float group_sum(float v) {
  if constexpr (G >= 2) v += dpp_f<kDppXor1>(v);
  if constexpr (G >= 4) v += dpp_f<kDppXor2>(v);
  if constexpr (G >= 8) v += dpp_f<kDppHalfMirror>(v);
  if constexpr (G >= 16) v += dpp_f<kDppMirror>(v);
  if constexpr (G >= 32) v += shfl_xor_f(v, 16);
  if constexpr (G >= 64) v += shfl_xor_f(v, 32);
  return v;
}

// sum over the wave, as a wave-uniform (scalar) value
__device__ __forceinline__ float wave_sum(float v) {
  v = group_sum<16>(v);
  return (readlane_f(v, 0) + readlane_f(v, 16)) + (readlane_f(v, 32) + readlane_f(v, 48));
}

// uniform (scalar) copy of a wave-uniform value
__device__ __forceinline__ int uniform_i(int v) { return __builtin_amdgcn_readfirstlane(v); }
__device__ __forceinline__ float uniform_f(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}

// (d, id) keys packed so that unsigned comparison is the lexicographic
// order: the distance's bits map to an unsigned value of the same order
// (negative values, from the inner-product metric, included; -0 is folded
// into +0 so that equal distances tie on the id); ids are < 2^31.
__device__ __forceinline__ uint32_t order_bits(float f) {
  const uint32_t u = __float_as_uint(f + 0.0f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float order_bits_inv(uint32_t u) {
  return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}
__device__ __forceinline__ uint64_t make_key(float d2, int id) {
  return ((uint64_t)order_bits(d2) << 32) | (uint32_t)id;
}
__device__ __forceinline__ float key_d2(uint64_t k) { return order_bits_inv((uint32_t)(k >> 32)); }
__device__ __forceinline__ int key_id(uint64_t k) { return (int)(uint32_t)k; }

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  int lo = __shfl((int)(uint32_t)v, src, 64);
  int hi = __shfl((int)(uint32_t)(v >> 32), src, 64);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}
// v from a wave-uniform lane (scalar result)
__device__ __forceinline__ uint64_t readlane_u64(uint64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), lane);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  int lo = __shfl_xor((int)(uint32_t)v, m, 64);
  int hi = __shfl_xor((int)(uint32_t)(v >> 32), m, 64);
  return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Bitonic sort of one 64-bit key per lane over the first N lanes (N a power
// of two <= 64), ascending by lane.
template <int N>
__device__ __forceinline__ uint64_t bitonic_sort(uint64_t v) {
  const int l = lane_id();
#pragma unroll
  for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
    for (int j = k >> 1; j > 0; j >>= 1) {
      uint64_t o = shfl_xor_u64(v, j);
      bool up = ((l & k) == 0);
      bool lower = ((l & j) == 0);
      // lower lane keeps min when sorting up
      bool take_min = (lower == up);
      uint64_t mn = v < o ? v : o;
      uint64_t mx = v < o ? o : v;
      v = take_min ? mn : mx;
    }
  }
  return v;
}

// float -> nearest bfloat16 value (round to nearest even), kept as float
__device__ __forceinline__ float round_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

// bf16 -> float
__device__ __forceinline__ float bf16_to_f(uint16_t h) { return __uint_as_float(((uint32_t)h) << 16); }

// OCP FP8 E4M3 (bias 7, no infinities, 0x7f/0xff = NaN, max 448) -> float
__device__ __forceinline__ float e4m3_to_f(uint8_t b) {
  const uint32_t s = (b >> 7) & 1u, e = (b >> 3) & 0xFu, mt = b & 7u;
  float v;
  if (e == 0) v = (float)mt * 0.001953125f;  // m * 2^-9 (subnormal: 2^-6 * m/8)
  else v = __uint_as_float(((e + 120u) << 23) | (mt << 20));
  return s ? -v : v;
}

}  // namespace finger
