// Device helpers shared by the operator sources.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

#include "plan.h"

namespace gpjc {

typedef float floatx4 __attribute__((ext_vector_type(4)));

// Reduced-precision storage of complex values (round to nearest even).
__device__ inline uint32_t f32_to_bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7fc0u;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}
__device__ inline float bf16_bits_to_f32(uint32_t h) { return __uint_as_float(h << 16); }
__device__ inline uint32_t f32_to_f16_bits(float f) {
  _Float16 h = (_Float16)f;
  return (uint32_t)__builtin_bit_cast(uint16_t, h);
}
__device__ inline float f16_bits_to_f32(uint32_t h) { return (float)__builtin_bit_cast(_Float16, (uint16_t)h); }

template <Store ST>
__device__ inline uint32_t to_bits16(float f) {
  if constexpr (ST == Store::BF16) return f32_to_bf16_bits(f);
  else return f32_to_f16_bits(f);
}

template <Store ST>
__device__ inline void store_c(void* base, size_t i, float2 v) {
  if constexpr (ST == Store::F32) {
    reinterpret_cast<float2*>(base)[i] = v;
  } else {
    reinterpret_cast<uint32_t*>(base)[i] = to_bits16<ST>(v.x) | (to_bits16<ST>(v.y) << 16);
  }
}
template <Store ST>
__device__ inline float from_bits16(uint32_t h) {
  if constexpr (ST == Store::BF16) return bf16_bits_to_f32(h);
  else return f16_bits_to_f32(h);
}

// Element k of Z^T row `row` (rows of kp complex values).  FP32 as is; the
// 16-bit types as a hi + lo pair, hi = rn(v) and lo = rn(v - hi), in a row of
// 2 kp pairs: hi at k, lo at kp + k.
template <Store ST>
__device__ inline void store_zt(void* Zt, size_t row, int kp, int k, float2 v) {
  if constexpr (ST == Store::F32) {
    reinterpret_cast<float2*>(Zt)[row * kp + k] = v;
  } else {
    const uint32_t hr = to_bits16<ST>(v.x), hi = to_bits16<ST>(v.y);
    const float lr = v.x - from_bits16<ST>(hr), li = v.y - from_bits16<ST>(hi);
    uint32_t* z = reinterpret_cast<uint32_t*>(Zt) + row * 2 * kp;
    z[k] = hr | (hi << 16);
    z[kp + k] = to_bits16<ST>(lr) | (to_bits16<ST>(li) << 16);
  }
}

template <Store ST>
__device__ inline float2 load_c(const void* base, size_t i) {
  if constexpr (ST == Store::F32) {
    return reinterpret_cast<const float2*>(base)[i];
  } else {
    const uint32_t w = reinterpret_cast<const uint32_t*>(base)[i];
    if constexpr (ST == Store::BF16) return make_float2(bf16_bits_to_f32(w & 0xffffu), bf16_bits_to_f32(w >> 16));
    else return make_float2(f16_bits_to_f32(w & 0xffffu), f16_bits_to_f32(w >> 16));
  }
}

// Sum over the nchunk partial images (stride n) at element i, in a fixed
// order: partial 0, then groups of eight partials, each loaded together (a
// group past nchunk reads partial nchunk - 1 and replaces it by zero, so no
// load sits behind a branch) and added as a balanced tree.
__device__ inline float2 sum_chunks(const float2* __restrict__ part, int nchunk, size_t n, size_t i) {
  auto add = [](float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); };
  float2 v = part[i];
  for (int c = 1; c < nchunk; c += 8) {
    float2 a[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const float2 x = part[(size_t)min(c + k, nchunk - 1) * n + i];
      a[k] = c + k < nchunk ? x : make_float2(0.f, 0.f);
    }
    v = add(v, add(add(add(a[0], a[1]), add(a[2], a[3])), add(add(a[4], a[5]), add(a[6], a[7]))));
  }
  return v;
}

// Work-group id remapped so that consecutive logical tiles share one XCD
// (work-groups are dealt round-robin over the 8 XCDs, each with its own L2).
__device__ inline int xcd_logical(int linear, int total) {
  const int per = total / 8, rem = total % 8;
  const int xcd = linear % 8, slot = linear / 8;
  return xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
}

}  // namespace gpjc
