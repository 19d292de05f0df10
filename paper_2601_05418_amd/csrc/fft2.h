// Register-resident DFTs and the two-pass LDS FFT built from them.
//
// A length N = N1 * N2 transform splits (Cooley-Tukey) as
//   X[k1 + N1 k2] = sum_{i2} w_N2^{i2 k2} [ w_N^{i2 k1} sum_{i1} w_N1^{i1 k1} x[i2 + N2 i1] ],
// so one thread computes an N1-point DFT of a stride-N2 subsequence in
// registers, applies the twiddles w_N^{i2 k1}, and after an exchange through
// LDS another thread computes an N2-point DFT over i2.  Small DFTs are
// themselves split the same way, entirely at compile time: every index and
// every root of unity is a constant, so a DFT costs only its flops.
//
// Roots of unity are evaluated at compile time in double precision from
// their Taylor series (own implementation below) and rounded once to float.
#pragma once
#include <hip/hip_runtime.h>

#include "fft.h"

namespace gpjc {

// exp(-2 pi i m / n) as float2, for constant m, n.
template <long M, long N>
__host__ __device__ constexpr float2 root() {
  return float2{(float)cos2pi(M, N), (float)(-sin2pi(M, N))};
}

// v * exp(-2 pi i M / N) with the trivial angles resolved at compile time.
template <long M, long N>
__host__ __device__ inline float2 twiddle(float2 v) {
  constexpr long m = ((M % N) + N) % N;
  if constexpr (m == 0) {
    return v;
  } else if constexpr (4 * m == N) {  // -i
    return make_float2(v.y, -v.x);
  } else if constexpr (2 * m == N) {  // -1
    return make_float2(-v.x, -v.y);
  } else if constexpr (4 * m == 3 * N) {  // +i
    return make_float2(-v.y, v.x);
  } else {
    constexpr float2 w = root<M, N>();
    return make_float2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
  }
}

// ---------------------------------------------------------------------------
// In-register forward DFT of size R (output in natural order, in place).
// ---------------------------------------------------------------------------
constexpr int first_factor(int r) {
  return (r % 4 == 0 && r != 4 && r != 8) ? 4 : (r % 2 == 0 && r != 2 && r != 4 && r != 8) ? 2
       : (r % 3 == 0 && r != 3) ? 3 : (r % 5 == 0 && r != 5) ? 5 : (r % 7 == 0 && r != 7) ? 7 : r;
}
// Sizes taken by one base DFT: 2, 4, 8, and odd primes up to 31 (the odd form
// of dft_fwd); larger sizes are split by first_factor.
constexpr bool base_dft(int r) {
  return r == 1 || r == 2 || r == 4 || r == 8 || (r % 2 == 1 && r <= kMaxOddRadix && first_factor(r) == r);
}

template <int R>
__host__ __device__ inline void rdft(float2* v);

template <int R, int R1, int R2, int I2 = 0>
__host__ __device__ inline void rdft_cols(float2* v, float2 (&t)[R]) {
  if constexpr (I2 < R2) {
    float2 col[R1];
#pragma unroll
    for (int i1 = 0; i1 < R1; ++i1) col[i1] = v[I2 + R2 * i1];
    rdft<R1>(col);
    [&]<int... K1>(std::integer_sequence<int, K1...>) {
      ((t[I2 * R1 + K1] = twiddle<(long)I2 * K1, R>(col[K1])), ...);
    }(std::make_integer_sequence<int, R1>{});
    rdft_cols<R, R1, R2, I2 + 1>(v, t);
  }
}

template <int R>
__host__ __device__ inline void rdft(float2* v) {
  if constexpr (R == 1) {
    return;
  } else if constexpr (base_dft(R)) {
    dft_fwd<R>(v);
  } else {
    constexpr int R1 = first_factor(R);
    constexpr int R2 = R / R1;
    static_assert(R1 > 1 && R1 * R2 == R, "unsupported register DFT size");
    float2 t[R];  // t[i2 * R1 + k1]
    rdft_cols<R, R1, R2>(v, t);
#pragma unroll
    for (int k1 = 0; k1 < R1; ++k1) {
      float2 row[R2];
#pragma unroll
      for (int i2 = 0; i2 < R2; ++i2) row[i2] = t[i2 * R1 + k1];
      rdft<R2>(row);
#pragma unroll
      for (int k2 = 0; k2 < R2; ++k2) v[k1 + R1 * k2] = row[k2];
    }
  }
}

// ---------------------------------------------------------------------------
// Two-pass split of the line lengths the library builds: N = N1 * N2 with
// N1 the first pass (16 where possible) and N2 <= 32.
// ---------------------------------------------------------------------------
// N1 is 16, 8 or 4 where that leaves N2 <= 32; otherwise the largest divisor
// N1 <= 16 with 1 < N2 <= 32 whose factors the register DFTs take (1: none,
// and the Stockham forms serve the length).
constexpr bool reg_dft_ok(int r) {
  while (r > 1) {
    const int f = first_factor(r);
    if (f > kMaxOddRadix) return false;
    r /= f;
  }
  return true;
}
constexpr int split_n1(int n) {
  const int first = n % 16 == 0 && n / 16 > 1 ? 16 : n % 8 == 0 && n / 8 > 1 ? 8 : n % 4 == 0 ? 4 : 1;
  if (first > 1 && n / first <= 32) return first;
  for (int d = 16; d >= 2; --d)
    if (n % d == 0 && n / d > 1 && n / d <= 32 && reg_dft_ok(d) && reg_dft_ok(n / d)) return d;
  return 1;
}
template <int N>
struct Split {
  static constexpr int N1 = split_n1(N);
  static constexpr int N2 = N / N1;
  static constexpr bool ok = N1 > 1 && N2 > 1 && N2 <= 32;
};

}  // namespace gpjc
