// FP64 complex arithmetic on double2 (re, im), for the calibration and the
// explicit readout matrices.
#pragma once
#include <hip/hip_runtime.h>

namespace gpjc {

__device__ inline double2 zadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 zsub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 zmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__device__ inline double2 zmulc(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
// conj(a) * b
__device__ inline double2 zcmul(double2 a, double2 b) {
  return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}
__device__ inline double2 zscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ inline double2 zconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double zabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ inline double2 z_of(float2 a) { return make_double2(a.x, a.y); }

// exp(-2 pi i m / n) for an integer m reduced exactly into [0, n).
__device__ inline double2 zroot(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  double s, c;
  sincospi(-2.0 * (double)m / (double)n, &s, &c);
  return make_double2(c, s);
}

}  // namespace gpjc
