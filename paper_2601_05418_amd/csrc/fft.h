// Mixed-radix Stockham FFT over batches of lines held in LDS.
//
// All transforms of the hybrid-space Wave operator have image-sized lengths:
// the phase-encode axis (Ny) directly, and the oversampled readout (Nt = os Nx)
// through os length-Nx transforms of pre-twiddled inputs (the zero padding
// prunes every other input).  Lengths are compile-time constants of the form
// 2^a 3^b 5^c 7^d, so every index division in a pass folds to a multiply.
//
// Only the forward transform X[k] = sum_n x[n] exp(-2 pi i n k / N)
// (unnormalised) is provided; callers take the inverse as
// conj(FFT(conj(x))) by conjugating at load and store.
//
// The Stockham autosort formulation (Govindaraju et al., "High performance
// discrete Fourier transforms on graphics processors", SC 2008): pass with
// radix R after a product NS of earlier radices reads butterfly j's inputs at
// stride N/R, twiddles them by w_{NS R}^{(j mod NS) r}, takes an R-point DFT
// and writes the outputs at stride NS from (j / NS) NS R + (j mod NS).  The
// final pass leaves the spectrum in natural order.
#pragma once
#include <hip/hip_runtime.h>

namespace gpjc {

__host__ __device__ inline float2 cmul(float2 a, float2 b) {
  return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a * conj(b)
__host__ __device__ inline float2 cmulc(float2 a, float2 b) {
  return make_float2(a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y);
}
__host__ __device__ inline float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__host__ __device__ inline float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__host__ __device__ inline float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__host__ __device__ inline float2 cconj(float2 a) { return make_float2(a.x, -a.y); }
// -i * a
__host__ __device__ inline float2 cmul_mi(float2 a) { return make_float2(a.y, -a.x); }

// Transform lengths the readout and phase-encode kernels are instantiated for
// (with 180, 230 and 280: the matrix sizes of the paper's scans).
#define GPJC_FFT_SIZES(X)                                                                                 \
  X(16) X(32) X(48) X(64) X(80) X(96) X(112) X(128) X(160) X(180) X(192) X(224) X(230) X(256) X(280) X(320) \
      X(384) X(448) X(512)

// Largest odd prime factor the DFT kernels take.
constexpr int kMaxOddRadix = 31;
// ---------------------------------------------------------------------------
// Compile-time sine / cosine of 2 pi m / n (double, |error| ~ 1e-16).
// ---------------------------------------------------------------------------
constexpr double kTwoPi = 6.283185307179586476925286766559;
constexpr double kHalfPi = 1.5707963267948966192313216916398;
constexpr double kPi = 3.1415926535897932384626433832795;

// Taylor series on |x| <= pi / 4.
constexpr double sin_series(double x) {
  double term = x, sum = x;
  for (int k = 1; k < 12; ++k) {
    term *= -x * x / ((2.0 * k) * (2.0 * k + 1.0));
    sum += term;
  }
  return sum;
}
constexpr double cos_series(double x) {
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 12; ++k) {
    term *= -x * x / ((2.0 * k - 1.0) * (2.0 * k));
    sum += term;
  }
  return sum;
}
// sin and cos of 2 pi m / n for integers m, n > 0, reduced by quadrant with
// exact integer arithmetic (4 m mod n picks the quadrant).
constexpr double sin2pi(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  const long q = (4 * m) / n;                          // quadrant 0..3
  const double r = kTwoPi * (double)(4 * m - q * n) / (4.0 * (double)n);  // in [0, pi/2)
  const double s = r <= kHalfPi / 2 ? sin_series(r) : cos_series(kHalfPi - r);
  const double c = r <= kHalfPi / 2 ? cos_series(r) : sin_series(kHalfPi - r);
  return q == 0 ? s : q == 1 ? c : q == 2 ? -s : -c;
}
constexpr double cos2pi(long m, long n) {
  m %= n;
  if (m < 0) m += n;
  const long q = (4 * m) / n;
  const double r = kTwoPi * (double)(4 * m - q * n) / (4.0 * (double)n);
  const double s = r <= kHalfPi / 2 ? sin_series(r) : cos_series(kHalfPi - r);
  const double c = r <= kHalfPi / 2 ? cos_series(r) : sin_series(kHalfPi - r);
  return q == 0 ? c : q == 1 ? -s : q == 2 ? -c : s;
}


// ---------------------------------------------------------------------------
// Compile-time radix plan: greedy 8, 4, 2, then 7, 5, 3, then odd primes up to 31.
// ---------------------------------------------------------------------------
constexpr int next_radix(int n) {
  if (n % 8 == 0) return 8;
  if (n % 4 == 0) return 4;
  if (n % 2 == 0) return 2;
  if (n % 7 == 0) return 7;
  if (n % 5 == 0) return 5;
  if (n % 3 == 0) return 3;
  for (int p = 11; p <= kMaxOddRadix; p += 2)
    if (n % p == 0) return p;  // the smallest remaining factor is prime
  return -1;
}
constexpr int radix_count(int n) {
  int c = 0;
  while (n > 1) {
    const int r = next_radix(n);
    if (r < 0) return -1;
    n /= r;
    ++c;
  }
  return c;
}
constexpr int radix_at(int n, int idx) {
  int i = 0;
  while (n > 1) {
    const int r = next_radix(n);
    if (i == idx) return r;
    n /= r;
    ++i;
  }
  return 1;
}
constexpr bool fft_length_ok(int n) { return n >= 2 && radix_count(n) > 0; }

// ---------------------------------------------------------------------------
// Small forward DFTs in registers.
// ---------------------------------------------------------------------------
// cos / sin of 2 pi m / R, m = 1 .. (R-1)/2, for an odd R (compile-time series,
// rounded once).
template <int R>
struct OddRoots {
  struct Tab {
    float c[(R - 1) / 2], s[(R - 1) / 2];
  };
  static constexpr Tab make() {
    Tab t{};
    for (int m = 1; m <= (R - 1) / 2; ++m) {
      t.c[m - 1] = (float)cos2pi(m, R);
      t.s[m - 1] = (float)sin2pi(m, R);
    }
    return t;
  }
  static constexpr Tab tab = make();
};

template <int R>
__host__ __device__ inline void dft_fwd(float2* v) {
  if constexpr (R == 2) {
    const float2 a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if constexpr (R == 4) {
    const float2 s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
    const float2 s13 = cadd(v[1], v[3]), d13 = cmul_mi(csub(v[1], v[3]));
    v[0] = cadd(s02, s13);
    v[2] = csub(s02, s13);
    v[1] = cadd(d02, d13);
    v[3] = csub(d02, d13);
  } else if constexpr (R == 8) {
    float2 e[4] = {v[0], v[2], v[4], v[6]};
    float2 o[4] = {v[1], v[3], v[5], v[7]};
    dft_fwd<4>(e);
    dft_fwd<4>(o);
    constexpr float h = 0.70710678118654752440f;
    // o[k] *= w8^k, w8 = exp(-i pi / 4)
    o[1] = make_float2(h * (o[1].x + o[1].y), h * (o[1].y - o[1].x));
    o[2] = cmul_mi(o[2]);
    o[3] = make_float2(h * (o[3].y - o[3].x), -h * (o[3].x + o[3].y));
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      v[k] = cadd(e[k], o[k]);
      v[k + 4] = csub(e[k], o[k]);
    }
  } else {
    // Odd R: pair r with R - r.  out[k] = a_k - i b_k, out[R-k] = a_k + i b_k with
    // a_k = v0 + sum_r (v_r + v_{R-r}) cos(2 pi r k / R),
    // b_k = sum_r (v_r - v_{R-r}) sin(2 pi r k / R).
    constexpr int H = (R - 1) / 2;
    float2 sp[H], dm[H];
    float2 dc = v[0];
#pragma unroll
    for (int r = 1; r <= H; ++r) {
      sp[r - 1] = cadd(v[r], v[R - r]);
      dm[r - 1] = csub(v[r], v[R - r]);
      dc = cadd(dc, sp[r - 1]);
    }
    float2 out[R];
    out[0] = dc;
#pragma unroll
    for (int k = 1; k <= H; ++k) {
      float2 a = v[0], b = make_float2(0.f, 0.f);
#pragma unroll
      for (int r = 1; r <= H; ++r) {
        const int m = (r * k) % R;  // angle index in [0, R)
        const int mm = m <= H ? m : R - m;
        const float cs = OddRoots<R>::tab.c[mm - 1];
        const float sn = m <= H ? OddRoots<R>::tab.s[mm - 1] : -OddRoots<R>::tab.s[mm - 1];
        a = cadd(a, cscale(sp[r - 1], cs));
        b = cadd(b, cscale(dm[r - 1], sn));
      }
      out[k] = cadd(a, cmul_mi(b));
      out[R - k] = csub(a, cmul_mi(b));
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = out[k];
  }
}

// LDS position of element e of a line: one padding slot after every 8
// elements, so the stride-R stores of a Stockham pass and the stride-os
// gathers of the readout stages spread over the banks.
__host__ __device__ constexpr int fpad(int e) { return e + (e >> 3); }
// Line stride (in complex elements) of a padded line of length N; odd, so
// lines accessed at equal offsets also land on different banks.
__host__ __device__ constexpr int fline(int n) { return n + (n >> 3) + 1; }

// One Stockham pass over `nlines` padded lines of length N (line l starts at
// l*stride).  tw[m] = exp(-2 pi i m / N), m in [0, N).
template <int N, int NS, int R>
__host__ __device__ inline void stockham_pass(const float2* __restrict__ in, float2* __restrict__ out,
                                              const float2* __restrict__ tw, int nlines, int stride,
                                              int tid, int nthr) {
  constexpr int NB = N / R;
  constexpr int TWS = N / (NS * R);
  const int total = nlines * NB;
  for (int b = tid; b < total; b += nthr) {
    const int line = b / NB;
    const int j = b - line * NB;
    const float2* src = in + line * stride;
    float2* dst = out + line * stride;
    float2 v[R];
#pragma unroll
    for (int r = 0; r < R; ++r) v[r] = src[fpad(j + r * NB)];
    if constexpr (NS > 1) {
      const int k = j % NS;
#pragma unroll
      for (int r = 1; r < R; ++r) v[r] = cmul(v[r], tw[k * r * TWS]);
    }
    dft_fwd<R>(v);
    const int idx = (j / NS) * NS * R + (j % NS);
#pragma unroll
    for (int r = 0; r < R; ++r) dst[fpad(idx + r * NS)] = v[r];
  }
}

// Forward FFT of `nlines` padded lines (element e of line l at
// l*stride + fpad(e)); data starts in `a`, `b` is scratch of the same
// extent.  `sync` separates passes (a workgroup barrier on the device).
// Returns the buffer holding the result.
template <int N, int P = 0, int NS = 1, class Sync>
__host__ __device__ inline float2* fft_lines(float2* a, float2* b, const float2* tw, int nlines, int stride,
                                             int tid, int nthr, Sync sync) {
  static_assert(fft_length_ok(N), "unsupported FFT length");
  if constexpr (P == radix_count(N)) {
    return a;
  } else {
    constexpr int R = radix_at(N, P);
    stockham_pass<N, NS, R>(a, b, tw, nlines, stride, tid, nthr);
    sync();
    return fft_lines<N, P + 1, NS * R>(b, a, tw, nlines, stride, tid, nthr, sync);
  }
}

}  // namespace gpjc
