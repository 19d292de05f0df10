// Host check of the compile-time register DFTs and the two-pass split:
// every size against a naive FP64 DFT.  Prints "<N> <max relative error>".
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2601_05418_amd/csrc/fft2.h"

static std::mt19937 rng(7);

template <int R>
static double ref_err(const std::vector<float2>& in, const std::vector<float2>& out) {
  double err = 0, mag = 0;
  for (int k = 0; k < R; ++k) {
    double sr = 0, si = 0;
    for (int n = 0; n < R; ++n) {
      const double a = -2 * M_PI * (double)((long)n * k % R) / R;
      sr += in[n].x * std::cos(a) - in[n].y * std::sin(a);
      si += in[n].x * std::sin(a) + in[n].y * std::cos(a);
    }
    err = std::max(err, std::hypot(out[k].x - sr, out[k].y - si));
    mag = std::max(mag, std::hypot(sr, si));
  }
  return err / mag;
}

template <int R>
static void check_reg() {
  std::normal_distribution<float> nd;
  std::vector<float2> in(R), v(R);
  for (auto& x : in) x = make_float2(nd(rng), nd(rng));
  v = in;
  gpjc::rdft<R>(v.data());
  std::printf("rdft %d %.3e\n", R, ref_err<R>(in, v));
}

// Two-pass transform of one line as the kernels do it (no LDS: plain arrays).
template <int N>
static void check_split() {
  using S = gpjc::Split<N>;
  std::normal_distribution<float> nd;
  std::vector<float2> in(N), out(N), a(N);
  for (auto& x : in) x = make_float2(nd(rng), nd(rng));
  std::vector<float2> tw(N);
  for (int m = 0; m < N; ++m) tw[m] = make_float2((float)std::cos(-2 * M_PI * m / N), (float)std::sin(-2 * M_PI * m / N));
  for (int i2 = 0; i2 < S::N2; ++i2) {
    float2 v[S::N1];
    for (int i1 = 0; i1 < S::N1; ++i1) v[i1] = in[i2 + S::N2 * i1];
    gpjc::rdft<S::N1>(v);
    for (int k1 = 0; k1 < S::N1; ++k1) a[i2 * S::N1 + k1] = gpjc::cmul(v[k1], tw[(i2 * k1) % N]);
  }
  for (int k1 = 0; k1 < S::N1; ++k1) {
    float2 w[S::N2];
    for (int i2 = 0; i2 < S::N2; ++i2) w[i2] = a[i2 * S::N1 + k1];
    gpjc::rdft<S::N2>(w);
    for (int k2 = 0; k2 < S::N2; ++k2) out[k1 + S::N1 * k2] = w[k2];
  }
  std::printf("split %d %.3e\n", N, ref_err<N>(in, out));
}

int main() {
  check_reg<2>(); check_reg<3>(); check_reg<4>(); check_reg<5>(); check_reg<6>(); check_reg<7>(); check_reg<8>();
  check_reg<10>(); check_reg<12>(); check_reg<14>(); check_reg<16>(); check_reg<20>(); check_reg<24>();
  check_reg<28>(); check_reg<32>();
  check_reg<11>(); check_reg<13>(); check_reg<15>(); check_reg<18>(); check_reg<22>(); check_reg<23>();
  check_reg<30>(); check_reg<31>();
  check_split<16>(); check_split<32>(); check_split<48>(); check_split<64>(); check_split<80>(); check_split<96>();
  check_split<112>(); check_split<128>(); check_split<160>(); check_split<192>(); check_split<224>();
  check_split<256>(); check_split<320>(); check_split<384>(); check_split<448>(); check_split<512>();
  check_split<180>(); check_split<230>(); check_split<280>();
  return 0;
}
