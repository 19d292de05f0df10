// Runs the library's Stockham FFT core on the host (one "thread", passes in
// sequence) and compares every supported length with a naive FP64 DFT.
// Prints "<N> <max relative error>" per length.
#include <cmath>
#include <cstdio>
#include <random>
#include <vector>

#include "../../paper_2601_05418_amd/csrc/fft.h"

template <int N>
static double check(std::mt19937& rng) {
  const int nl = 3;
  const int ls = gpjc::fline(N);
  std::normal_distribution<float> nd;
  std::vector<float2> a(nl * ls), b(nl * ls), tw(N), in(nl * N);
  for (int m = 0; m < N; ++m) tw[m] = make_float2((float)std::cos(-2 * M_PI * m / N), (float)std::sin(-2 * M_PI * m / N));
  for (auto& v : in) v = make_float2(nd(rng), nd(rng));
  for (int l = 0; l < nl; ++l)
    for (int n = 0; n < N; ++n) a[l * ls + gpjc::fpad(n)] = in[l * N + n];
  float2* res_buf = gpjc::fft_lines<N>(a.data(), b.data(), tw.data(), nl, ls, 0, 1, [] {});
  std::vector<float2> res(nl * N);
  for (int l = 0; l < nl; ++l)
    for (int n = 0; n < N; ++n) res[l * N + n] = res_buf[l * ls + gpjc::fpad(n)];
  double err = 0, ref = 0;
  for (int l = 0; l < nl; ++l)
    for (int k = 0; k < N; ++k) {
      double sr = 0, si = 0;
      for (int n = 0; n < N; ++n) {
        const double ang = -2 * M_PI * (double)((long)n * k % N) / N;
        sr += in[l * N + n].x * std::cos(ang) - in[l * N + n].y * std::sin(ang);
        si += in[l * N + n].x * std::sin(ang) + in[l * N + n].y * std::cos(ang);
      }
      const float2 o = res[l * N + k];
      err = std::fmax(err, std::hypot(o.x - sr, o.y - si));
      ref = std::fmax(ref, std::hypot(sr, si));
    }
  std::printf("%d %.3e\n", N, err / ref);
  return err / ref;
}

int main() {
  std::mt19937 rng(5);
  double worst = 0;
  worst = std::fmax(worst, check<2>(rng));
  worst = std::fmax(worst, check<6>(rng));
  worst = std::fmax(worst, check<8>(rng));
  worst = std::fmax(worst, check<10>(rng));
  worst = std::fmax(worst, check<12>(rng));
  worst = std::fmax(worst, check<14>(rng));
  worst = std::fmax(worst, check<16>(rng));
  worst = std::fmax(worst, check<48>(rng));
  worst = std::fmax(worst, check<64>(rng));
  worst = std::fmax(worst, check<80>(rng));
  worst = std::fmax(worst, check<96>(rng));
  worst = std::fmax(worst, check<105>(rng));
  worst = std::fmax(worst, check<112>(rng));
  worst = std::fmax(worst, check<128>(rng));
  worst = std::fmax(worst, check<160>(rng));
  worst = std::fmax(worst, check<192>(rng));
  worst = std::fmax(worst, check<224>(rng));
  worst = std::fmax(worst, check<256>(rng));
  worst = std::fmax(worst, check<384>(rng));
  worst = std::fmax(worst, check<448>(rng));
  worst = std::fmax(worst, check<512>(rng));
  worst = std::fmax(worst, check<180>(rng));
  worst = std::fmax(worst, check<230>(rng));
  worst = std::fmax(worst, check<280>(rng));
  worst = std::fmax(worst, check<1440>(rng));
  worst = std::fmax(worst, check<920>(rng));
  std::printf("worst %.3e\n", worst);
  return worst < 2e-6 ? 0 : 1;
}
