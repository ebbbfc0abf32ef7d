// Host build of the radix butterflies of fft_lds.hpp, checked against a direct DFT in double.
// Prints one line per radix and direction: "R INV max_abs_error".
#include <cmath>
#include <cstdio>
#include <random>

#include "fft_lds.hpp"

using namespace aahrt;

template <int R, bool INV>
static double check(std::mt19937& rng) {
  std::normal_distribution<float> nd(0.f, 1.f);
  double worst = 0.0;
  for (int trial = 0; trial < 20; ++trial) {
    float2 v[R], x[R];
    for (int i = 0; i < R; ++i) x[i] = v[i] = make_float2(nd(rng), nd(rng));
    Dft<R, INV>::run(v);
    for (int k = 0; k < R; ++k) {
      double re = 0.0, im = 0.0;
      for (int n = 0; n < R; ++n) {
        const double a = (INV ? 2.0 : -2.0) * M_PI * (double)((n * k) % R) / R;
        re += x[n].x * std::cos(a) - x[n].y * std::sin(a);
        im += x[n].x * std::sin(a) + x[n].y * std::cos(a);
      }
      worst = std::fmax(worst, std::fabs(re - v[k].x) + std::fabs(im - v[k].y));
    }
  }
  return worst;
}

template <int R>
static void both(std::mt19937& rng) {
  std::printf("%d 0 %.3e\n", R, check<R, false>(rng));
  std::printf("%d 1 %.3e\n", R, check<R, true>(rng));
}

int main() {
  std::mt19937 rng(2505);
  both<2>(rng);
  both<3>(rng);
  both<4>(rng);
  both<5>(rng);
  both<8>(rng);
  both<9>(rng);
  both<15>(rng);
  both<16>(rng);
  return 0;
}
