// Host-only check of the in-register DFTs of the FFT passes (csrc/fft_regs.h): every radix the
// radix plans use (2, 4, 8, 16 and the radix-3 forms 12 = 3 x 4, 24 = 3 x 8), both signs, against
// the direct sum out[k] = sum_r v[r] exp(SIGN 2 pi i r k / R) in long double.  Prints the worst
// error relative to the largest output for each radix and exits non-zero above 1e-15.
#include <cmath>
#include <cstdio>
#include <random>

#include "../../paper_1504_02897_amd/csrc/fft_regs.h"

template <int R, int SIGN>
static double check(std::mt19937_64& rng) {
  std::normal_distribution<double> nd;
  double worst = 0.0;
  for (int trial = 0; trial < 20; ++trial) {
    ddi::Complex<double> v[R];
    long double re[R], im[R];
    for (int r = 0; r < R; ++r) {
      v[r] = {nd(rng), nd(rng)};
      re[r] = v[r].re;
      im[r] = v[r].im;
    }
    ddi::dft_any<double, R, SIGN>(v);
    long double big = 0.0L, err = 0.0L;
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int k = 0; k < R; ++k) {
      long double sr = 0.0L, si = 0.0L;
      for (int r = 0; r < R; ++r) {
        const long double a = SIGN * 2.0L * pi * ((r * k) % R) / R;
        sr += re[r] * cosl(a) - im[r] * sinl(a);
        si += re[r] * sinl(a) + im[r] * cosl(a);
      }
      big = fmaxl(big, hypotl(sr, si));
      err = fmaxl(err, hypotl(v[k].re - sr, v[k].im - si));
    }
    worst = fmax(worst, static_cast<double>(err / big));
  }
  std::printf("R %2d sign %+d: %.3e\n", R, SIGN, worst);
  return worst;
}

int main() {
  std::mt19937_64 rng(7);
  double w = 0.0;
  w = fmax(w, check<2, -1>(rng));
  w = fmax(w, check<4, -1>(rng));
  w = fmax(w, check<8, 1>(rng));
  w = fmax(w, check<16, -1>(rng));
  w = fmax(w, check<12, -1>(rng));
  w = fmax(w, check<12, 1>(rng));
  w = fmax(w, check<24, -1>(rng));
  w = fmax(w, check<24, 1>(rng));
  return w < 1e-15 ? 0 : 1;
}
