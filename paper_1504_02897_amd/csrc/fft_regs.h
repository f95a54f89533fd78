// In-register DFTs of the FFT passes (host and device: the host build is checked on the CPU).
#pragma once

#include "ddi_internal.h"

namespace ddi {

template <typename T>
using C = Complex<T>;

template <typename T>
__host__ __device__ __forceinline__ C<T> cmul(C<T> a, C<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__host__ __device__ __forceinline__ C<T> cadd(C<T> a, C<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__host__ __device__ __forceinline__ C<T> csub(C<T> a, C<T> b) { return {a.re - b.re, a.im - b.im}; }

// cos(2 pi j / 16) from the first-quadrant values
__host__ __device__ constexpr double cos_16(int j) {
  j &= 15;
  const double q[5] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173, 0.0};
  return j <= 4 ? q[j] : (j <= 8 ? -q[8 - j] : (j <= 12 ? -q[j - 8] : q[16 - j]));
}

// ------------------------------------------------------------------ in-register DFT of size R <= 16
// out[k] = sum_r v[r] exp(SIGN 2 pi i r k / R), iterative radix-2 decimation in time.
template <int R>
__host__ __device__ __forceinline__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) { r = (r << 1) | (i & 1); i >>= 1; }
  return r;
}

template <typename T, int R, int SIGN>
__host__ __device__ __forceinline__ void dft_regs(C<T>* v) {
#pragma unroll
  for (int i = 0; i < R; ++i) {
    const int j = bitrev<R>(i);
    if (j > i) { C<T> t = v[i]; v[i] = v[j]; v[j] = t; }
  }
#pragma unroll
  for (int m = 2; m <= R; m <<= 1) {
#pragma unroll
    for (int k = 0; k < R; k += m) {
#pragma unroll
      for (int j = 0; j < m / 2; ++j) {
        const int idx = j * (16 / m);      // angle index in units of 2 pi / 16, in [0, 8)
        C<T> b = v[k + j + m / 2];
        C<T> t;
        if (idx == 0) {
          t = b;
        } else if (idx == 4) {             // exp(SIGN i pi/2) = SIGN i
          t = SIGN > 0 ? C<T>{-b.im, b.re} : C<T>{b.im, -b.re};
        } else {
          const T c = static_cast<T>(cos_16(idx));
          const T s = static_cast<T>(SIGN * cos_16(idx - 4));
          t = {b.re * c - b.im * s, b.re * s + b.im * c};
        }
        C<T> a = v[k + j];
        v[k + j] = cadd(a, t);
        v[k + j + m / 2] = csub(a, t);
      }
    }
  }
}

// cos(2 pi j / 24) from the values at multiples of 15 degrees
__host__ __device__ constexpr double cos_24(int j) {
  j = ((j % 24) + 24) % 24;
  const double q[7] = {1.0, 0.96592582628906828675, 0.86602540378443864676, 0.70710678118654752440, 0.5,
                       0.25881904510252076235, 0.0};
  return j <= 6 ? q[j] : (j <= 12 ? -q[12 - j] : (j <= 18 ? -q[j - 12] : q[24 - j]));
}

// out[k] = sum_r v[r] exp(SIGN 2 pi i r k / R) for R = 3 M (M = 4 or 8), in place, natural order.
// With r = M r1 + r2 and k = k1 + 3 k2: a 3-point DFT over r1 for each r2, the twiddles
// exp(SIGN 2 pi i r2 k1 / R), then an M-point DFT over r2 for each k1.
template <typename T, int M, int SIGN>
__host__ __device__ __forceinline__ void dft_regs3(C<T>* v) {
  constexpr int R = 3 * M;
  static_assert(24 % R == 0, "3 M must divide 24");
  const T h = static_cast<T>(0.86602540378443864676);       // sqrt(3)/2
  C<T> y[3][M];
#pragma unroll
  for (int r2 = 0; r2 < M; ++r2) {
    const C<T> a = v[r2], b = v[M + r2], c = v[2 * M + r2];
    const C<T> t1 = cadd(b, c), t2 = csub(b, c);
    const C<T> m = {a.re - t1.re / 2, a.im - t1.im / 2};
    // SIGN i sqrt(3)/2 (b - c)
    const C<T> j = SIGN > 0 ? C<T>{-h * t2.im, h * t2.re} : C<T>{h * t2.im, -h * t2.re};
    y[0][r2] = cadd(a, t1);
    y[1][r2] = cadd(m, j);
    y[2][r2] = csub(m, j);
  }
#pragma unroll
  for (int k1 = 1; k1 < 3; ++k1) {
#pragma unroll
    for (int r2 = 1; r2 < M; ++r2) {
      const int idx = r2 * k1 * (24 / R);             // angle in units of 2 pi / 24
      const T c = static_cast<T>(cos_24(idx));
      const T sn = static_cast<T>(SIGN * cos_24(idx - 6));
      const C<T> b = y[k1][r2];
      y[k1][r2] = {b.re * c - b.im * sn, b.re * sn + b.im * c};
    }
  }
#pragma unroll
  for (int k1 = 0; k1 < 3; ++k1) {
    dft_regs<T, M, SIGN>(y[k1]);
#pragma unroll
    for (int k2 = 0; k2 < M; ++k2) v[k1 + 3 * k2] = y[k1][k2];
  }
}

// In-register DFT of any radix a plan uses: powers of two, or three times 4 or 8.
template <typename T, int R, int SIGN>
__host__ __device__ __forceinline__ void dft_any(C<T>* v) {
  if constexpr (R % 3 == 0) dft_regs3<T, R / 3, SIGN>(v);
  else dft_regs<T, R, SIGN>(v);
}

}  // namespace ddi
