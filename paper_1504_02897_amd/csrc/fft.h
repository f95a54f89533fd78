// Batched FFT passes used by the NUFFT (fine grid) and by the GPE kernels (unpadded grid).
#pragma once

#include "ddi_internal.h"

namespace ddi {

// Last-axis pass modes: R2C_PAD reads a real compact grid times the deconvolution
// factors into the active half of each oversampled line; C2C is a plain complex
// transform; C2R_TRUNC keeps the active modes, applies the deconvolution factors
// and writes the real part to a compact grid.
enum ContigMode { R2C_PAD = 0, C2C = 1, C2R_TRUNC = 2, C2R_ADD = 3,   // C2R_ADD: as C2R_TRUNC, added to the output
                  C2C_GF_RES = 4, C2C_GF_SOLVE = 5, C2C_TS_KIN = 6 };

// Elementwise steps of the gradient flow (Sec. 3.1) folded into the loads of a C2C pass over
// an N0 x N1 x N2 grid (lines along axis 2):
//   C2C_GF_RES:   x = (alpha - B) in, B a real grid (aux);
//   C2C_GF_SOLVE: x = (rhs0 / dt + in) / ((1/dt + alpha + |mu|^2 / 2) prod(N)), rhs0 complex (aux),
//                 mu_i = pi p_i / L_i with p_i the signed mode of index i on axis i (axis 0 counted
//                 only when N0 > 1);
//   C2C_TS_KIN:   x = in exp(-i qdt |mu|^2) / prod(N), the kinetic sub-step of the time splitting
//                 (Sec. 4.1, Eq. tssp2).
// alpha is read from device memory (the flow's stabilisation, computed on the device).
struct GfLoad {
  const void* aux = nullptr;
  const double* alpha = nullptr;
  double inv_dt = 0.0, inv_ntot = 0.0, qdt = 0.0;
  double L[3] = {1.0, 1.0, 1.0};    // half-lengths L_i of the box
  int n[3] = {1, 1, 1};
};

// The multiplier of the split's short-range part (Eq. 3.9) on the zero-padded grid, p = (1 - q) Uhat
// at k_i = m_i dk[i], times scale:
//   3D: (1 - exp(-|k|^2/s^2)) (3 (n.k)(m.k)/|k|^2 - n.m);
//   2D: erf(|k|/s) 3 [(n.k)(m.k) - n3 m3 |k|^2] / (2 |k|), the paper's (x, y) carried on the
//       kernel's axes 0 and 2 (n = (n1, 0, n2), dk[1] unused).
struct SplitSymbol {
  double n[3], m[3];
  double nm;
  double inv_s2;
  double dk[3];
  double scale;
  int dim;            // 3, or 2 for the quasi-2D symbol
  double inv_s;       // 1/s (2D)
  double n3m3;        // n3 m3 (2D)
};

// In-place transforms of length n along axis 0 or 1 of a [d0][d1][d2] complex
// array.  The other non-last axis runs over n_o lines (the compact modes of an
// oversampled axis when o_compact); in_c: only the nc active positions of each
// line are read (the rest taken as zero); out_c: only the nc_out active positions
// are written (exp(SIGN 2 pi i jk/n)).  Only the lines at last-axis positions
// [z0, z0 + nz) (mod d2) are transformed: z0 and nz are multiples of 8, or z0 = 0
// and nz = d2.
template <typename T, int SIGN>
hipError_t launch_strided(int n, Complex<T>* F, int axis, int d0, int d1, int d2, int n_o, int o_compact, int nc,
                          int in_c, int out_c, int nc_out, int z0, int nz, const Complex<T>* tw, hipStream_t s);

// Transforms of length n along the last axis; lines run over the n0 x n1 compact
// grid (R2C_PAD, C2R_TRUNC: mapped into a [d0][d1][n] oversampled array) or over
// d0 x d1 = n0 x n1 directly (C2C).  Only the positions [z0, z0 + nz) (mod n) of
// the complex lines are written (R2C_PAD) or read, the rest taken as zero
// (C2R_TRUNC, C2C); z0 = 0 and nz = n: the whole line.
template <typename T, int SIGN, int MODE>
hipError_t launch_contig(int n, const void* in, void* out, int n0, int n1, int d0, int d1, int nc2, int z0, int nz,
                         const double* D0, const double* D1, const double* D2, const Complex<T>* tw,
                         hipStream_t s, const GfLoad& gl = GfLoad{});

// Lines along axis 0 of the [d0][d1][d2] padded spectrum of a real field, at last-axis
// positions [0, nz) (the modes m2 in [0, nz), nz <= d2/2): transform the nc active inputs
// with exp(-2 pi i jk/n), multiply by the split symbol times 1 at m2 = 0 and 2 above (the
// half set; the partner modes are the complex conjugates), zero on the Nyquist planes
// m_i = -d_i/2, transform back with exp(+2 pi i jk/n) and write the nc active outputs.
// A 2D spectrum [n][d2] is passed as d1 = 1 (its lines along axis 0 are then the paper's x).
template <typename T>
hipError_t launch_symbol(int n, Complex<T>* F, int d1, int d2, int nc, int nz, const SplitSymbol& sp,
                         const Complex<T>* tw, hipStream_t s);

inline int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

// Slot of the twiddle table of an FFT length: n = 2^a (a <= 10) at slot a, n = 3 * 2^a
// (a <= 8) at slot 11 + a.
inline int tw_slot(int n) { return n % 3 == 0 ? 11 + ilog2(n / 3) : ilog2(n); }

}  // namespace ddi
