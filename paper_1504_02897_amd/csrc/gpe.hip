// GPE kernels (Sec. 1, Eq. energy; Sec. 3.2 energy split; Sec. 3.1 gradient flow):
// density, spectral kinetic energy and Laplacian through the batched FFT passes,
// energy sums with FP64 block reductions (fixed order, deterministic), the
// gradient dE/dconj(psi), the stabilised backward-Euler Fourier step, and the time-splitting
// step of the dynamics (Sec. 4.1, Eq. tssp2).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "fft.h"

namespace ddi {

template <typename T>
using C = Complex<T>;

// ------------------------------------------------------------------ GPE kernels
// Grid helpers on the unpadded N0 x N1 x N2 grid (N0 = 1 in 2D).
struct GridGeo {
  int N0, N1, N2;
  double L0, L1, L2, h0, h1, h2;
  double g0, g1, g2;          // trap frequencies per internal axis
};

__device__ __forceinline__ void grid_index(int64_t i, const GridGeo& G, int& a, int& b, int& c) {
  c = static_cast<int>(i % G.N2);
  b = static_cast<int>((i / G.N2) % G.N1);
  a = static_cast<int>(i / (static_cast<int64_t>(G.N2) * G.N1));
}

template <typename T>
__device__ __forceinline__ double trap_v(int64_t i, const GridGeo& G, const T* __restrict__ Vext) {
  if (Vext) return static_cast<double>(Vext[i]);
  int a, b, c;
  grid_index(i, G, a, b, c);
  const double x = -G.L0 + a * G.h0, y = -G.L1 + b * G.h1, z = -G.L2 + c * G.h2;
  return 0.5 * (G.g0 * G.g0 * x * x + G.g1 * G.g1 * y * y + G.g2 * G.g2 * z * z);
}

__device__ __forceinline__ double mu2_of(int64_t i, const GridGeo& G) {
  int a, b, c;
  grid_index(i, G, a, b, c);
  const double pa = a < G.N0 / 2 ? a : a - G.N0;
  const double pb = b < G.N1 / 2 ? b : b - G.N1;
  const double pc = c < G.N2 / 2 ? c : c - G.N2;
  const double ma = M_PI * pa / G.L0, mb = M_PI * pb / G.L1, mc = M_PI * pc / G.L2;
  return (G.N0 > 1 ? ma * ma : 0.0) + mb * mb + mc * mc;
}

constexpr int kRedThreads = 256;
#ifndef DDI_GF_FUSED
#define DDI_GF_FUSED 1
#endif
// the gradient-flow step's residual and solve, and the time splitting's kinetic factor, folded
// into the first passes of their transforms
constexpr bool kGfFused = DDI_GF_FUSED != 0;

template <typename T>
__global__ void __launch_bounds__(256) k_density(const C<T>* __restrict__ psi, T* __restrict__ rho, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const C<T> p = psi[i];
    rho[i] = static_cast<T>(static_cast<double>(p.re) * p.re + static_cast<double>(p.im) * p.im);
  }
}

// Block-level FP64 sum of up to 4 values; partial sums to red[block*4 + j].
__device__ __forceinline__ void block_sum4(double v[4], double* __restrict__ red) {
  __shared__ double sh[4][kRedThreads / 64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < 4; ++j) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[j] += __shfl_xor(v[j], off, 64);
    if (lane == 0) sh[j][wv] = v[j];
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double s = 0.0;
    for (int w = 0; w < kRedThreads / 64; ++w) s += sh[threadIdx.x][w];
    red[blockIdx.x * 4 + threadIdx.x] = s;
  }
}

// Combines slot j of the nblocks block partials red[b*4 + j] across one workgroup (a multiple of
// 64 threads, at most kRedThreads), in a fixed order: thread t takes b = t, t + blockDim.x, ...;
// then a butterfly within each wave and the waves in order.  Every thread returns the same value.
template <typename Op>
__device__ __forceinline__ double reduce_partials(const double* __restrict__ red, int nblocks, int j, double init,
                                                  Op op) {
  __shared__ double sh[kRedThreads / 64];
  double v = init;
  for (int b = threadIdx.x; b < nblocks; b += blockDim.x) v = op(v, red[b * 4 + j]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = op(v, __shfl_xor(v, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  double r = init;
  for (int w = 0; w < static_cast<int>(blockDim.x) / 64; ++w) r = op(r, sh[w]);
  __syncthreads();   // sh may be reused by the next call
  return r;
}

struct OpSum { __device__ double operator()(double a, double b) const { return a + b; } };
struct OpMax { __device__ double operator()(double a, double b) const { return fmax(a, b); } };
struct OpMin { __device__ double operator()(double a, double b) const { return fmin(a, b); } };

// sums of mu^2 |psihat|^2 (slot 0); also writes lap = 1/2 mu^2 psihat / prod(N) in place
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_kinetic(C<T>* __restrict__ ph, int64_t n, GridGeo G,
                                                          double inv_ntot, double* __restrict__ red) {
  double v[4] = {0, 0, 0, 0};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double m2 = mu2_of(i, G);
    const C<T> p = ph[i];
    v[0] += m2 * (static_cast<double>(p.re) * p.re + static_cast<double>(p.im) * p.im);
    const double f = 0.5 * m2 * inv_ntot;
    ph[i] = C<T>{static_cast<T>(f * p.re), static_cast<T>(f * p.im)};
  }
  block_sum4(v, red);
}

// sums of V rho (1), rho^2 (2), Phi rho (3)
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_energy_terms(const T* __restrict__ rho, const T* __restrict__ phi,
                                                               const T* __restrict__ Vext, int64_t n, GridGeo G,
                                                               double* __restrict__ red) {
  double v[4] = {0, 0, 0, 0};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double r = rho[i];
    v[1] += trap_v(i, G, Vext) * r;
    v[2] += r * r;
    v[3] += static_cast<double>(phi[i]) * r;
  }
  block_sum4(v, red);
}

// E_out[0..4] from the block partials (fixed order -> deterministic)
__global__ void k_energy_final(const double* __restrict__ red_kin, const double* __restrict__ red_terms, int nblocks,
                               double cell, double inv_ntot, double beta, double lam, double* __restrict__ E) {
  double s[4];
  s[0] = reduce_partials(red_kin, nblocks, 0, 0.0, OpSum());
  for (int j = 1; j < 4; ++j) s[j] = reduce_partials(red_terms, nblocks, j, 0.0, OpSum());
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  E[0] = 0.5 * cell * inv_ntot * s[0];
  E[1] = cell * s[1];
  E[2] = 0.5 * beta * cell * s[2];
  E[3] = 0.5 * lam * cell * s[3];
  E[4] = E[0] + E[1] + E[2] + E[3];
}

template <typename T>
__global__ void __launch_bounds__(256) k_grad(const C<T>* __restrict__ psi, const C<T>* __restrict__ lap,
                                              const T* __restrict__ rho, const T* __restrict__ phi,
                                              const T* __restrict__ phit, const T* __restrict__ Vext, int64_t n,
                                              GridGeo G, double cell, double beta, double lam,
                                              C<T>* __restrict__ grad) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double pot = trap_v(i, G, Vext) + beta * static_cast<double>(rho[i]) +
                       0.5 * lam * (static_cast<double>(phi[i]) + static_cast<double>(phit[i]));
    const C<T> p = psi[i];
    const C<T> l = lap[i];
    grad[i] = C<T>{static_cast<T>(cell * (static_cast<double>(l.re) + pot * p.re)),
                   static_cast<T>(cell * (static_cast<double>(l.im) + pot * p.im))};
  }
}

// B = V + beta rho + lam Phi (into bout), block max/min partials to red[b*4+0/1]
template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_gf_coeff(const T* __restrict__ rho, const T* __restrict__ phi,
                                                           const T* __restrict__ Vext, int64_t n, GridGeo G,
                                                           double beta, double lam, T* __restrict__ bout,
                                                           double* __restrict__ red) {
  double mx = -1e300, mn = 1e300;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double B = trap_v(i, G, Vext) + beta * static_cast<double>(rho[i]) + lam * static_cast<double>(phi[i]);
    bout[i] = static_cast<T>(B);
    mx = fmax(mx, B);
    mn = fmin(mn, B);
  }
  __shared__ double sx[kRedThreads / 64], sn[kRedThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmax(mx, __shfl_xor(mx, off, 64));
    mn = fmin(mn, __shfl_xor(mn, off, 64));
  }
  if ((threadIdx.x & 63) == 0) { sx[threadIdx.x >> 6] = mx; sn[threadIdx.x >> 6] = mn; }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kRedThreads / 64; ++w) { mx = fmax(mx, sx[w]); mn = fmin(mn, sn[w]); }
    mx = fmax(mx, sx[0]);
    mn = fmin(mn, sn[0]);
    red[blockIdx.x * 4 + 0] = mx;
    red[blockIdx.x * 4 + 1] = mn;
  }
}

// scal[0] = alpha = (max + min)/2
__global__ void k_gf_alpha(const double* __restrict__ red, int nblocks, double* __restrict__ scal) {
  const double mx = reduce_partials(red, nblocks, 0, -1e300, OpMax());
  const double mn = reduce_partials(red, nblocks, 1, 1e300, OpMin());
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  scal[0] = 0.5 * (mx + mn);
}

// r = (alpha - B) phi
template <typename T>
__global__ void __launch_bounds__(256) k_gf_residual(const C<T>* phi, const T* __restrict__ B,
                                                     const double* __restrict__ scal, int64_t n, C<T>* r) {
  const double alpha = scal[0];
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double f = alpha - static_cast<double>(B[i]);
    const C<T> p = phi[i];
    r[i] = C<T>{static_cast<T>(f * p.re), static_cast<T>(f * p.im)};
  }
}

// rhat <- (rhs0 + rhat) / (1/dt + alpha + mu^2/2) / prod(N)   (the 1/prod(N) of the inverse FFT folded in)
template <typename T>
__global__ void __launch_bounds__(256) k_gf_solve(C<T>* __restrict__ rh, const C<T>* __restrict__ rhs0,
                                                  const double* __restrict__ scal, int64_t n, GridGeo G, double dt,
                                                  double inv_ntot) {
  const double alpha = scal[0];
  const double inv_dt = 1.0 / dt;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double den = (inv_dt + alpha + 0.5 * mu2_of(i, G)) / inv_ntot;
    const C<T> a = rhs0[i], b = rh[i];
    rh[i] = C<T>{static_cast<T>((inv_dt * a.re + b.re) / den), static_cast<T>((inv_dt * a.im + b.im) / den)};
  }
}

template <typename T>
__global__ void __launch_bounds__(kRedThreads) k_norm2(const C<T>* __restrict__ x, int64_t n,
                                                       double* __restrict__ red) {
  double v[4] = {0, 0, 0, 0};
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const C<T> p = x[i];
    v[0] += static_cast<double>(p.re) * p.re + static_cast<double>(p.im) * p.im;
  }
  block_sum4(v, red);
}

// y <- x / sqrt(cell * sum) (y may be x).  RES: also the block maxima of |y - prev| (the step's
// change, prev = the step's input, which y may overwrite: each element is read before it is
// written) to res[block * 4]; launched with one block per reduction slot.
template <typename T, bool RES>
__global__ void __launch_bounds__(kRedThreads) k_normalise(const C<T>* x, C<T>* y, const C<T>* prev, int64_t n,
                                                           const double* __restrict__ red, int nblocks, double cell,
                                                           double* __restrict__ res) {
  const double f = 1.0 / sqrt(cell * reduce_partials(red, nblocks, 0, 0.0, OpSum()));
  double mx = 0.0;
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const C<T> p = x[i];
    const C<T> v = C<T>{static_cast<T>(f * p.re), static_cast<T>(f * p.im)};
    if (RES) {
      const C<T> o = prev[i];
      mx = fmax(mx, hypot(static_cast<double>(v.re) - o.re, static_cast<double>(v.im) - o.im));
    }
    y[i] = v;
  }
  if (RES) {
    __shared__ double sm[kRedThreads / 64];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < kRedThreads / 64; ++w) mx = fmax(mx, sm[w]);
      res[blockIdx.x * 4] = mx;
    }
  }
}

// out[0] = max over the block maxima / dt: the stopping residual max |phi^{n+1} - phi^n| / dt
__global__ void k_gf_change(const double* __restrict__ res, int nblocks, double inv_dt, double* __restrict__ out) {
  const double mx = reduce_partials(res, nblocks, 0, 0.0, OpMax());
  if (threadIdx.x == 0 && blockIdx.x == 0) out[0] = mx * inv_dt;
}

// Time splitting (Eq. tssp2): x <- x exp(-i dt |mu|^2 / 4) / prod(N), in Fourier space (the
// 1/prod(N) of the inverse FFT folded in)
template <typename T>
__global__ void __launch_bounds__(256) k_ts_kinetic(C<T>* __restrict__ x, int64_t n, GridGeo G, double qdt,
                                                    double inv_ntot) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    double sn, cs;
    sincos(qdt * mu2_of(i, G), &sn, &cs);    // exp(-i a) = cos a - i sin a
    const C<T> v = x[i];
    const double re = static_cast<double>(v.re), im = static_cast<double>(v.im);
    x[i] = C<T>{static_cast<T>((re * cs + im * sn) * inv_ntot), static_cast<T>((im * cs - re * sn) * inv_ntot)};
  }
}

// Time splitting, nonlinear sub-step (Eq. tssp2, Cases I/II): x <- x exp(-i [dt V + s (beta rho +
// lam Phi)]) * damp, with rho = |x|^2 and Phi = A rho taken before the step
template <typename T>
__global__ void __launch_bounds__(256) k_ts_potential(C<T>* __restrict__ x, const T* __restrict__ rho,
                                                      const T* __restrict__ phi, const T* __restrict__ Vext,
                                                      int64_t n, GridGeo G, double dt, double sfac, double beta,
                                                      double lam, double damp, double loss_q, double loss_c) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double th = dt * trap_v(i, G, Vext) +
                      sfac * (beta * static_cast<double>(rho[i]) + lam * static_cast<double>(phi[i]));
    double sn, cs;
    sincos(th, &sn, &cs);
    const C<T> v = x[i];
    const double re = static_cast<double>(v.re), im = static_cast<double>(v.im);
    double a = damp;
    if (loss_q > 0.0) {
      // Case III: exp(-F) = (1 + 2 q delta dt rho1^q)^(-1/(2q)), loss_c = 2 q delta dt
      const double r = re * re + im * im;
      a = exp(-log1p(loss_c * pow(r, loss_q)) / (2.0 * loss_q));
    }
    x[i] = C<T>{static_cast<T>((re * cs + im * sn) * a), static_cast<T>((im * cs - re * sn) * a)};
  }
}

// Case III (loss f(rho) = delta rho^q): w(rho1), the time integral of the decaying density over
// the step, which enters H = beta w and G = lam A w.  loss_c = 2 q delta dt.
template <typename T>
__global__ void __launch_bounds__(256) k_loss_w(const C<T>* __restrict__ psi, T* __restrict__ w, int64_t n,
                                                double q, double delta, double loss_c) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double re = static_cast<double>(psi[i].re), im = static_cast<double>(psi[i].im);
    const double r = re * re + im * im;
    double v = 0.0;
    if (r > 0.0) {
      const double l = log1p(loss_c * pow(r, q));
      v = q == 1.0 ? l / (2.0 * delta) : expm1((1.0 - 1.0 / q) * l) / (2.0 * delta * (q - 1.0) * pow(r, q - 1.0));
    }
    w[i] = static_cast<T>(v);
  }
}

static GridGeo geo_of(const HostTables& H, const gpe_params& gp) {
  GridGeo G;
  G.N0 = H.N[0]; G.N1 = H.N[1]; G.N2 = H.N[2];
  G.L0 = H.L[0]; G.L1 = H.L[1]; G.L2 = H.L[2];
  G.h0 = H.h[0]; G.h1 = H.h[1]; G.h2 = H.h[2];
  if (H.dim == 3) { G.g0 = gp.gamma[0]; G.g1 = gp.gamma[1]; G.g2 = gp.gamma[2]; }
  else { G.g0 = 0.0; G.g1 = gp.gamma[0]; G.g2 = gp.gamma[1]; }
  return G;
}

template <typename T>
int gpe_reduction_blocks(const DevicePlan& P) {
  const int64_t n = static_cast<int64_t>(P.H.N[0]) * P.H.N[1] * P.H.N[2];
  int64_t b = (n + kRedThreads * 8 - 1) / (kRedThreads * 8);
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return static_cast<int>(b);
}

// Complex 3D FFT of an unpadded N0 x N1 x N2 grid into X, in place, or from `in` when it is
// given (the first pass reads it; `in` is not modified).
template <typename T, int SIGN, int MODE0 = C2C>
static hipError_t fft3_full(DevicePlan& P, C<T>* X, hipStream_t s, const C<T>* in = nullptr,
                            const GfLoad& gl = GfLoad{}) {
  const HostTables& H = P.H;
  const C<T>* tw2 = reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.N[2])]);
  const C<T>* src = in ? in : X;
  DDI_CHECK((launch_contig<T, SIGN, MODE0>(H.N[2], src, X, H.N[0], H.N[1], H.N[0], H.N[1], H.N[2], 0, H.N[2],
                                           nullptr, nullptr, nullptr, tw2, s, gl)));
  DDI_CHECK((launch_strided<T, SIGN>(H.N[1], X, 1, H.N[0], H.N[1], H.N[2], H.N[0], 0, H.N[1], 0, 0, H.N[1], 0, H.N[2],
                                     reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.N[1])]), s)));
  if (H.N[0] > 1) {
    DDI_CHECK((launch_strided<T, SIGN>(H.N[0], X, 0, H.N[0], H.N[1], H.N[2], H.N[1], 0, H.N[0], 0, 0, H.N[0], 0, H.N[2],
                                       reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.N[0])]), s)));
  }
  return hipSuccess;
}

static int ew_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return static_cast<int>(b > 16384 ? 16384 : b);
}

template <typename T>
hipError_t run_gpe_energy_grad(DevicePlan& P, const GpeWork& W, const gpe_params& gp, const Complex<T>* psi,
                               double* E_dev, Complex<T>* grad, hipStream_t s) {
  const HostTables& H = P.H;
  const int64_t n = static_cast<int64_t>(H.N[0]) * H.N[1] * H.N[2];
  const GridGeo G = geo_of(H, gp);
  const double inv_ntot = 1.0 / static_cast<double>(n);
  const int nb = W.red_blocks;
  T* rho = reinterpret_cast<T*>(W.rho);
  T* phi = reinterpret_cast<T*>(W.phi);
  T* phit = reinterpret_cast<T*>(W.phit);
  C<T>* c1 = reinterpret_cast<C<T>*>(W.c1);
  const T* Vext = reinterpret_cast<const T*>(gp.V_dev);
  double* red_kin = W.red;
  double* red_terms = W.red + 4 * nb;
  hipLaunchKernelGGL((k_density<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi, rho, n);
  DDI_CHECK(hipGetLastError());
  DDI_CHECK(run_ddi<T>(P, rho, phi, +1, s, nullptr));
  DDI_CHECK((fft3_full<T, -1>(P, c1, s, psi)));
  hipLaunchKernelGGL((k_kinetic<T>), dim3(nb), dim3(kRedThreads), 0, s, c1, n, G, inv_ntot, red_kin);
  DDI_CHECK(hipGetLastError());
  hipLaunchKernelGGL((k_energy_terms<T>), dim3(nb), dim3(kRedThreads), 0, s, rho, phi, Vext, n, G, red_terms);
  DDI_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(kRedThreads), 0, s, red_kin, red_terms, nb, H.cell, inv_ntot, gp.beta,
                     gp.lambda, E_dev);
  DDI_CHECK(hipGetLastError());
  if (grad) {
    DDI_CHECK(run_ddi<T>(P, rho, phit, -1, s, nullptr));
    DDI_CHECK((fft3_full<T, +1>(P, c1, s)));     // c1 = -1/2 Lap psi
    hipLaunchKernelGGL((k_grad<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi, c1, rho, phi, phit, Vext, n, G, H.cell,
                       gp.beta, gp.lambda, grad);
    DDI_CHECK(hipGetLastError());
  }
  return hipSuccess;
}

template <typename T>
hipError_t run_gf_step(DevicePlan& P, const gpe_params& gp, double dt, int n_inner, const Complex<T>* psi_in,
                       Complex<T>* psi_out, double* residual, hipStream_t s) {
  const HostTables& H = P.H;
  const int64_t n = static_cast<int64_t>(H.N[0]) * H.N[1] * H.N[2];
  const GridGeo G = geo_of(H, gp);
  const double inv_ntot = 1.0 / static_cast<double>(n);
  const int nb = P.gpe.red_blocks;
  T* rho = reinterpret_cast<T*>(P.gpe.rho);
  T* phi = reinterpret_cast<T*>(P.gpe.phi);
  T* Bc = reinterpret_cast<T*>(P.gpe.phit);
  C<T>* rhs0 = reinterpret_cast<C<T>*>(P.gpe.c1);
  C<T>* r = reinterpret_cast<C<T>*>(P.gpe.c2);
  const T* Vext = reinterpret_cast<const T*>(gp.V_dev);
  double* red = P.gpe.red;
  double* scal = P.gpe.red + 8 * nb;
  hipLaunchKernelGGL((k_density<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi_in, rho, n);
  DDI_CHECK(hipGetLastError());
  DDI_CHECK(run_ddi<T>(P, rho, phi, +1, s, nullptr));
  hipLaunchKernelGGL((k_gf_coeff<T>), dim3(nb), dim3(kRedThreads), 0, s, rho, phi, Vext, n, G, gp.beta, gp.lambda,
                     Bc, red);
  DDI_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_gf_alpha, dim3(1), dim3(kRedThreads), 0, s, red, nb, scal);
  DDI_CHECK(hipGetLastError());
  // rhs0 = FFT(psi_in); k_gf_solve divides it by dt
  DDI_CHECK((fft3_full<T, -1>(P, rhs0, s, psi_in)));
  // the iterate: psi_in, then r (updated in place); normalised into psi_out at the end.  The
  // residual (alpha - B) cur is formed in the loads of the forward transform's first pass, and
  // the Fourier-space solve in the loads of the inverse transform's first pass.
  GfLoad gl;
  gl.alpha = scal;
  gl.inv_dt = 1.0 / dt;
  gl.inv_ntot = inv_ntot;
  gl.L[0] = G.L0; gl.L[1] = G.L1; gl.L[2] = G.L2;
  gl.n[0] = G.N0; gl.n[1] = G.N1; gl.n[2] = G.N2;
  const Complex<T>* cur = psi_in;
  for (int it = 0; it < n_inner; ++it) {
    if (kGfFused) {
      gl.aux = Bc;
      DDI_CHECK((fft3_full<T, -1, C2C_GF_RES>(P, r, s, cur, gl)));
      gl.aux = rhs0;
      DDI_CHECK((fft3_full<T, +1, C2C_GF_SOLVE>(P, r, s, nullptr, gl)));
    } else {
      hipLaunchKernelGGL((k_gf_residual<T>), dim3(ew_blocks(n)), dim3(256), 0, s, cur, Bc, scal, n, r);
      DDI_CHECK(hipGetLastError());
      DDI_CHECK((fft3_full<T, -1>(P, r, s)));
      hipLaunchKernelGGL((k_gf_solve<T>), dim3(ew_blocks(n)), dim3(256), 0, s, r, rhs0, scal, n, G, dt, inv_ntot);
      DDI_CHECK(hipGetLastError());
      DDI_CHECK((fft3_full<T, +1>(P, r, s)));
    }
    cur = r;
  }
  hipLaunchKernelGGL((k_norm2<T>), dim3(nb), dim3(kRedThreads), 0, s, cur, n, red);
  DDI_CHECK(hipGetLastError());
  if (residual) {
    // the block maxima of the change go to the second half of the reduction scratch
    hipLaunchKernelGGL((k_normalise<T, true>), dim3(nb), dim3(kRedThreads), 0, s, cur, psi_out, psi_in, n, red, nb,
                       H.cell, red + 4 * nb);
    DDI_CHECK(hipGetLastError());
    hipLaunchKernelGGL(k_gf_change, dim3(1), dim3(kRedThreads), 0, s, red + 4 * nb, nb, 1.0 / dt, residual);
  } else {
    hipLaunchKernelGGL((k_normalise<T, false>), dim3(nb), dim3(kRedThreads), 0, s, cur, psi_out, psi_in, n, red, nb,
                       H.cell, nullptr);
  }
  return hipGetLastError();
}


// One step of the second-order time splitting (Eq. tssp2), cubic nonlinearity, time-independent
// dipole axis, damping f = delta >= 0 (Case I: 0; Case II: linear) or, with q > 0, the loss
// f = delta rho^q (Case III): half kinetic step, the nonlinear step with rho (Case III: w(rho))
// and Phi = A rho (A w) of the half-stepped state, half kinetic step.
template <typename T>
hipError_t run_ts_step(DevicePlan& P, const gpe_params& gp, double dt, double delta, double q,
                       const Complex<T>* psi_in, Complex<T>* psi_out, hipStream_t s) {
  const HostTables& H = P.H;
  const int64_t n = static_cast<int64_t>(H.N[0]) * H.N[1] * H.N[2];
  const GridGeo G = geo_of(H, gp);
  const double inv_ntot = 1.0 / static_cast<double>(n);
  T* rho = reinterpret_cast<T*>(P.gpe.rho);
  T* phi = reinterpret_cast<T*>(P.gpe.phi);
  const T* Vext = reinterpret_cast<const T*>(gp.V_dev);
  // Case II time factor (1 - exp(-2 delta dt)) / (2 delta), dt in Case I; Case III: w carries it
  const bool loss = q > 0.0;
  const double loss_c = 2.0 * q * delta * dt;
  const double sfac = loss ? 1.0 : (delta == 0.0 ? dt : -std::expm1(-2.0 * delta * dt) / (2.0 * delta));
  // the first transform reads psi_in; everything after it works in place on psi_out
  auto half_kinetic = [&](const Complex<T>* from) -> hipError_t {
    DDI_CHECK((fft3_full<T, -1>(P, psi_out, s, from)));
    if (kGfFused) {   // the kinetic factor in the loads of the inverse transform's first pass
      GfLoad gl;
      gl.qdt = 0.25 * dt;
      gl.inv_ntot = inv_ntot;
      gl.L[0] = G.L0; gl.L[1] = G.L1; gl.L[2] = G.L2;
      gl.n[0] = G.N0; gl.n[1] = G.N1; gl.n[2] = G.N2;
      return fft3_full<T, +1, C2C_TS_KIN>(P, psi_out, s, nullptr, gl);
    }
    hipLaunchKernelGGL((k_ts_kinetic<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi_out, n, G, 0.25 * dt, inv_ntot);
    DDI_CHECK(hipGetLastError());
    return fft3_full<T, +1>(P, psi_out, s);
  };
  DDI_CHECK(half_kinetic(psi_in));
  if (loss) hipLaunchKernelGGL((k_loss_w<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi_out, rho, n, q, delta, loss_c);
  else hipLaunchKernelGGL((k_density<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi_out, rho, n);
  DDI_CHECK(hipGetLastError());
  if (gp.lambda != 0.0) DDI_CHECK(run_ddi<T>(P, rho, phi, +1, s, nullptr));
  hipLaunchKernelGGL((k_ts_potential<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi_out, rho,
                     gp.lambda != 0.0 ? phi : rho, Vext, n, G, dt, sfac, gp.beta, gp.lambda,
                     loss ? 1.0 : std::exp(-delta * dt), loss ? q : 0.0, loss_c);
  DDI_CHECK(hipGetLastError());
  return half_kinetic(psi_out);
}

template hipError_t run_gpe_energy_grad<double>(DevicePlan&, const GpeWork&, const gpe_params&,
                                                const Complex<double>*, double*, Complex<double>*, hipStream_t);
template hipError_t run_gpe_energy_grad<float>(DevicePlan&, const GpeWork&, const gpe_params&,
                                               const Complex<float>*, double*, Complex<float>*, hipStream_t);
template hipError_t run_gf_step<double>(DevicePlan&, const gpe_params&, double, int, const Complex<double>*,
                                        Complex<double>*, double*, hipStream_t);
template hipError_t run_gf_step<float>(DevicePlan&, const gpe_params&, double, int, const Complex<float>*,
                                       Complex<float>*, double*, hipStream_t);
template hipError_t run_ts_step<double>(DevicePlan&, const gpe_params&, double, double, double,
                                        const Complex<double>*, Complex<double>*, hipStream_t);
template hipError_t run_ts_step<float>(DevicePlan&, const gpe_params&, double, double, double,
                                       const Complex<float>*, Complex<float>*, hipStream_t);
template int gpe_reduction_blocks<double>(const DevicePlan&);
template int gpe_reduction_blocks<float>(const DevicePlan&);

}  // namespace ddi
