// HIP kernels of the NUFFT DDI path for gfx950 (CDNA4, wave64).
//
// Forward operator (Sec. 2.1, Eqs. DDI-Con, DDI-Trun1), one pass:
//   type-2 NUFFT  rho -> rhohat_q   : deconvolve + zero-pad fused into the first FFT pass,
//                                     pruned 3-pass FFT on the oversampled grid,
//                                     interpolation at the quadrature nodes (one wave per node),
//   weights       g_q = c_q prod(h) rhohat_q (fused into the interpolation epilogue),
//   type-1 NUFFT  g -> Phi          : tile-owned spread (no atomics; hot tiles split into chunks
//                                     and summed by a reduce kernel), pruned 3-pass FFT,
//                                     truncate + deconvolve + real part fused into the last pass.
// The kernel is the exponential-of-semicircle function; its weights are tabulated per node
// at plan time, so no transcendental is evaluated per apply.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ddi_internal.h"

namespace ddi {

template <typename T>
using C = Complex<T>;

template <typename T>
__device__ __forceinline__ C<T> cmul(C<T> a, C<T> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename T>
__device__ __forceinline__ C<T> cadd(C<T> a, C<T> b) { return {a.re + b.re, a.im + b.im}; }
template <typename T>
__device__ __forceinline__ C<T> csub(C<T> a, C<T> b) { return {a.re - b.re, a.im - b.im}; }

// cos(2 pi j / 16) from the first-quadrant values
__host__ __device__ constexpr double cos_16(int j) {
  j &= 15;
  const double q[5] = {1.0, 0.92387953251128675613, 0.70710678118654752440, 0.38268343236508977173, 0.0};
  return j <= 4 ? q[j] : (j <= 8 ? -q[8 - j] : (j <= 12 ? -q[j - 8] : q[16 - j]));
}

// ------------------------------------------------------------------ in-register DFT of size R <= 16
// out[k] = sum_r v[r] exp(SIGN 2 pi i r k / R), iterative radix-2 decimation in time.
template <int R>
__device__ __forceinline__ constexpr int bitrev(int i) {
  int r = 0;
  for (int b = 1; b < R; b <<= 1) { r = (r << 1) | (i & 1); i >>= 1; }
  return r;
}

template <typename T, int R, int SIGN>
__device__ __forceinline__ void dft_regs(C<T>* v) {
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

// ------------------------------------------------------------------ radix plans
template <int N> struct RadixPlan;
template <> struct RadixPlan<8> { static constexpr int R1 = 8, R2 = 1, R3 = 1; };
template <> struct RadixPlan<16> { static constexpr int R1 = 4, R2 = 4, R3 = 1; };
template <> struct RadixPlan<32> { static constexpr int R1 = 8, R2 = 4, R3 = 1; };
template <> struct RadixPlan<64> { static constexpr int R1 = 8, R2 = 8, R3 = 1; };
template <> struct RadixPlan<128> { static constexpr int R1 = 16, R2 = 8, R3 = 1; };
template <> struct RadixPlan<256> { static constexpr int R1 = 16, R2 = 16, R3 = 1; };
template <> struct RadixPlan<512> { static constexpr int R1 = 8, R2 = 8, R3 = 8; };
template <> struct RadixPlan<1024> { static constexpr int R1 = 16, R2 = 16, R3 = 4; };

// One Stockham pass (radix R, Ns = product of earlier radices) over LDS, for the
// butterflies j = j0 + TL*b owned by this thread.  The thread's registers hold
// R1 values (R1/R butterflies of R values).
template <typename T, int N, int R1, int R, int SIGN, typename Addr>
__device__ __forceinline__ void stockham_load(C<T>* lds, Addr addr, int j0, int Ns, const C<T>* __restrict__ tw,
                                              C<T>* v) {
  constexpr int TL = N / R1;
  constexpr int NB = R1 / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = j0 + TL * b;
    const int jm = j % Ns;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      C<T> x = lds[addr(j + r * (N / R))];
      if (r > 0) {
        C<T> w = tw[(r * jm * (N / (Ns * R))) & (N - 1)];
        if (SIGN > 0) w.im = -w.im;
        x = cmul(x, w);
      }
      v[b * R + r] = x;
    }
    dft_regs<T, R, SIGN>(v + b * R);
  }
}

template <typename T, int N, int R1, int R, typename Addr>
__device__ __forceinline__ void stockham_store(C<T>* lds, Addr addr, int j0, int Ns, const C<T>* v) {
  constexpr int TL = N / R1;
  constexpr int NB = R1 / R;
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int j = j0 + TL * b;
    const int idxD = (j / Ns) * Ns * R + (j % Ns);
#pragma unroll
    for (int r = 0; r < R; ++r) lds[addr(idxD + r * Ns)] = v[b * R + r];
  }
}

// Full line FFT.  On entry v[r] = x[j0 + r*TL] (r < R1).  On exit the thread
// holds the outputs k = j + r*(N/Rlast), j = j0 + TL*b, in v[b*Rlast + r].
template <typename T, int N, int SIGN, typename Addr>
__device__ __forceinline__ void line_fft(C<T>* lds, Addr addr, int j0, const C<T>* __restrict__ tw, C<T>* v) {
  using P = RadixPlan<N>;
  dft_regs<T, P::R1, SIGN>(v);
  if constexpr (P::R2 > 1) {
    stockham_store<T, N, P::R1, P::R1>(lds, addr, j0, 1, v);
    __syncthreads();
    stockham_load<T, N, P::R1, P::R2, SIGN>(lds, addr, j0, P::R1, tw, v);
    if constexpr (P::R3 > 1) {
      __syncthreads();
      stockham_store<T, N, P::R1, P::R2>(lds, addr, j0, P::R1, v);
      __syncthreads();
      stockham_load<T, N, P::R1, P::R3, SIGN>(lds, addr, j0, P::R1 * P::R2, tw, v);
    }
  }
}

template <int N>
struct LineOut {
  using P = RadixPlan<N>;
  static constexpr int RL = P::R3 > 1 ? P::R3 : (P::R2 > 1 ? P::R2 : P::R1);
  static constexpr int TL = N / P::R1;
  // output index held in v[i] by thread j0
  __device__ static __forceinline__ int k(int j0, int i) {
    const int b = i / RL, r = i % RL;
    return j0 + TL * b + r * (N / RL);
  }
};

// Modes m = c - nc/2, c in [0, nc), sit at fine index m mod n: the active set is
// [0, nc - nc/2) and [n - nc/2, n).
__device__ __forceinline__ bool active(int k, int n, int nc) { return k < nc - nc / 2 || k >= n - nc / 2; }
// compact index c in [0, nc) -> fine index of mode c - nc/2
__device__ __forceinline__ int fmap(int c, int n, int nc) { return c < nc / 2 ? n - nc / 2 + c : c - nc / 2; }
// fine index -> compact index (only for active k)
__device__ __forceinline__ int cmap(int k, int n, int nc) { return k < nc - nc / 2 ? k + nc / 2 : k - (n - nc / 2); }

// Remap the block index so that consecutive logical blocks land on the same XCD
// (blocks are dispatched round-robin over the 8 XCDs, each with its own L2).
__device__ __forceinline__ int xcd_remap(int b, int nb) {
  constexpr int X = 8;
  const int x = b % X, local = b / X;
  const int base = nb / X, rem = nb % X;
  return x * base + (x < rem ? x : rem) + local;
}

// ------------------------------------------------------------------ strided-axis FFT pass
// Lines along axis `axis` (0 or 1) of a [d0][d1][d2] complex array, B consecutive
// z per workgroup.  The other non-z axis runs over n_o lines (compact when
// o_compact: index o -> fine index fmap(o, d_o, n_o)).  in_compact / out_compact:
// only the N_c active positions of the line are read (rest zero) / written.
template <typename T, int N, int SIGN>
__global__ void __launch_bounds__(256) k_fft_strided(C<T>* __restrict__ F, int axis, int d0, int d1, int d2,
                                                     int n_o, int o_compact, int nc_axis, int in_compact,
                                                     int out_compact, const C<T>* __restrict__ tw, int B) {
  extern __shared__ unsigned char smem_raw[];
  C<T>* lds = reinterpret_cast<C<T>*>(smem_raw);
  using P = RadixPlan<N>;
  constexpr int TL = N / P::R1;
  const int b = threadIdx.x % B;
  const int j0 = threadIdx.x / B;
  const int zblocks = d2 / B;
  const int blk = blockIdx.x;
  const int o = blk / zblocks;
  const int z = (blk % zblocks) * B + b;
  const int d_o = axis == 0 ? d1 : d0;
  const int of = o_compact ? fmap(o, d_o, n_o) : o;
  int64_t base, stride;
  if (axis == 0) { base = static_cast<int64_t>(of) * d2 + z; stride = static_cast<int64_t>(d1) * d2; }
  else { base = static_cast<int64_t>(of) * d1 * d2 + z; stride = d2; }
  auto addr = [B, b](int k) { return k * B + b; };
  C<T> v[P::R1];
#pragma unroll
  for (int r = 0; r < P::R1; ++r) {
    const int k = j0 + r * TL;
    if (in_compact && !active(k, N, nc_axis)) v[r] = C<T>{0, 0};
    else v[r] = F[base + k * stride];
  }
  line_fft<T, N, SIGN>(lds, addr, j0, tw, v);
#pragma unroll
  for (int i = 0; i < P::R1; ++i) {
    const int k = LineOut<N>::k(j0, i);
    if (!out_compact || active(k, N, nc_axis)) F[base + k * stride] = v[i];
  }
}

// ------------------------------------------------------------------ last-axis (contiguous) FFT pass
enum ContigMode { R2C_PAD = 0, C2C = 1, C2R_TRUNC = 2 };

// Lines along axis 2.  Line l -> (o0, o1); in R2C_PAD / C2R_TRUNC modes (o0, o1)
// run over the compact N0 x N1 grid and map to fine indices; in C2C they run
// over d0 x d1 directly.  R2C_PAD: input real rho[N0][N1][N2] times the
// deconvolution factors, placed at the active positions of a length-N line,
// output complex line.  C2R_TRUNC: input complex line, output
// Re(line[fmap(c2)]) times the deconvolution factors into phi[N0][N1][N2].
template <typename T, int N, int SIGN, int MODE>
__global__ void __launch_bounds__(256) k_fft_contig(const void* in, void* out,
                                                    int n0, int n1, int d0, int d1, int nc2,
                                                    const double* __restrict__ D0, const double* __restrict__ D1,
                                                    const double* __restrict__ D2,
                                                    const C<T>* __restrict__ tw, int B, int nlines) {
  extern __shared__ unsigned char smem_raw[];
  C<T>* lds = reinterpret_cast<C<T>*>(smem_raw);
  using P = RadixPlan<N>;
  constexpr int TL = N / P::R1;
  constexpr int LS = N + N / P::R1;      // padded line stride in LDS
  const int j0 = threadIdx.x % TL;
  const int lb = threadIdx.x / TL;
  const int line = blockIdx.x * B + lb;
  const bool valid = line < nlines;
  const int o0 = valid ? line / n1 : 0;
  const int o1 = valid ? line % n1 : 0;
  C<T>* my = lds + lb * LS;
  auto addr = [](int k) { return k + k / RadixPlan<N>::R1; };
  C<T> v[P::R1];
  if (MODE == R2C_PAD) {
    const T* rho = reinterpret_cast<const T*>(in);
    const double s01 = D0[o0] * D1[o1];
    const int64_t rb = (static_cast<int64_t>(o0) * n1 + o1) * nc2;
#pragma unroll
    for (int r = 0; r < P::R1; ++r) {
      const int k = j0 + r * TL;
      if (valid && active(k, N, nc2)) {
        const int c2 = cmap(k, N, nc2);
        v[r] = C<T>{static_cast<T>(static_cast<double>(rho[rb + c2]) * s01 * D2[c2]), T(0)};
      } else {
        v[r] = C<T>{0, 0};
      }
    }
  } else {
    const C<T>* F = reinterpret_cast<const C<T>*>(in);
    int64_t lbase;
    if (MODE == C2C) lbase = static_cast<int64_t>(line) * N;
    else lbase = (static_cast<int64_t>(fmap(o0, d0, n0)) * d1 + fmap(o1, d1, n1)) * N;
#pragma unroll
    for (int r = 0; r < P::R1; ++r) {
      const int k = j0 + r * TL;
      v[r] = valid ? F[lbase + k] : C<T>{0, 0};
    }
  }
  line_fft<T, N, SIGN>(my, addr, j0, tw, v);
  if (!valid) return;
  if (MODE == C2R_TRUNC) {
    T* phi = reinterpret_cast<T*>(out);
    const double s01 = D0[o0] * D1[o1];
    const int64_t rb = (static_cast<int64_t>(o0) * n1 + o1) * nc2;
#pragma unroll
    for (int i = 0; i < P::R1; ++i) {
      const int k = LineOut<N>::k(j0, i);
      if (active(k, N, nc2)) {
        const int c2 = cmap(k, N, nc2);
        phi[rb + c2] = static_cast<T>(static_cast<double>(v[i].re) * s01 * D2[c2]);
      }
    }
  } else {
    C<T>* F = reinterpret_cast<C<T>*>(out);
    int64_t lbase;
    if (MODE == C2C) lbase = static_cast<int64_t>(line) * N;
    else lbase = (static_cast<int64_t>(fmap(o0, d0, n0)) * d1 + fmap(o1, d1, n1)) * N;
#pragma unroll
    for (int i = 0; i < P::R1; ++i) F[lbase + LineOut<N>::k(j0, i)] = v[i];
  }
}

// ------------------------------------------------------------------ interpolation (type-2 tail)
// One wave per node: lanes cover the (y, z) support, the x support is looped.
// out_q = scale_q * sum psi_x psi_y psi_z F[l0 + i], accumulated in FP64.
template <typename T>
__global__ void __launch_bounds__(256) k_interp(const C<T>* __restrict__ F, const NodeRec<T>* __restrict__ nodes,
                                                int64_t M, int nf0, int nf1, int nf2, int w0, int w1, int w2,
                                                const double* __restrict__ scale, double sscalar,
                                                C<T>* __restrict__ out) {
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t q = static_cast<int64_t>(blk) * 4 + wv;
  if (q >= M) return;
  const NodeRec<T>& nd = nodes[q];
  const int lx = nd.l0[0], ly = nd.l0[1], lz = nd.l0[2];
  double are = 0.0, aim = 0.0;
  const int npair = w1 * w2;
  for (int p = lane; p < npair; p += 64) {
    const int iy = p / w2, iz = p - iy * w2;
    int gy = ly + iy; if (gy >= nf1) gy -= nf1;
    int gz = lz + iz; if (gz >= nf2) gz -= nf2;
    const double wyz = static_cast<double>(nd.w[1][iy]) * static_cast<double>(nd.w[2][iz]);
    double sre = 0.0, sim = 0.0;
    for (int ix = 0; ix < w0; ++ix) {
      int gx = lx + ix; if (gx >= nf0) gx -= nf0;
      const C<T> f = F[(static_cast<int64_t>(gx) * nf1 + gy) * nf2 + gz];
      const double wx = static_cast<double>(nd.w[0][ix]);
      sre += wx * static_cast<double>(f.re);
      sim += wx * static_cast<double>(f.im);
    }
    are += wyz * sre;
    aim += wyz * sim;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    are += __shfl_xor(are, off, 64);
    aim += __shfl_xor(aim, off, 64);
  }
  if (lane == 0) {
    const double s = scale ? scale[q] * sscalar : sscalar;
    out[q] = C<T>{static_cast<T>(s * are), static_cast<T>(s * aim)};
  }
}

// ------------------------------------------------------------------ spread (type-1 head)
// One wave per work item.  The item's tile (TX x TY x kTileZ points, TX*TY = 64)
// is owned by the wave: lane (lx, ly) accumulates kTileZ points along z in
// registers over the item's node list; no atomics.  FP32 accumulation is
// Kahan-compensated.
template <typename T, bool KAHAN>
__global__ void __launch_bounds__(64) k_spread(C<T>* __restrict__ F, C<T>* __restrict__ partial,
                                               const NodeRec<T>* __restrict__ nodes, const C<T>* __restrict__ g,
                                               const int32_t* __restrict__ list,
                                               const SpreadItem* __restrict__ items, int nf0, int nf1, int nf2,
                                               int TX, int TY, int nt1, int nt2, int w0, int w1, int w2) {
  const int lane = threadIdx.x;
  const SpreadItem it = items[blockIdx.x];
  const int tz = it.tile % nt2;
  const int ty = (it.tile / nt2) % nt1;
  const int tx = it.tile / (nt2 * nt1);
  const int lxo = lane / TY, lyo = lane % TY;
  const int x = tx * TX + lxo, y = ty * TY + lyo, z0 = tz * kTileZ;
  C<T> acc[kTileZ];
  C<T> cmp[kTileZ];
#pragma unroll
  for (int i = 0; i < kTileZ; ++i) { acc[i] = C<T>{0, 0}; cmp[i] = C<T>{0, 0}; }
  for (int e = 0; e < it.count; ++e) {
    const int q = list[it.start + e];
    const NodeRec<T>& nd = nodes[q];
    int dx = x - nd.l0[0]; if (dx < 0) dx += nf0;
    int dy = y - nd.l0[1]; if (dy < 0) dy += nf1;
    int dz0 = z0 - nd.l0[2]; if (dz0 < 0) dz0 += nf2;
    const T wx = dx < w0 ? nd.w[0][dx] : T(0);
    const T wy = dy < w1 ? nd.w[1][dy] : T(0);
    const C<T> gq = g[q];
    const T wxy = wx * wy;
    const C<T> pq = {gq.re * wxy, gq.im * wxy};
#pragma unroll
    for (int i = 0; i < kTileZ; ++i) {
      int dz = dz0 + i; if (dz >= nf2) dz -= nf2;
      const T wz = dz < w2 ? nd.w[2][dz] : T(0);
      if (KAHAN) {
        T yr = pq.re * wz - cmp[i].re;
        T tr = acc[i].re + yr;
        cmp[i].re = (tr - acc[i].re) - yr;
        acc[i].re = tr;
        T yi = pq.im * wz - cmp[i].im;
        T ti = acc[i].im + yi;
        cmp[i].im = (ti - acc[i].im) - yi;
        acc[i].im = ti;
      } else {
        acc[i].re += pq.re * wz;
        acc[i].im += pq.im * wz;
      }
    }
  }
  if (it.slot < 0) {
    C<T>* row = F + (static_cast<int64_t>(x) * nf1 + y) * nf2 + z0;
#pragma unroll
    for (int i = 0; i < kTileZ; ++i) row[i] = acc[i];
  } else {
    C<T>* pt = partial + static_cast<int64_t>(it.slot) * 64 * kTileZ;
#pragma unroll
    for (int i = 0; i < kTileZ; ++i) pt[i * 64 + lane] = acc[i];
  }
}

// Sum the partial tiles of each split tile in slot order (deterministic).
template <typename T>
__global__ void __launch_bounds__(64) k_spread_reduce(C<T>* __restrict__ F, const C<T>* __restrict__ partial,
                                                      const ReduceItem* __restrict__ red, int nf1, int nf2, int TX,
                                                      int TY, int nt1, int nt2) {
  const int lane = threadIdx.x;
  const ReduceItem r = red[blockIdx.x];
  const int tz = r.tile % nt2;
  const int ty = (r.tile / nt2) % nt1;
  const int tx = r.tile / (nt2 * nt1);
  const int x = tx * TX + lane / TY, y = ty * TY + lane % TY, z0 = tz * kTileZ;
  C<T>* row = F + (static_cast<int64_t>(x) * nf1 + y) * nf2 + z0;
#pragma unroll
  for (int i = 0; i < kTileZ; ++i) {
    double sr = 0.0, si = 0.0;
    for (int s = 0; s < r.nslots; ++s) {
      const C<T> v = partial[(static_cast<int64_t>(r.first_slot + s) * kTileZ + i) * 64 + lane];
      sr += static_cast<double>(v.re);
      si += static_cast<double>(v.im);
    }
    row[i] = C<T>{static_cast<T>(sr), static_cast<T>(si)};
  }
}

// ------------------------------------------------------------------ FFT dispatch
template <typename T, int N, int SIGN>
static hipError_t launch_strided_n(C<T>* F, int axis, int d0, int d1, int d2, int n_o, int o_compact, int nc,
                                   int in_c, int out_c, const C<T>* tw, hipStream_t s) {
  constexpr int TL = N / RadixPlan<N>::R1;
  int B = 256 / TL;
  while (B > d2) B >>= 1;
  const size_t shm = static_cast<size_t>(B) * N * sizeof(C<T>);
  const int blocks = n_o * (d2 / B);
  hipLaunchKernelGGL((k_fft_strided<T, N, SIGN>), dim3(blocks), dim3(B * TL), shm, s, F, axis, d0, d1, d2, n_o,
                     o_compact, nc, in_c, out_c, tw, B);
  return hipGetLastError();
}

template <typename T, int SIGN>
static hipError_t launch_strided(int n, C<T>* F, int axis, int d0, int d1, int d2, int n_o, int o_compact, int nc,
                                 int in_c, int out_c, const C<T>* tw, hipStream_t s) {
  switch (n) {
    case 8: return launch_strided_n<T, 8, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, tw, s);
    case 16: return launch_strided_n<T, 16, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, tw, s);
    case 32: return launch_strided_n<T, 32, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, tw, s);
    case 64: return launch_strided_n<T, 64, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, tw, s);
    case 128: return launch_strided_n<T, 128, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, tw, s);
    case 256: return launch_strided_n<T, 256, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, tw, s);
    case 512: return launch_strided_n<T, 512, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, tw, s);
    case 1024: return launch_strided_n<T, 1024, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, tw, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int N, int SIGN, int MODE>
static hipError_t launch_contig_n(const void* in, void* out, int n0, int n1, int d0, int d1, int nc2,
                                  const double* D0, const double* D1, const double* D2, const C<T>* tw,
                                  hipStream_t s) {
  constexpr int TL = N / RadixPlan<N>::R1;
  constexpr int LS = N + N / RadixPlan<N>::R1;
  int B = 256 / TL;
  while (B > 1 && static_cast<size_t>(B) * LS * sizeof(C<T>) > 65536) B >>= 1;
  const int nlines = n0 * n1;
  const size_t shm = static_cast<size_t>(B) * LS * sizeof(C<T>);
  const int blocks = (nlines + B - 1) / B;
  hipLaunchKernelGGL((k_fft_contig<T, N, SIGN, MODE>), dim3(blocks), dim3(B * TL), shm, s, in, out, n0, n1, d0, d1,
                     nc2, D0, D1, D2, tw, B, nlines);
  return hipGetLastError();
}

template <typename T, int SIGN, int MODE>
static hipError_t launch_contig(int n, const void* in, void* out, int n0, int n1, int d0, int d1, int nc2,
                                const double* D0, const double* D1, const double* D2, const C<T>* tw,
                                hipStream_t s) {
  switch (n) {
    case 8: return launch_contig_n<T, 8, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, D0, D1, D2, tw, s);
    case 16: return launch_contig_n<T, 16, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, D0, D1, D2, tw, s);
    case 32: return launch_contig_n<T, 32, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, D0, D1, D2, tw, s);
    case 64: return launch_contig_n<T, 64, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, D0, D1, D2, tw, s);
    case 128: return launch_contig_n<T, 128, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, D0, D1, D2, tw, s);
    case 256: return launch_contig_n<T, 256, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, D0, D1, D2, tw, s);
    case 512: return launch_contig_n<T, 512, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, D0, D1, D2, tw, s);
    case 1024: return launch_contig_n<T, 1024, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, D0, D1, D2, tw, s);
    default: return hipErrorInvalidValue;
  }
}

static int ilog2(int n) {
  int l = 0;
  while ((1 << l) < n) ++l;
  return l;
}

#define DDI_CHECK(x)                         \
  do {                                       \
    hipError_t e_ = (x);                     \
    if (e_ != hipSuccess) return e_;         \
  } while (0)

// Forward transform of the padded, deconvolved density onto the fine grid
// (pruned: only lines that can hold non-zeros are transformed).
#define DDI_REC(i)                                  \
  do {                                              \
    if (ev) DDI_CHECK(hipEventRecord(ev[(i)], s));  \
  } while (0)

template <typename T, int SIGN>
static hipError_t type2_fft(DevicePlan& P, const T* rho, hipStream_t s, hipEvent_t* ev) {
  const HostTables& H = P.H;
  C<T>* F = reinterpret_cast<C<T>*>(P.fine);
  const C<T>* tw2 = reinterpret_cast<const C<T>*>(P.twiddles[ilog2(H.nf[2])]);
  DDI_CHECK((launch_contig<T, SIGN, R2C_PAD>(H.nf[2], rho, F, H.N[0], H.N[1], H.nf[0], H.nf[1], H.N[2],
                                             P.deconv[0], P.deconv[1], P.deconv[2], tw2, s)));
  DDI_REC(1);
  // axis 1: lines (x active, all z), input active y only
  DDI_CHECK((launch_strided<T, SIGN>(H.nf[1], F, 1, H.nf[0], H.nf[1], H.nf[2], H.N[0], 1, H.N[1], 1, 0,
                                     reinterpret_cast<const C<T>*>(P.twiddles[ilog2(H.nf[1])]), s)));
  DDI_REC(2);
  if (H.nf[0] > 1) {
    DDI_CHECK((launch_strided<T, SIGN>(H.nf[0], F, 0, H.nf[0], H.nf[1], H.nf[2], H.nf[1], 0, H.N[0], 1, 0,
                                       reinterpret_cast<const C<T>*>(P.twiddles[ilog2(H.nf[0])]), s)));
  }
  DDI_REC(3);
  return hipSuccess;
}

template <typename T, int SIGN>
static hipError_t type1_fft(DevicePlan& P, T* phi, hipStream_t s, hipEvent_t* ev) {
  const HostTables& H = P.H;
  C<T>* F = reinterpret_cast<C<T>*>(P.fine);
  if (H.nf[0] > 1) {
    DDI_CHECK((launch_strided<T, SIGN>(H.nf[0], F, 0, H.nf[0], H.nf[1], H.nf[2], H.nf[1], 0, H.N[0], 0, 1,
                                       reinterpret_cast<const C<T>*>(P.twiddles[ilog2(H.nf[0])]), s)));
  }
  DDI_REC(7);
  DDI_CHECK((launch_strided<T, SIGN>(H.nf[1], F, 1, H.nf[0], H.nf[1], H.nf[2], H.N[0], 1, H.N[1], 0, 1,
                                     reinterpret_cast<const C<T>*>(P.twiddles[ilog2(H.nf[1])]), s)));
  DDI_REC(8);
  const C<T>* tw2 = reinterpret_cast<const C<T>*>(P.twiddles[ilog2(H.nf[2])]);
  DDI_CHECK((launch_contig<T, SIGN, C2R_TRUNC>(H.nf[2], F, phi, H.N[0], H.N[1], H.nf[0], H.nf[1], H.N[2],
                                               P.deconv[0], P.deconv[1], P.deconv[2], tw2, s)));
  DDI_REC(9);
  return hipSuccess;
}

template <typename T>
static hipError_t interp(DevicePlan& P, C<T>* out, const double* scale, double sscalar, hipStream_t s) {
  const HostTables& H = P.H;
  const int blocks = static_cast<int>((H.M + 3) / 4);
  hipLaunchKernelGGL((k_interp<T>), dim3(blocks), dim3(256), 0, s, reinterpret_cast<const C<T>*>(P.fine),
                     reinterpret_cast<const NodeRec<T>*>(P.nodes), H.M, H.nf[0], H.nf[1], H.nf[2], H.W[0], H.W[1],
                     H.W[2], scale, sscalar, out);
  return hipGetLastError();
}

template <typename T>
static hipError_t spread(DevicePlan& P, const C<T>* g, hipStream_t s, hipEvent_t* ev) {
  const HostTables& H = P.H;
  C<T>* F = reinterpret_cast<C<T>*>(P.fine);
  const int nitems = static_cast<int>(H.items.size());
  constexpr bool kahan = sizeof(T) == 4;
  hipLaunchKernelGGL((k_spread<T, kahan>), dim3(nitems), dim3(64), 0, s, F, reinterpret_cast<C<T>*>(P.partial),
                     reinterpret_cast<const NodeRec<T>*>(P.nodes), g, P.list, P.items, H.nf[0], H.nf[1], H.nf[2],
                     H.tile[0], H.tile[1], H.ntiles[1], H.ntiles[2], H.W[0], H.W[1], H.W[2]);
  DDI_CHECK(hipGetLastError());
  DDI_REC(5);
  if (!H.reduces.empty()) {
    hipLaunchKernelGGL((k_spread_reduce<T>), dim3(static_cast<int>(H.reduces.size())), dim3(64), 0, s, F,
                       reinterpret_cast<const C<T>*>(P.partial), P.reduces, H.nf[1], H.nf[2], H.tile[0],
                       H.tile[1], H.ntiles[1], H.ntiles[2]);
    DDI_CHECK(hipGetLastError());
  }
  DDI_REC(6);
  return hipSuccess;
}

// ev (nullable): events recorded on s at the start (ev[0]) and after each stage:
// 1 last-axis FFT (pad), 2 axis-1 FFT, 3 axis-0 FFT, 4 interpolation, 5 spread,
// 6 spread reduce, 7 axis-0 FFT, 8 axis-1 FFT, 9 last-axis FFT (truncate).
template <typename T>
hipError_t run_type2(DevicePlan& P, const T* rho, Complex<T>* out, const double* scale, double cscalar, int sign,
                     hipStream_t s, hipEvent_t* ev) {
  DDI_REC(0);
  if (sign < 0) DDI_CHECK((type2_fft<T, -1>(P, rho, s, ev)));
  else DDI_CHECK((type2_fft<T, +1>(P, rho, s, ev)));
  DDI_CHECK((interp<T>(P, out, scale, cscalar, s)));
  DDI_REC(4);
  return hipSuccess;
}

template <typename T>
hipError_t run_type1(DevicePlan& P, const Complex<T>* g, T* phi, int sign, hipStream_t s, hipEvent_t* ev) {
  DDI_CHECK(spread<T>(P, g, s, ev));
  if (sign > 0) return type1_fft<T, +1>(P, phi, s, ev);
  return type1_fft<T, -1>(P, phi, s, ev);
}

// Forward (sign = +1: exp(-ikx) to the nodes, exp(+ikx) back) or literal adjoint (sign = -1).
template <typename T>
hipError_t run_apply(DevicePlan& P, const T* rho, T* phi, int sign, hipStream_t s, hipEvent_t* ev) {
  C<T>* g = reinterpret_cast<C<T>*>(P.gnodes);
  DDI_CHECK(run_type2<T>(P, rho, g, P.c_scaled, 1.0, -sign, s, ev));
  return run_type1<T>(P, g, phi, sign, s, ev);
}

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

template <typename T>
__global__ void __launch_bounds__(256) k_density(const C<T>* __restrict__ psi, T* __restrict__ rho, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const C<T> p = psi[i];
    rho[i] = static_cast<T>(static_cast<double>(p.re) * p.re + static_cast<double>(p.im) * p.im);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_copy(const C<T>* __restrict__ a, C<T>* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    b[i] = a[i];
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
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double s[4] = {0, 0, 0, 0};
  for (int b = 0; b < nblocks; ++b) {
    s[0] += red_kin[b * 4 + 0];
    s[1] += red_terms[b * 4 + 1];
    s[2] += red_terms[b * 4 + 2];
    s[3] += red_terms[b * 4 + 3];
  }
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
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double mx = -1e300, mn = 1e300;
  for (int b = 0; b < nblocks; ++b) { mx = fmax(mx, red[b * 4]); mn = fmin(mn, red[b * 4 + 1]); }
  scal[0] = 0.5 * (mx + mn);
}

// r = (alpha - B) phi
template <typename T>
__global__ void __launch_bounds__(256) k_gf_residual(const C<T>* __restrict__ phi, const T* __restrict__ B,
                                                     const double* __restrict__ scal, int64_t n,
                                                     C<T>* __restrict__ r) {
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
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double den = (1.0 / dt + alpha + 0.5 * mu2_of(i, G)) / inv_ntot;
    const C<T> a = rhs0[i], b = rh[i];
    rh[i] = C<T>{static_cast<T>((static_cast<double>(a.re) + b.re) / den),
                 static_cast<T>((static_cast<double>(a.im) + b.im) / den)};
  }
}

// x <- x * f
template <typename T>
__global__ void __launch_bounds__(256) k_scale(C<T>* __restrict__ x, int64_t n, double f) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const C<T> p = x[i];
    x[i] = C<T>{static_cast<T>(f * p.re), static_cast<T>(f * p.im)};
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

// x <- x / sqrt(cell * sum)
template <typename T>
__global__ void __launch_bounds__(256) k_normalise(C<T>* __restrict__ x, int64_t n, const double* __restrict__ red,
                                                   int nblocks, double cell) {
  __shared__ double f;
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int b = 0; b < nblocks; ++b) s += red[b * 4];
    f = 1.0 / sqrt(cell * s);
  }
  __syncthreads();
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const C<T> p = x[i];
    x[i] = C<T>{static_cast<T>(f * p.re), static_cast<T>(f * p.im)};
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

// In-place complex 3D FFT of an unpadded N0 x N1 x N2 grid.
template <typename T, int SIGN>
static hipError_t fft3_full(DevicePlan& P, C<T>* X, hipStream_t s) {
  const HostTables& H = P.H;
  const C<T>* tw2 = reinterpret_cast<const C<T>*>(P.twiddles[ilog2(H.N[2])]);
  DDI_CHECK((launch_contig<T, SIGN, C2C>(H.N[2], X, X, H.N[0], H.N[1], H.N[0], H.N[1], H.N[2], nullptr, nullptr,
                                         nullptr, tw2, s)));
  DDI_CHECK((launch_strided<T, SIGN>(H.N[1], X, 1, H.N[0], H.N[1], H.N[2], H.N[0], 0, H.N[1], 0, 0,
                                     reinterpret_cast<const C<T>*>(P.twiddles[ilog2(H.N[1])]), s)));
  if (H.N[0] > 1) {
    DDI_CHECK((launch_strided<T, SIGN>(H.N[0], X, 0, H.N[0], H.N[1], H.N[2], H.N[1], 0, H.N[0], 0, 0,
                                       reinterpret_cast<const C<T>*>(P.twiddles[ilog2(H.N[0])]), s)));
  }
  return hipSuccess;
}

static int ew_blocks(int64_t n) {
  int64_t b = (n + 255) / 256;
  return static_cast<int>(b > 16384 ? 16384 : b);
}

template <typename T>
hipError_t run_gpe_energy_grad(DevicePlan& P, const gpe_params& gp, const Complex<T>* psi, double* E_dev,
                               Complex<T>* grad, hipStream_t s) {
  const HostTables& H = P.H;
  const int64_t n = static_cast<int64_t>(H.N[0]) * H.N[1] * H.N[2];
  const GridGeo G = geo_of(H, gp);
  const double inv_ntot = 1.0 / static_cast<double>(n);
  const int nb = P.gpe_red_blocks;
  T* rho = reinterpret_cast<T*>(P.gpe_rho);
  T* phi = reinterpret_cast<T*>(P.gpe_phi);
  T* phit = reinterpret_cast<T*>(P.gpe_phit);
  C<T>* c1 = reinterpret_cast<C<T>*>(P.gpe_c1);
  const T* Vext = reinterpret_cast<const T*>(gp.V_dev);
  double* red_kin = P.gpe_red;
  double* red_terms = P.gpe_red + 4 * nb;
  hipLaunchKernelGGL((k_density<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi, rho, n);
  DDI_CHECK(hipGetLastError());
  DDI_CHECK(run_apply<T>(P, rho, phi, +1, s, nullptr));
  hipLaunchKernelGGL((k_copy<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi, c1, n);
  DDI_CHECK(hipGetLastError());
  DDI_CHECK((fft3_full<T, -1>(P, c1, s)));
  hipLaunchKernelGGL((k_kinetic<T>), dim3(nb), dim3(kRedThreads), 0, s, c1, n, G, inv_ntot, red_kin);
  DDI_CHECK(hipGetLastError());
  hipLaunchKernelGGL((k_energy_terms<T>), dim3(nb), dim3(kRedThreads), 0, s, rho, phi, Vext, n, G, red_terms);
  DDI_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_energy_final, dim3(1), dim3(64), 0, s, red_kin, red_terms, nb, H.cell, inv_ntot, gp.beta,
                     gp.lambda, E_dev);
  DDI_CHECK(hipGetLastError());
  if (grad) {
    DDI_CHECK(run_apply<T>(P, rho, phit, -1, s, nullptr));
    DDI_CHECK((fft3_full<T, +1>(P, c1, s)));     // c1 = -1/2 Lap psi
    hipLaunchKernelGGL((k_grad<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi, c1, rho, phi, phit, Vext, n, G, H.cell,
                       gp.beta, gp.lambda, grad);
    DDI_CHECK(hipGetLastError());
  }
  return hipSuccess;
}

template <typename T>
hipError_t run_gf_step(DevicePlan& P, const gpe_params& gp, double dt, int n_inner, const Complex<T>* psi_in,
                       Complex<T>* psi_out, hipStream_t s) {
  const HostTables& H = P.H;
  const int64_t n = static_cast<int64_t>(H.N[0]) * H.N[1] * H.N[2];
  const GridGeo G = geo_of(H, gp);
  const double inv_ntot = 1.0 / static_cast<double>(n);
  const int nb = P.gpe_red_blocks;
  T* rho = reinterpret_cast<T*>(P.gpe_rho);
  T* phi = reinterpret_cast<T*>(P.gpe_phi);
  T* Bc = reinterpret_cast<T*>(P.gpe_phit);
  C<T>* rhs0 = reinterpret_cast<C<T>*>(P.gpe_c1);
  C<T>* r = reinterpret_cast<C<T>*>(P.gpe_c2);
  const T* Vext = reinterpret_cast<const T*>(gp.V_dev);
  double* red = P.gpe_red;
  double* scal = P.gpe_red + 8 * nb;
  hipLaunchKernelGGL((k_density<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi_in, rho, n);
  DDI_CHECK(hipGetLastError());
  DDI_CHECK(run_apply<T>(P, rho, phi, +1, s, nullptr));
  hipLaunchKernelGGL((k_gf_coeff<T>), dim3(nb), dim3(kRedThreads), 0, s, rho, phi, Vext, n, G, gp.beta, gp.lambda,
                     Bc, red);
  DDI_CHECK(hipGetLastError());
  hipLaunchKernelGGL(k_gf_alpha, dim3(1), dim3(64), 0, s, red, nb, scal);
  DDI_CHECK(hipGetLastError());
  // rhs0 = FFT(psi_in) / dt
  hipLaunchKernelGGL((k_copy<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi_in, rhs0, n);
  DDI_CHECK(hipGetLastError());
  DDI_CHECK((fft3_full<T, -1>(P, rhs0, s)));
  hipLaunchKernelGGL((k_scale<T>), dim3(ew_blocks(n)), dim3(256), 0, s, rhs0, n, 1.0 / dt);
  DDI_CHECK(hipGetLastError());
  if (psi_out != psi_in) {
    hipLaunchKernelGGL((k_copy<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi_in, psi_out, n);
    DDI_CHECK(hipGetLastError());
  }
  for (int it = 0; it < n_inner; ++it) {
    hipLaunchKernelGGL((k_gf_residual<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi_out, Bc, scal, n, r);
    DDI_CHECK(hipGetLastError());
    DDI_CHECK((fft3_full<T, -1>(P, r, s)));
    hipLaunchKernelGGL((k_gf_solve<T>), dim3(ew_blocks(n)), dim3(256), 0, s, r, rhs0, scal, n, G, dt, inv_ntot);
    DDI_CHECK(hipGetLastError());
    DDI_CHECK((fft3_full<T, +1>(P, r, s)));
    hipLaunchKernelGGL((k_copy<T>), dim3(ew_blocks(n)), dim3(256), 0, s, r, psi_out, n);
    DDI_CHECK(hipGetLastError());
  }
  hipLaunchKernelGGL((k_norm2<T>), dim3(nb), dim3(kRedThreads), 0, s, psi_out, n, red);
  DDI_CHECK(hipGetLastError());
  hipLaunchKernelGGL((k_normalise<T>), dim3(ew_blocks(n)), dim3(256), 0, s, psi_out, n, red, nb, H.cell);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t run_type2<double>(DevicePlan&, const double*, Complex<double>*, const double*, double, int,
                                      hipStream_t, hipEvent_t*);
template hipError_t run_type2<float>(DevicePlan&, const float*, Complex<float>*, const double*, double, int,
                                     hipStream_t, hipEvent_t*);
template hipError_t run_type1<double>(DevicePlan&, const Complex<double>*, double*, int, hipStream_t, hipEvent_t*);
template hipError_t run_type1<float>(DevicePlan&, const Complex<float>*, float*, int, hipStream_t, hipEvent_t*);
template hipError_t run_apply<double>(DevicePlan&, const double*, double*, int, hipStream_t, hipEvent_t*);
template hipError_t run_apply<float>(DevicePlan&, const float*, float*, int, hipStream_t, hipEvent_t*);
template hipError_t run_gpe_energy_grad<double>(DevicePlan&, const gpe_params&, const Complex<double>*, double*,
                                                Complex<double>*, hipStream_t);
template hipError_t run_gpe_energy_grad<float>(DevicePlan&, const gpe_params&, const Complex<float>*, double*,
                                               Complex<float>*, hipStream_t);
template hipError_t run_gf_step<double>(DevicePlan&, const gpe_params&, double, int, const Complex<double>*,
                                        Complex<double>*, hipStream_t);
template hipError_t run_gf_step<float>(DevicePlan&, const gpe_params&, double, int, const Complex<float>*,
                                       Complex<float>*, hipStream_t);
template int gpe_reduction_blocks<double>(const DevicePlan&);
template int gpe_reduction_blocks<float>(const DevicePlan&);

}  // namespace ddi
