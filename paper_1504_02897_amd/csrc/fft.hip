// Batched 1D FFT passes on gfx950 (wave64): Stockham radix-4/8/16 with the
// butterflies in registers and one LDS exchange per pass.  Lines along the
// last (contiguous) axis fuse the NUFFT prologue (deconvolution, zero padding)
// or epilogue (truncation, deconvolution, real part); lines along the strided
// axes are processed in bundles of consecutive last-axis indices so that every
// global access is coalesced, and skip the zero (input) or unused (output)
// half of the oversampled line.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "fft.h"
#include "fft_regs.h"

namespace ddi {

#ifndef DDI_STRIDED_SEG
#define DDI_STRIDED_SEG 128
#endif
#ifndef DDI_STRIDED_THREADS
#define DDI_STRIDED_THREADS 1024
#endif
#ifndef DDI_CONTIG_THREADS
#define DDI_CONTIG_THREADS 256
#endif
// Launch shapes (measured optima): strided passes bundle lines until a row segment along the last
// axis has kStridedSeg bytes (at most kStridedThreads threads); contiguous passes run
// kContigThreads threads per workgroup.
constexpr int kStridedSeg = DDI_STRIDED_SEG;
constexpr int kStridedThreads = DDI_STRIDED_THREADS;
constexpr int kContigThreads = DDI_CONTIG_THREADS;
#ifndef DDI_CONTIG_BLOCKS
#define DDI_CONTIG_BLOCKS -1
#endif
#ifndef DDI_CONTIG_WAVESYNC
#define DDI_CONTIG_WAVESYNC 1
#endif
// Workgroups of a contiguous pass: each loops over line groups with the next group's loads in
// flight during this group's transform and stores.  -1: a quarter as many as there are line
// groups, at least 512 (or all of them) and at most 1024; 0: one per line group; n > 0: n.
// Wave-local LDS barriers where a line lies inside one wave.
constexpr int kContigBlocks = DDI_CONTIG_BLOCKS;

#ifndef DDI_STRIDED_BLOCKS
#define DDI_STRIDED_BLOCKS -1
#endif
// Workgroups of a strided pass, each looping over line bundles with the next bundle's loads in
// flight.  -1: 131072 threads' worth, clamped to [256, 512] workgroups (512 of 256 threads, 256
// of 1024); 0: one per bundle; n > 0: n.
constexpr int kStridedBlocks = DDI_STRIDED_BLOCKS;
constexpr bool kContigWaveSync = DDI_CONTIG_WAVESYNC != 0;

// ------------------------------------------------------------------ radix plans
template <int N> struct RadixPlan;
template <> struct RadixPlan<8> { static constexpr int R1 = 8, R2 = 1, R3 = 1, R4 = 1; };
template <> struct RadixPlan<16> { static constexpr int R1 = 4, R2 = 4, R3 = 1, R4 = 1; };
template <> struct RadixPlan<32> { static constexpr int R1 = 8, R2 = 4, R3 = 1, R4 = 1; };
template <> struct RadixPlan<64> { static constexpr int R1 = 8, R2 = 8, R3 = 1, R4 = 1; };
template <> struct RadixPlan<128> { static constexpr int R1 = 16, R2 = 8, R3 = 1, R4 = 1; };
template <> struct RadixPlan<256> { static constexpr int R1 = 16, R2 = 16, R3 = 1, R4 = 1; };
template <> struct RadixPlan<512> { static constexpr int R1 = 8, R2 = 8, R3 = 8, R4 = 1; };
template <> struct RadixPlan<1024> { static constexpr int R1 = 16, R2 = 16, R3 = 4, R4 = 1; };
// lengths 3 * 2^a: the first radix carries the factor 3 (the later ones must divide it); 384 and
// 768 take a fourth pass instead of a first radix of 24
template <> struct RadixPlan<12> { static constexpr int R1 = 12, R2 = 1, R3 = 1, R4 = 1; };
template <> struct RadixPlan<24> { static constexpr int R1 = 12, R2 = 2, R3 = 1, R4 = 1; };
template <> struct RadixPlan<48> { static constexpr int R1 = 12, R2 = 4, R3 = 1, R4 = 1; };
template <> struct RadixPlan<96> { static constexpr int R1 = 12, R2 = 4, R3 = 2, R4 = 1; };
template <> struct RadixPlan<192> { static constexpr int R1 = 12, R2 = 4, R3 = 4, R4 = 1; };
template <> struct RadixPlan<384> { static constexpr int R1 = 12, R2 = 4, R3 = 4, R4 = 2; };
template <> struct RadixPlan<768> { static constexpr int R1 = 12, R2 = 4, R3 = 4, R4 = 4; };
// Plan per element type and pass kind: FP64 256-point lines use radix 8 x 8 x 4 (eight values
// per thread: half the registers of radix 16, one more LDS exchange).  In the looping strided
// passes the next bundle's prefetched values double the registers, so radix 16 leaves one wave
// per SIMD there; FP32 strided lines keep radix 16 x 16 (measured faster).
template <typename T, int N, bool CONTIG> struct Radix : RadixPlan<N> {};
template <> struct Radix<double, 256, true> { static constexpr int R1 = 8, R2 = 8, R3 = 4, R4 = 1; };
template <> struct Radix<double, 256, false> { static constexpr int R1 = 8, R2 = 8, R3 = 4, R4 = 1; };

// FP64 lines of up to 512 points exchange the real parts through LDS, then the imaginary
// parts: half the LDS footprint of a line (twice the resident lines per CU) for the same
// bytes moved.
template <typename T, int N>
struct SplitExchange {
  static constexpr bool value = sizeof(T) == 8 && N <= 512;   // measured slower for 1024-point lines
};
template <typename T, int N>
using LdsElem = typename std::conditional<SplitExchange<T, N>::value, T, C<T>>::type;

// Barrier between the LDS writes and reads of an exchange: the whole workgroup, or (WAVE) only
// the wave, when every line lies inside one wave (LDS operations of a wave complete in order;
// the fences keep the compiler from moving them across the barrier).
template <bool WAVE>
__device__ __forceinline__ void lds_sync() {
  if constexpr (WAVE) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  } else {
    __syncthreads();
  }
}

// One LDS exchange between radix passes: the thread's R1 values (grouped for radix Rs,
// written with stride Ns) are stored, then regathered for radix Rl.  On exit v holds the
// raw (untwiddled) inputs of the next pass.
template <typename T, int N, int R1, int Rs, int Rl, bool WAVE = false, typename Addr>
__device__ __forceinline__ void stockham_exchange(LdsElem<T, N>* lds, Addr addr, int j0, int Ns, C<T>* v) {
  constexpr int TL = N / R1;
  if constexpr (SplitExchange<T, N>::value) {
    T keep[R1];
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
      for (int b = 0; b < R1 / Rs; ++b) {
        const int j = j0 + TL * b;
        const int idxD = (j / Ns) * Ns * Rs + (j % Ns);
#pragma unroll
        for (int r = 0; r < Rs; ++r) lds[addr(idxD + r * Ns)] = part == 0 ? v[b * Rs + r].re : v[b * Rs + r].im;
      }
      lds_sync<WAVE>();
#pragma unroll
      for (int b = 0; b < R1 / Rl; ++b) {
        const int j = j0 + TL * b;
#pragma unroll
        for (int r = 0; r < Rl; ++r) {
          const T x = lds[addr(j + r * (N / Rl))];
          if (part == 0) keep[b * Rl + r] = x;
          else v[b * Rl + r] = C<T>{keep[b * Rl + r], x};
        }
      }
      if (part == 0) lds_sync<WAVE>();
    }
  } else {
#pragma unroll
    for (int b = 0; b < R1 / Rs; ++b) {
      const int j = j0 + TL * b;
      const int idxD = (j / Ns) * Ns * Rs + (j % Ns);
#pragma unroll
      for (int r = 0; r < Rs; ++r) lds[addr(idxD + r * Ns)] = v[b * Rs + r];
    }
    lds_sync<WAVE>();
#pragma unroll
    for (int b = 0; b < R1 / Rl; ++b) {
      const int j = j0 + TL * b;
#pragma unroll
      for (int r = 0; r < Rl; ++r) v[b * Rl + r] = lds[addr(j + r * (N / Rl))];
    }
  }
}

// Twiddles and radix-R DFTs of one Stockham pass (Ns = product of the earlier radices) on
// the thread's R1 values.
template <typename T, int N, int R1, int R, int SIGN>
__device__ __forceinline__ void stockham_compute(int j0, int Ns, const C<T>* __restrict__ tw, C<T>* v) {
  constexpr int TL = N / R1;
#pragma unroll
  for (int b = 0; b < R1 / R; ++b) {
    const int jm = (j0 + TL * b) % Ns;
#pragma unroll
    for (int r = 1; r < R; ++r) {
      C<T> w = tw[r * jm * (N / (Ns * R))];      // r jm < Ns R: the index stays below N
      if (SIGN > 0) w.im = -w.im;
      v[b * R + r] = cmul(v[b * R + r], w);
    }
    dft_any<T, R, SIGN>(v + b * R);
  }
}

// Full line FFT.  On entry v[r] = x[j0 + r*TL] (r < R1).  On exit the thread
// holds the outputs k = j + r*(N/Rlast), j = j0 + TL*b, in v[b*Rlast + r].
template <typename T, int N, int SIGN, typename P, bool WAVE = false, typename Addr>
__device__ __forceinline__ void line_fft(LdsElem<T, N>* lds, Addr addr, int j0, const C<T>* __restrict__ tw, C<T>* v) {
  dft_any<T, P::R1, SIGN>(v);
  if constexpr (P::R2 > 1) {
    stockham_exchange<T, N, P::R1, P::R1, P::R2, WAVE>(lds, addr, j0, 1, v);
    stockham_compute<T, N, P::R1, P::R2, SIGN>(j0, P::R1, tw, v);
    if constexpr (P::R3 > 1) {
      lds_sync<WAVE>();
      stockham_exchange<T, N, P::R1, P::R2, P::R3, WAVE>(lds, addr, j0, P::R1, v);
      stockham_compute<T, N, P::R1, P::R3, SIGN>(j0, P::R1 * P::R2, tw, v);
      if constexpr (P::R4 > 1) {
        lds_sync<WAVE>();
        stockham_exchange<T, N, P::R1, P::R3, P::R4, WAVE>(lds, addr, j0, P::R1 * P::R2, v);
        stockham_compute<T, N, P::R1, P::R4, SIGN>(j0, P::R1 * P::R2 * P::R3, tw, v);
      }
    }
  }
}

template <typename P, int N>
struct LineOut {
  static constexpr int RL = P::R4 > 1 ? P::R4 : (P::R3 > 1 ? P::R3 : (P::R2 > 1 ? P::R2 : P::R1));
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


// ------------------------------------------------------------------ strided-axis FFT pass
// Lines along axis `axis` (0 or 1) of a [d0][d1][d2] complex array, B consecutive
// z per workgroup.  The other non-z axis runs over n_o lines (compact when
// o_compact: index o -> fine index fmap(o, d_o, n_o)).  in_compact / out_compact:
// only the nc_axis / nc_out active positions of the line are read (rest zero) / written.
template <typename T, int N, int SIGN, int MAXT, bool PF>
__global__ void __launch_bounds__(MAXT) k_fft_strided(C<T>* __restrict__ F, int axis, int d0, int d1, int d2,
                                                     int n_o, int o_compact, int nc_axis, int in_compact,
                                                     int out_compact, int nc_out, int z0, int nzb,
                                                     const C<T>* __restrict__ tw, int B) {
  extern __shared__ unsigned char smem_raw[];
  LdsElem<T, N>* lds = reinterpret_cast<LdsElem<T, N>*>(smem_raw);
  using P = Radix<T, N, false>;
  constexpr int TL = N / P::R1;
  const int b = threadIdx.x % B;
  const int j0 = threadIdx.x / B;
  const int d_o = axis == 0 ? d1 : d0;
  const int nblk = n_o * nzb;
  const int64_t stride = axis == 0 ? static_cast<int64_t>(d1) * d2 : d2;
  // first element of the thread's line in line bundle blk
  auto line_base = [&](int blk) -> int64_t {
    const int o = blk / nzb;
    const int z = (z0 + (blk % nzb) * B) % d2 + b;   // z0 is a multiple of B
    const int of = o_compact ? fmap(o, d_o, n_o) : o;
    return axis == 0 ? static_cast<int64_t>(of) * d2 + z : static_cast<int64_t>(of) * d1 * d2 + z;
  };
  auto load = [&](int64_t base, C<T>* v) {
#pragma unroll
    for (int r = 0; r < P::R1; ++r) {
      const int k = j0 + r * TL;
      if (in_compact && !active(k, N, nc_axis)) v[r] = C<T>{0, 0};
      else v[r] = F[base + k * stride];
    }
  };
  auto addr = [B, b](int k) { return k * B + b; };
  // bundles blockIdx.x, blockIdx.x + gridDim.x, ...: with PF the next bundle's loads are in flight
  // during this bundle's transform and stores (bundles are disjoint sets of lines); without, the
  // grid covers every bundle once (no second register set)
  int blk = blockIdx.x;
  int64_t base = line_base(blk);
  C<T> v[P::R1];
  load(base, v);
  for (;;) {
    const int nb = blk + static_cast<int>(gridDim.x);
    C<T> nx[PF ? P::R1 : 1];
    int64_t nbase = 0;
    if (PF && nb < nblk) {
      nbase = line_base(nb);
      load(nbase, nx);
    }
    line_fft<T, N, SIGN, P>(lds, addr, j0, tw, v);
#pragma unroll
    for (int i = 0; i < P::R1; ++i) {
      const int k = LineOut<P, N>::k(j0, i);
      if (!out_compact || active(k, N, nc_out)) F[base + k * stride] = v[i];
    }
    if (!PF || nb >= nblk) break;
#pragma unroll
    for (int r = 0; r < (PF ? P::R1 : 1); ++r) v[r] = nx[r];
    base = nbase;
    blk = nb;
    __syncthreads();                         // the last exchange's reads precede the next writes
  }
}

// ------------------------------------------------------------------ split: axis-0 pass with the symbol
// Moves a line from the output distribution of line_fft (thread j0 holds k = LineOut::k(j0, i)
// in v[i]) to its input distribution (v[r] = x[j0 + r*TL]) through LDS, in place: every value of
// a component is stored before any is read back, so no second array is held.  Ends with a
// barrier, so the next line_fft may write LDS at once.
template <typename T, int N, typename P, typename Addr>
__device__ __forceinline__ void line_to_natural(LdsElem<T, N>* lds, Addr addr, int j0, C<T>* v) {
  constexpr int TL = N / P::R1;
  if constexpr (SplitExchange<T, N>::value) {
#pragma unroll
    for (int part = 0; part < 2; ++part) {
      __syncthreads();
#pragma unroll
      for (int i = 0; i < P::R1; ++i) lds[addr(LineOut<P, N>::k(j0, i))] = part == 0 ? v[i].re : v[i].im;
      __syncthreads();
#pragma unroll
      for (int r = 0; r < P::R1; ++r) {
        const T x = lds[addr(j0 + r * TL)];
        if (part == 0) v[r].re = x;
        else v[r].im = x;
      }
    }
  } else {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < P::R1; ++i) lds[addr(LineOut<P, N>::k(j0, i))] = v[i];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < P::R1; ++r) v[r] = lds[addr(j0 + r * TL)];
  }
  __syncthreads();
}

// Radices of the symbol pass: eight values per thread from 128 points up, so that two
// transforms, the symbol and the exchange fit in 128 VGPRs (four waves per SIMD; with sixteen
// FP64 values per thread the kernel spills or runs one wave per SIMD).
template <int N> struct SymbolRadix : RadixPlan<N> {};
template <> struct SymbolRadix<128> { static constexpr int R1 = 8, R2 = 4, R3 = 4, R4 = 1; };
template <> struct SymbolRadix<256> { static constexpr int R1 = 8, R2 = 8, R3 = 4, R4 = 1; };

// Lines (., y, z) of the padded spectrum for y in [0, d1) and z in [0, nz); B consecutive z per
// workgroup.  See launch_symbol.
template <typename T, int N, int MAXT>
__global__ void __launch_bounds__(MAXT, 1024 / MAXT) k_fft_symbol(C<T>* __restrict__ F, int d1, int d2, int nc_axis, int nzb,
                                                    SplitSymbol sp, const C<T>* __restrict__ tw, int B) {
  extern __shared__ unsigned char smem_raw[];
  LdsElem<T, N>* lds = reinterpret_cast<LdsElem<T, N>*>(smem_raw);
  using P = SymbolRadix<N>;
  constexpr int TL = N / P::R1;
  const int b = threadIdx.x % B;
  const int j0 = threadIdx.x / B;
  const int y = blockIdx.x / nzb;
  const int z = (blockIdx.x % nzb) * B + b;
  const int64_t base = static_cast<int64_t>(y) * d2 + z;
  const int64_t stride = static_cast<int64_t>(d1) * d2;
  auto addr = [B, b](int k) { return k * B + b; };
  // the multiplier of each output mode this thread will hold, evaluated before the line is
  // loaded (the transcendental work then does not overlap the transform's live values)
  // modes: m1 signed from y (Nyquist plane y = d1/2 dropped); m2 = z in [0, d2/2)
  const bool nyq1 = 2 * y == d1;
  const double k1 = (y < d1 / 2 ? y : y - d1) * sp.dk[1];
  const double k2 = z * sp.dk[2];
  const double w2 = z == 0 ? sp.scale : 2.0 * sp.scale;
  const double kn12 = k1 * sp.n[1] + k2 * sp.n[2];
  const double km12 = k1 * sp.m[1] + k2 * sp.m[2];
  const double u12 = k1 * k1 + k2 * k2;
  double mult[P::R1];
#pragma unroll
  for (int i = 0; i < P::R1; ++i) {
    const int k = LineOut<P, N>::k(j0, i);
    const double k0 = (k < N / 2 ? k : k - N) * sp.dk[0];
    const double u = k0 * k0 + u12;
    mult[i] = 0.0;
    if (!nyq1 && 2 * k != N && u > 0.0) {
      const double kn = k0 * sp.n[0] + kn12;
      const double km = k0 * sp.m[0] + km12;
      if (sp.dim == 3) {
        mult[i] = -expm1(-u * sp.inv_s2) * (3.0 * kn * km / u - sp.nm) * w2;
      } else {
        const double kk = sqrt(u);
        mult[i] = erf(kk * sp.inv_s) * (1.5 * (kn * km - sp.n3m3 * u) / kk) * w2;
      }
    }
  }
  C<T> v[P::R1];
#pragma unroll
  for (int r = 0; r < P::R1; ++r) {
    const int k = j0 + r * TL;
    v[r] = active(k, N, nc_axis) ? F[base + k * stride] : C<T>{0, 0};
  }
  line_fft<T, N, -1, P>(lds, addr, j0, tw, v);
#pragma unroll
  for (int i = 0; i < P::R1; ++i)
    v[i] = C<T>{static_cast<T>(v[i].re * mult[i]), static_cast<T>(v[i].im * mult[i])};
  line_to_natural<T, N, P>(lds, addr, j0, v);
  line_fft<T, N, 1, P>(lds, addr, j0, tw, v);
#pragma unroll
  for (int i = 0; i < P::R1; ++i) {
    const int k = LineOut<P, N>::k(j0, i);
    if (active(k, N, nc_axis)) F[base + k * stride] = v[i];
  }
}

// ------------------------------------------------------------------ last-axis (contiguous) FFT pass


// Lines along axis 2.  Line l -> (o0, o1); in R2C_PAD / C2R_TRUNC modes (o0, o1)
// run over the compact N0 x N1 grid and map to fine indices; in C2C they run
// over d0 x d1 directly.  R2C_PAD: input real rho[N0][N1][N2] times the
// deconvolution factors, placed at the active positions of a length-N line,
// output complex line.  C2R_TRUNC: input complex line, output
// Re(line[fmap(c2)]) times the deconvolution factors into phi[N0][N1][N2].
template <typename T, int N, int SIGN, int MODE, bool PF>
__global__ void __launch_bounds__(kContigThreads) k_fft_contig(const void* in, void* out,
                                                    int n0, int n1, int d0, int d1, int nc2, int z0, int nz,
                                                    const double* __restrict__ D0, const double* __restrict__ D1,
                                                    const double* __restrict__ D2,
                                                    const C<T>* __restrict__ tw, int B, int nlines, GfLoad gl) {
  extern __shared__ unsigned char smem_raw[];
  LdsElem<T, N>* lds = reinterpret_cast<LdsElem<T, N>*>(smem_raw);
  using P = Radix<T, N, true>;
  constexpr bool kGf = MODE == C2C_GF_RES || MODE == C2C_GF_SOLVE || MODE == C2C_TS_KIN;
  constexpr int TL = N / P::R1;
  constexpr bool kWave = kContigWaveSync && 64 % TL == 0;   // every line inside one wave
  constexpr int LS = N + N / P::R1;      // padded line stride in LDS
  const int j0 = threadIdx.x % TL;
  const int lb = threadIdx.x / TL;
  const int ngroups = (nlines + B - 1) / B;
  LdsElem<T, N>* my = lds + lb * LS;
  auto addr = [](int k) { return k + k / Radix<T, N, true>::R1; };
  // Deconvolution factors along the last axis at the thread's positions (inputs for R2C_PAD,
  // outputs for C2R_*): the same for every line, loaded once.  The line's factor D0 D1 is loaded
  // with the line's inputs and applied only when the line is transformed or stored, so that a
  // prefetched group's loads are not waited for ahead of the current group's transform.
  constexpr bool kIn = MODE == R2C_PAD, kOut = MODE == C2R_TRUNC || MODE == C2R_ADD;
  double d2f[(kIn || kOut) ? P::R1 : 1];
  if constexpr (kIn || kOut) {
#pragma unroll
    for (int r = 0; r < P::R1; ++r) {
      const int k = kIn ? j0 + r * TL : LineOut<P, N>::k(j0, r);
      d2f[r] = active(k, N, nc2) ? D2[cmap(k, N, nc2)] : 0.0;
    }
  }
  // the thread's raw inputs of line group g (zeros outside the line's active or windowed
  // positions) and the line's D0, D1
  auto load = [&](int g, C<T>* v, double* f01) {
    const int line = g * B + lb;
    const bool valid = line < nlines;
    const int o0 = valid ? line / n1 : 0;
    const int o1 = valid ? line % n1 : 0;
    if constexpr (kIn || kOut) {
      f01[0] = D0[o0];
      f01[1] = D1[o1];
    }
    if (MODE == R2C_PAD) {
      const T* rho = reinterpret_cast<const T*>(in);
      const int64_t rb = (static_cast<int64_t>(o0) * n1 + o1) * nc2;
#pragma unroll
      for (int r = 0; r < P::R1; ++r) {
        const int k = j0 + r * TL;
        v[r] = valid && active(k, N, nc2) ? C<T>{rho[rb + cmap(k, N, nc2)], T(0)} : C<T>{0, 0};
      }
    } else if constexpr (kGf) {
      const C<T>* F = reinterpret_cast<const C<T>*>(in);
      const int64_t lbase = static_cast<int64_t>(valid ? line : 0) * N;
      if constexpr (MODE == C2C_TS_KIN) {
        const double pa = o0 < gl.n[0] / 2 ? o0 : o0 - gl.n[0];
        const double pb = o1 < gl.n[1] / 2 ? o1 : o1 - gl.n[1];
        const double ma = M_PI * pa / gl.L[0], mb = M_PI * pb / gl.L[1];
        const double mab = (gl.n[0] > 1 ? ma * ma : 0.0) + mb * mb;
#pragma unroll
        for (int r = 0; r < P::R1; ++r) {
          const int k = j0 + r * TL;
          const double pc = k < N / 2 ? k : k - N;
          const double mc = M_PI * pc / gl.L[2];
          double sn, cs;
          sincos(gl.qdt * (mab + mc * mc), &sn, &cs);   // exp(-i a) = cos a - i sin a
          const C<T> x = F[lbase + k];
          const double re = static_cast<double>(x.re), im = static_cast<double>(x.im);
          v[r] = C<T>{static_cast<T>((re * cs + im * sn) * gl.inv_ntot), static_cast<T>((im * cs - re * sn) * gl.inv_ntot)};
        }
        return;
      }
      const double alpha = *gl.alpha;
      if constexpr (MODE == C2C_GF_RES) {
        const T* Bg = reinterpret_cast<const T*>(gl.aux);
#pragma unroll
        for (int r = 0; r < P::R1; ++r) {
          const int k = j0 + r * TL;
          const double f = alpha - static_cast<double>(Bg[lbase + k]);
          const C<T> p = F[lbase + k];
          v[r] = C<T>{static_cast<T>(f * p.re), static_cast<T>(f * p.im)};
        }
      } else {
        const C<T>* R0 = reinterpret_cast<const C<T>*>(gl.aux);
        const double pa = o0 < gl.n[0] / 2 ? o0 : o0 - gl.n[0];
        const double pb = o1 < gl.n[1] / 2 ? o1 : o1 - gl.n[1];
        const double ma = M_PI * pa / gl.L[0], mb = M_PI * pb / gl.L[1];
        const double mab = (gl.n[0] > 1 ? ma * ma : 0.0) + mb * mb;
#pragma unroll
        for (int r = 0; r < P::R1; ++r) {
          const int k = j0 + r * TL;
          const double pc = k < N / 2 ? k : k - N;
          const double mc = M_PI * pc / gl.L[2];
          const double den = (gl.inv_dt + alpha + 0.5 * (mab + mc * mc)) / gl.inv_ntot;
          const C<T> a = R0[lbase + k], b = F[lbase + k];
          v[r] = C<T>{static_cast<T>((gl.inv_dt * a.re + b.re) / den), static_cast<T>((gl.inv_dt * a.im + b.im) / den)};
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
        v[r] = valid && (k - z0 + N) % N < nz ? F[lbase + k] : C<T>{0, 0};
      }
    }
  };
  auto store = [&](int g, const C<T>* v, const double* f01) {
    const int line = g * B + lb;
    if (line >= nlines) return;
    const int o0 = line / n1;
    const int o1 = line % n1;
    if constexpr (kOut) {
      T* phi = reinterpret_cast<T*>(out);
      const double s01 = f01[0] * f01[1];
      const int64_t rb = (static_cast<int64_t>(o0) * n1 + o1) * nc2;
#pragma unroll
      for (int i = 0; i < P::R1; ++i) {
        const int k = LineOut<P, N>::k(j0, i);
        if (active(k, N, nc2)) {
          const T val = static_cast<T>(static_cast<double>(v[i].re) * s01 * d2f[i]);
          if (MODE == C2R_ADD) phi[rb + cmap(k, N, nc2)] += val;
          else phi[rb + cmap(k, N, nc2)] = val;
        }
      }
    } else {
      C<T>* F = reinterpret_cast<C<T>*>(out);
      int64_t lbase;
      if (MODE == C2C || kGf) lbase = static_cast<int64_t>(line) * N;
      else lbase = (static_cast<int64_t>(fmap(o0, d0, n0)) * d1 + fmap(o1, d1, n1)) * N;
#pragma unroll
      for (int i = 0; i < P::R1; ++i) {
        const int k = LineOut<P, N>::k(j0, i);
        if ((k - z0 + N) % N < nz) F[lbase + k] = v[i];
      }
    }
  };
  // line groups blockIdx.x, blockIdx.x + gridDim.x, ...: with PF the next group's loads are in
  // flight during this group's transform and stores; without, the grid covers every group once
  C<T> v[P::R1];
  double f01[2] = {0.0, 0.0};
  int g = blockIdx.x;
  load(g, v, f01);
  for (;;) {
    const int gn = g + static_cast<int>(gridDim.x);
    C<T> nx[PF ? P::R1 : 1];
    double nf01[2] = {0.0, 0.0};
    if (PF && gn < ngroups) load(gn, nx, nf01);
    if constexpr (kIn) {
      const double s01 = f01[0] * f01[1];
#pragma unroll
      for (int r = 0; r < P::R1; ++r) v[r].re = static_cast<T>(static_cast<double>(v[r].re) * s01 * d2f[r]);
    }
    line_fft<T, N, SIGN, P, kWave>(my, addr, j0, tw, v);
    store(g, v, f01);
    if (!PF || gn >= ngroups) break;
#pragma unroll
    for (int r = 0; r < (PF ? P::R1 : 1); ++r) v[r] = nx[r];
    f01[0] = nf01[0];
    f01[1] = nf01[1];
    g = gn;
    lds_sync<kWave>();                       // the last exchange's reads precede the next writes
  }
}

// ------------------------------------------------------------------ dispatch
template <typename T, int N, int SIGN>
static hipError_t launch_strided_n(C<T>* F, int axis, int d0, int d1, int d2, int n_o, int o_compact, int nc,
                                   int in_c, int out_c, int nc_out, int z0, int nz, const C<T>* tw, hipStream_t s) {
  constexpr int TL = N / Radix<T, N, false>::R1;
  // lines per workgroup: at least 256 threads, and row segments of >= 128 B along the
  // contiguous axis (coalescing) as far as 1024 threads and 64 KB of LDS allow; a window
  // of the last axis is covered in blocks of lines that divide its start and length
  int B = 256 / TL;
  while (B * static_cast<int>(sizeof(C<T>)) < kStridedSeg && 2 * B * TL <= kStridedThreads &&
         static_cast<size_t>(2 * B) * N * sizeof(LdsElem<T, N>) <= 65536)
    B *= 2;
  while (B > 1 && static_cast<size_t>(B) * N * sizeof(LdsElem<T, N>) > 65536) B >>= 1;
  while (B > d2) B >>= 1;
  while (B > 1 && (z0 % B != 0 || nz % B != 0)) B >>= 1;
  if (z0 % B != 0 || nz % B != 0 || nz > d2 || z0 < 0 || z0 >= d2) return hipErrorInvalidValue;
  if (n_o < 0 || n_o > (axis == 0 ? d1 : d0) || nc < 0 || nc > N || nc_out < 0 || nc_out > N)
    return hipErrorInvalidValue;
  const size_t shm = static_cast<size_t>(B) * N * sizeof(LdsElem<T, N>);
  const int nzb = nz / B;
  const int nblk = n_o * nzb;
  if (nblk == 0) return hipSuccess;
  const int blocks = kStridedBlocks < 0 ? std::min(nblk, std::max(256, std::min(512, 131072 / (B * TL))))
                     : kStridedBlocks > 0 ? std::min(nblk, kStridedBlocks) : nblk;
  const bool pf = blocks < nblk;
  if (B * TL <= 256 && pf)
    hipLaunchKernelGGL((k_fft_strided<T, N, SIGN, 256, true>), dim3(blocks), dim3(B * TL), shm, s, F, axis, d0, d1,
                       d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nzb, tw, B);
  else if (B * TL <= 256)
    hipLaunchKernelGGL((k_fft_strided<T, N, SIGN, 256, false>), dim3(blocks), dim3(B * TL), shm, s, F, axis, d0, d1,
                       d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nzb, tw, B);
  else if (pf)
    hipLaunchKernelGGL((k_fft_strided<T, N, SIGN, 1024, true>), dim3(blocks), dim3(B * TL), shm, s, F, axis, d0, d1,
                       d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nzb, tw, B);
  else
    hipLaunchKernelGGL((k_fft_strided<T, N, SIGN, 1024, false>), dim3(blocks), dim3(B * TL), shm, s, F, axis, d0, d1,
                       d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nzb, tw, B);
  return hipGetLastError();
}

template <typename T, int SIGN>
hipError_t launch_strided(int n, C<T>* F, int axis, int d0, int d1, int d2, int n_o, int o_compact, int nc,
                                 int in_c, int out_c, int nc_out, int z0, int nz, const C<T>* tw, hipStream_t s) {
  switch (n) {
    case 8: return launch_strided_n<T, 8, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 16: return launch_strided_n<T, 16, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 32: return launch_strided_n<T, 32, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 64: return launch_strided_n<T, 64, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 128: return launch_strided_n<T, 128, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 256: return launch_strided_n<T, 256, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 512: return launch_strided_n<T, 512, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 1024: return launch_strided_n<T, 1024, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 12: return launch_strided_n<T, 12, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 24: return launch_strided_n<T, 24, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 48: return launch_strided_n<T, 48, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 96: return launch_strided_n<T, 96, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 192: return launch_strided_n<T, 192, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 384: return launch_strided_n<T, 384, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    case 768: return launch_strided_n<T, 768, SIGN>(F, axis, d0, d1, d2, n_o, o_compact, nc, in_c, out_c, nc_out, z0, nz, tw, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int N>
static hipError_t launch_symbol_n(C<T>* F, int d1, int d2, int nc, int nz, const SplitSymbol& sp, const C<T>* tw,
                                  hipStream_t s) {
  constexpr int TL = N / SymbolRadix<N>::R1;
  int B = 256 / TL;   // as in the strided pass: >= kStridedSeg-byte row segments where LDS allows
  while (B * static_cast<int>(sizeof(C<T>)) < kStridedSeg && 2 * B * TL <= kStridedThreads &&
         static_cast<size_t>(2 * B) * N * sizeof(LdsElem<T, N>) <= 65536)
    B *= 2;
  while (B > 1 && static_cast<size_t>(B) * N * sizeof(LdsElem<T, N>) > 65536) B >>= 1;
  while (B > 1 && nz % B != 0) B >>= 1;
  if (nz <= 0 || 2 * nz > d2 || nz % B != 0 || nc > N || nc < 1) return hipErrorInvalidValue;
  const size_t shm = static_cast<size_t>(B) * N * sizeof(LdsElem<T, N>);
  const int nzb = nz / B;
  const int blocks = d1 * nzb;
  if (B * TL <= 256)
    hipLaunchKernelGGL((k_fft_symbol<T, N, 256>), dim3(blocks), dim3(B * TL), shm, s, F, d1, d2, nc, nzb, sp, tw, B);
  else
    hipLaunchKernelGGL((k_fft_symbol<T, N, 1024>), dim3(blocks), dim3(B * TL), shm, s, F, d1, d2, nc, nzb, sp, tw, B);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_symbol(int n, C<T>* F, int d1, int d2, int nc, int nz, const SplitSymbol& sp, const C<T>* tw,
                         hipStream_t s) {
  switch (n) {
    case 16: return launch_symbol_n<T, 16>(F, d1, d2, nc, nz, sp, tw, s);
    case 32: return launch_symbol_n<T, 32>(F, d1, d2, nc, nz, sp, tw, s);
    case 64: return launch_symbol_n<T, 64>(F, d1, d2, nc, nz, sp, tw, s);
    case 128: return launch_symbol_n<T, 128>(F, d1, d2, nc, nz, sp, tw, s);
    case 256: return launch_symbol_n<T, 256>(F, d1, d2, nc, nz, sp, tw, s);
    case 512: return launch_symbol_n<T, 512>(F, d1, d2, nc, nz, sp, tw, s);
    case 1024: return launch_symbol_n<T, 1024>(F, d1, d2, nc, nz, sp, tw, s);
    case 12: return launch_symbol_n<T, 12>(F, d1, d2, nc, nz, sp, tw, s);
    case 24: return launch_symbol_n<T, 24>(F, d1, d2, nc, nz, sp, tw, s);
    case 48: return launch_symbol_n<T, 48>(F, d1, d2, nc, nz, sp, tw, s);
    case 96: return launch_symbol_n<T, 96>(F, d1, d2, nc, nz, sp, tw, s);
    case 192: return launch_symbol_n<T, 192>(F, d1, d2, nc, nz, sp, tw, s);
    case 384: return launch_symbol_n<T, 384>(F, d1, d2, nc, nz, sp, tw, s);
    case 768: return launch_symbol_n<T, 768>(F, d1, d2, nc, nz, sp, tw, s);
    default: return hipErrorInvalidValue;
  }
}

template <typename T, int N, int SIGN, int MODE>
static hipError_t launch_contig_n(const void* in, void* out, int n0, int n1, int d0, int d1, int nc2, int z0,
                                  int nz, const double* D0, const double* D1, const double* D2, const C<T>* tw,
                                  hipStream_t s, const GfLoad& gl) {
  if ((MODE == C2C_GF_RES || MODE == C2C_GF_SOLVE) && (gl.aux == nullptr || gl.alpha == nullptr))
    return hipErrorInvalidValue;
  if ((MODE == C2C_GF_RES || MODE == C2C_GF_SOLVE || MODE == C2C_TS_KIN) &&
      (z0 != 0 || nz != N || d0 != n0 || d1 != n1))
    return hipErrorInvalidValue;
  if (z0 < 0 || z0 >= N || nz < 0 || nz > N) return hipErrorInvalidValue;
  constexpr int TL = N / Radix<T, N, true>::R1;
  constexpr int LS = N + N / Radix<T, N, true>::R1;
  int B = kContigThreads / TL;
  if (B < 1) B = 1;
  while (B > 1 && static_cast<size_t>(B) * LS * sizeof(LdsElem<T, N>) > 65536) B >>= 1;
  const int nlines = n0 * n1;
  const size_t shm = static_cast<size_t>(B) * LS * sizeof(LdsElem<T, N>);
  const int ngroups = (nlines + B - 1) / B;
  const int blocks = kContigBlocks < 0 ? std::min(ngroups, std::max(512, std::min(1024, ngroups / 4)))
                     : kContigBlocks > 0 ? std::min(ngroups, kContigBlocks) : ngroups;
  if (blocks < ngroups)
    hipLaunchKernelGGL((k_fft_contig<T, N, SIGN, MODE, true>), dim3(blocks), dim3(B * TL), shm, s, in, out, n0, n1,
                       d0, d1, nc2, z0, nz, D0, D1, D2, tw, B, nlines, gl);
  else
    hipLaunchKernelGGL((k_fft_contig<T, N, SIGN, MODE, false>), dim3(blocks), dim3(B * TL), shm, s, in, out, n0, n1,
                       d0, d1, nc2, z0, nz, D0, D1, D2, tw, B, nlines, gl);
  return hipGetLastError();
}

template <typename T, int SIGN, int MODE>
hipError_t launch_contig(int n, const void* in, void* out, int n0, int n1, int d0, int d1, int nc2, int z0, int nz,
                                const double* D0, const double* D1, const double* D2, const C<T>* tw,
                                hipStream_t s, const GfLoad& gl) {
  switch (n) {
    case 8: return launch_contig_n<T, 8, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 16: return launch_contig_n<T, 16, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 32: return launch_contig_n<T, 32, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 64: return launch_contig_n<T, 64, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 128: return launch_contig_n<T, 128, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 256: return launch_contig_n<T, 256, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 512: return launch_contig_n<T, 512, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 1024: return launch_contig_n<T, 1024, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 12: return launch_contig_n<T, 12, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 24: return launch_contig_n<T, 24, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 48: return launch_contig_n<T, 48, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 96: return launch_contig_n<T, 96, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 192: return launch_contig_n<T, 192, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 384: return launch_contig_n<T, 384, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    case 768: return launch_contig_n<T, 768, SIGN, MODE>(in, out, n0, n1, d0, d1, nc2, z0, nz, D0, D1, D2, tw, s, gl);
    default: return hipErrorInvalidValue;
  }
}

#define DDI_INST_STRIDED(T, S)                                                                                  \
  template hipError_t launch_strided<T, S>(int, C<T>*, int, int, int, int, int, int, int, int, int, int, int, int, \
                                           const C<T>*, hipStream_t);
#define DDI_INST_CONTIG(T, S, M)                                                                                \
  template hipError_t launch_contig<T, S, M>(int, const void*, void*, int, int, int, int, int, int, int,        \
                                             const double*, const double*, const double*, const C<T>*, hipStream_t, \
                                             const GfLoad&);
DDI_INST_STRIDED(double, 1)
DDI_INST_STRIDED(double, -1)
DDI_INST_STRIDED(float, 1)
DDI_INST_STRIDED(float, -1)
DDI_INST_CONTIG(double, 1, R2C_PAD)
DDI_INST_CONTIG(double, -1, R2C_PAD)
DDI_INST_CONTIG(float, 1, R2C_PAD)
DDI_INST_CONTIG(float, -1, R2C_PAD)
DDI_INST_CONTIG(double, 1, C2C)
DDI_INST_CONTIG(double, -1, C2C)
DDI_INST_CONTIG(float, 1, C2C)
DDI_INST_CONTIG(float, -1, C2C)
DDI_INST_CONTIG(double, 1, C2R_TRUNC)
DDI_INST_CONTIG(double, -1, C2R_TRUNC)
DDI_INST_CONTIG(float, 1, C2R_TRUNC)
DDI_INST_CONTIG(float, -1, C2R_TRUNC)
DDI_INST_CONTIG(double, 1, C2R_ADD)
DDI_INST_CONTIG(float, 1, C2R_ADD)
DDI_INST_CONTIG(double, -1, C2C_GF_RES)
DDI_INST_CONTIG(float, -1, C2C_GF_RES)
DDI_INST_CONTIG(double, 1, C2C_GF_SOLVE)
DDI_INST_CONTIG(float, 1, C2C_GF_SOLVE)
DDI_INST_CONTIG(double, 1, C2C_TS_KIN)
DDI_INST_CONTIG(float, 1, C2C_TS_KIN)
template hipError_t launch_symbol<double>(int, C<double>*, int, int, int, int, const SplitSymbol&, const C<double>*,
                                          hipStream_t);
template hipError_t launch_symbol<float>(int, C<float>*, int, int, int, int, const SplitSymbol&, const C<float>*,
                                         hipStream_t);

}  // namespace ddi
