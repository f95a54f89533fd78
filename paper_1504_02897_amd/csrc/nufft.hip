// NUFFT halves of the DDI operator on gfx950 (Sec. 2.1, Eqs. DDI-Con, DDI-Trun1).
//
//   type-2 (grid -> nodes): deconvolve + zero-pad fused into the first FFT pass, pruned
//     3-pass FFT on the oversampled grid, then interpolation at the quadrature nodes with the
//     weights g_q = c_q prod(h) rhohat_q applied at the end.  FP64 interpolation in 3D is
//     tile-owned: per 8 x 8 x 8 tile of the fine grid, the (tile, node) entries of the tile are
//     contracted with the tile as FP64 matrix products (k_interp_mfma), one partial per entry,
//     summed per node by a gather kernel (the fine grid is read once).  Otherwise interpolation
//     is node-owned: nodes grouped by home block read an LDS-staged support region, the rest
//     read the grid directly (one wave per four nodes, compile-time kernel width).
//   type-1 (nodes -> grid): tile-owned spread, no atomics.  In 3D a tile is accumulated in
//     registers by FP64 matrix products over its entries (k_spread_mfma); in 2D a wave owns a
//     tile and sums the nodes staged 64 at a time in LDS as tile-relative weight vectors.  Hot
//     tiles are split into chunks whose partial tiles a reduce kernel sums in a fixed order.
//     Then a pruned 3-pass FFT with truncation, deconvolution and real part fused into the
//     last pass.
//   The operator (one node per +-k pair, all on one side of the last axis) transforms and
//   spreads only the last-axis window that the kept nodes' supports cover.
// Kernel weights are tabulated per node at plan time: nothing transcendental runs per apply.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fft.h"

namespace ddi {

template <typename T>
using C = Complex<T>;

// ------------------------------------------------------------------ interpolation
// A wave interpolates NS = 64/SL nodes at once: SL sub-lanes per node, sub-lane u owning the
// support row z = l0z + u, looping over the (x, y) support; the partial sums of a node are
// then reduced over its SL sub-lanes (log2 SL shuffle steps shared by all NS nodes).
template <int W>
struct InterpShape {
  static constexpr int SL = W <= 4 ? 4 : (W <= 8 ? 8 : 16);
  static constexpr int NS = 64 / SL;
};

// Grouped nodes: the workgroup stages the support region of its group (IB + W - 1 cells
// per axis; 1 on the unused axis of a 2D grid) in LDS once.  Region strides are
// compile-time, so every LDS read uses an immediate offset from one base address.
template <typename T, int W0, int W, int IB, int NT>
__global__ void __launch_bounds__(NT) k_interp_lds(const C<T>* __restrict__ F, const NodeRec<T>* __restrict__ nodes,
                                                    const InterpItem* __restrict__ items, int nf0, int nf1, int nf2,
                                                    const double* __restrict__ scale, double sscalar,
                                                    C<T>* __restrict__ out) {
  constexpr int SL = InterpShape<W>::SL, NS = InterpShape<W>::NS;
  constexpr int R = IB + W - 1;
  constexpr int R0 = W0 == 1 ? 1 : IB + W0 - 1;
  extern __shared__ unsigned char smem_raw[];
  C<T>* reg = reinterpret_cast<C<T>*>(smem_raw);
  // items are pre-ordered so that round-robin dispatch gives each XCD one region of equal work
  const InterpItem it = items[blockIdx.x];
  if (it.count == 0) return;                 // padding item
  for (int i = threadIdx.x; i < R0 * R * R; i += NT) {
    const int rz = i % R;
    const int t = i / R;
    const int ry = t % R, rx = t / R;
    int gx = it.org[0] + rx;
    if (gx >= nf0) gx -= nf0;
    int gy = it.org[1] + ry;
    if (gy >= nf1) gy -= nf1;
    int gz = it.org[2] + rz;
    if (gz >= nf2) gz -= nf2;
    reg[i] = F[(static_cast<uint32_t>(gx) * nf1 + gy) * nf2 + gz];
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int sl = lane / SL, u = lane % SL;
  const bool zin = u < W;
  for (int n0 = wv * NS; n0 < it.count; n0 += (NT / 64) * NS) {
    const int n = n0 + sl;
    const bool valid = n < it.count;
    const int64_t q = static_cast<int64_t>(it.start) + (valid ? n : it.count - 1);
    const NodeRec<T>* nd = nodes + q;
    int lx = nd->l0[0] - it.org[0];
    if (lx < 0) lx += nf0;
    int ly = nd->l0[1] - it.org[1];
    if (ly < 0) ly += nf1;
    int lz = nd->l0[2] - it.org[2];
    if (lz < 0) lz += nf2;
    double wx[W0], wy[W];
#pragma unroll
    for (int i = 0; i < W0; ++i) wx[i] = static_cast<double>(nd->w[0][i]);
#pragma unroll
    for (int i = 0; i < W; ++i) wy[i] = static_cast<double>(nd->w[1][i]);
    const double wz = zin ? static_cast<double>(nd->w[2][u]) : 0.0;
    const C<T>* p = reg + (lx * R + ly) * R + lz + (zin ? u : 0);
    double are = 0.0, aim = 0.0;
#pragma unroll
    for (int iy = 0; iy < W; ++iy) {
      double sre = 0.0, sim = 0.0;
#pragma unroll
      for (int ix = 0; ix < W0; ++ix) {
        const C<T> f = p[ix * R * R + iy * R];
        sre += wx[ix] * static_cast<double>(f.re);
        sim += wx[ix] * static_cast<double>(f.im);
      }
      are += wy[iy] * sre;
      aim += wy[iy] * sim;
    }
    are *= wz;
    aim *= wz;
#pragma unroll
    for (int off = SL / 2; off > 0; off >>= 1) {
      are += __shfl_xor(are, off, 64);
      aim += __shfl_xor(aim, off, 64);
    }
    if (u == 0 && valid) {
      const double s = scale ? scale[q] * sscalar : sscalar;
      out[q] = C<T>{static_cast<T>(s * are), static_cast<T>(s * aim)};
    }
  }
}

// Nodes without enough neighbours in their group block: the same lane layout, reading the
// oversampled grid directly (x-plane and y-row offsets precomputed with the periodic wrap).
template <typename T, int W0, int W>
__global__ void __launch_bounds__(256) k_interp(const C<T>* __restrict__ F, const NodeRec<T>* __restrict__ nodes,
                                                const int32_t* __restrict__ list, int64_t nlist, int nf0, int nf1,
                                                int nf2, const double* __restrict__ scale, double sscalar,
                                                C<T>* __restrict__ out) {
  constexpr int SL = InterpShape<W>::SL, NS = InterpShape<W>::NS;
  const int lane = threadIdx.x & 63;
  const int wv = threadIdx.x >> 6;
  const int sl = lane / SL, u = lane % SL;
  const bool zin = u < W;
  const int blk = xcd_remap(blockIdx.x, gridDim.x);
  const int64_t li = (static_cast<int64_t>(blk) * 4 + wv) * NS + sl;
  const bool valid = li < nlist;
  const int64_t q = list[valid ? li : nlist - 1];
  const NodeRec<T>* nd = nodes + q;
  const int lx = nd->l0[0], ly = nd->l0[1], lz = nd->l0[2];
  double wx[W0], wy[W];
  uint32_t xo[W0];
#pragma unroll
  for (int i = 0; i < W0; ++i) {
    wx[i] = static_cast<double>(nd->w[0][i]);
    int gx = lx + i;
    if (gx >= nf0) gx -= nf0;
    xo[i] = static_cast<uint32_t>(gx) * nf1 * nf2;
  }
#pragma unroll
  for (int i = 0; i < W; ++i) wy[i] = static_cast<double>(nd->w[1][i]);
  const double wz = zin ? static_cast<double>(nd->w[2][u]) : 0.0;
  int gz = lz + (zin ? u : 0);
  if (gz >= nf2) gz -= nf2;
  double are = 0.0, aim = 0.0;
#pragma unroll
  for (int iy = 0; iy < W; ++iy) {
    int gy = ly + iy;
    if (gy >= nf1) gy -= nf1;
    const C<T>* row = F + (static_cast<uint32_t>(gy) * nf2 + gz);
    double sre = 0.0, sim = 0.0;
#pragma unroll
    for (int ix = 0; ix < W0; ++ix) {
      const C<T> f = row[xo[ix]];
      sre += wx[ix] * static_cast<double>(f.re);
      sim += wx[ix] * static_cast<double>(f.im);
    }
    are += wy[iy] * sre;
    aim += wy[iy] * sim;
  }
  are *= wz;
  aim *= wz;
#pragma unroll
  for (int off = SL / 2; off > 0; off >>= 1) {
    are += __shfl_xor(are, off, 64);
    aim += __shfl_xor(aim, off, 64);
  }
  if (u == 0 && valid) {
    const double s = scale ? scale[q] * sscalar : sscalar;
    out[q] = C<T>{static_cast<T>(s * are), static_cast<T>(s * aim)};
  }
}

// ------------------------------------------------------------------ spread
// One wave per work item; tile TX x TY x kTileZ with TX*TY = 64 lanes, each lane owning
// kTileZ points along the last axis in registers.
template <typename T, bool KAHAN, int TX, int TY>
__global__ void __launch_bounds__(64) k_spread(C<T>* __restrict__ F, C<T>* __restrict__ partial,
                                               const NodeRec<T>* __restrict__ nodes, const C<T>* __restrict__ g,
                                               const int32_t* __restrict__ list,
                                               const SpreadItem* __restrict__ items, int nf0, int nf1, int nf2,
                                               int nt1, int nt2, int w0, int w1, int w2) {
  static_assert(TX * TY == 64, "one wave per tile");
  constexpr int TZ = kTileZ;
  constexpr int NB = kSpreadBatch;           // nodes staged per batch
  __shared__ T sx[NB][TX];
  __shared__ T sy[NB][TY];
  __shared__ T sz[NB][TZ];
  __shared__ C<T> sg[NB];
  const int lane = threadIdx.x;
  const SpreadItem it = items[blockIdx.x];
  if (it.tile < 0) return;                   // padding item
  const int tz = it.tile % nt2;
  const int ty = (it.tile / nt2) % nt1;
  const int tx = it.tile / (nt2 * nt1);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  const int lxo = lane / TY, lyo = lane % TY;
  C<T> acc[TZ];
  C<T> cmp[TZ];
#pragma unroll
  for (int i = 0; i < TZ; ++i) {
    acc[i] = C<T>{0, 0};
    cmp[i] = C<T>{0, 0};
  }
  for (int base = 0; base < it.count; base += NB) {
    const int n = it.count - base < NB ? it.count - base : NB;
    // stage the weights of up to 64 nodes restricted to this tile (one node per lane);
    // loads are unconditional (index clamped into the record) so that all are in flight
    if (lane < n) {
      const int q = list[it.start + base + lane];
      const NodeRec<T>* nd = nodes + q;
      const int l0x = nd->l0[0], l0y = nd->l0[1], l0z = nd->l0[2];
      const C<T> gq = g[q];
      int dx = x0 - l0x;
      if (dx < 0) dx += nf0;
      int dy = y0 - l0y;
      if (dy < 0) dy += nf1;
      int dz = z0 - l0z;
      if (dz < 0) dz += nf2;
      T vx[TX], vy[TY], vz[TZ];
#pragma unroll
      for (int i = 0; i < TX; ++i) {
        int d = dx + i;
        if (d >= nf0) d -= nf0;
        vx[i] = nd->w[0][d < kWMax ? d : kWMax - 1];
        vx[i] = d < w0 ? vx[i] : T(0);
      }
#pragma unroll
      for (int i = 0; i < TY; ++i) {
        int d = dy + i;
        if (d >= nf1) d -= nf1;
        vy[i] = nd->w[1][d < kWMax ? d : kWMax - 1];
        vy[i] = d < w1 ? vy[i] : T(0);
      }
#pragma unroll
      for (int i = 0; i < TZ; ++i) {
        int d = dz + i;
        if (d >= nf2) d -= nf2;
        vz[i] = nd->w[2][d < kWMax ? d : kWMax - 1];
        vz[i] = d < w2 ? vz[i] : T(0);
      }
#pragma unroll
      for (int i = 0; i < TX; ++i) sx[lane][i] = vx[i];
#pragma unroll
      for (int i = 0; i < TY; ++i) sy[lane][i] = vy[i];
#pragma unroll
      for (int i = 0; i < TZ; ++i) sz[lane][i] = vz[i];
      sg[lane] = gq;
    }
    __syncthreads();
#pragma unroll DDI_SPREAD_UNROLL
    for (int e = 0; e < n; ++e) {
      const C<T> gq = sg[e];
      T wz[TZ];
#pragma unroll
      for (int i = 0; i < TZ; ++i) wz[i] = sz[e][i];
      const T wxy = sx[e][lxo] * sy[e][lyo];
      const C<T> p = {gq.re * wxy, gq.im * wxy};
#pragma unroll
      for (int i = 0; i < TZ; ++i) {
        if (KAHAN) {
          T yr = p.re * wz[i] - cmp[i].re;
          T tr = acc[i].re + yr;
          cmp[i].re = (tr - acc[i].re) - yr;
          acc[i].re = tr;
          T yi = p.im * wz[i] - cmp[i].im;
          T ti = acc[i].im + yi;
          cmp[i].im = (ti - acc[i].im) - yi;
          acc[i].im = ti;
        } else {
          acc[i].re += p.re * wz[i];
          acc[i].im += p.im * wz[i];
        }
      }
    }
    __syncthreads();
  }
  const int x = x0 + lxo, y = y0 + lyo;
  if (it.slot < 0) {
    C<T>* row = F + (static_cast<int64_t>(x) * nf1 + y) * nf2 + z0;
#pragma unroll
    for (int i = 0; i < TZ; ++i) row[i] = acc[i];
  } else {
    C<T>* pt = partial + static_cast<int64_t>(it.slot) * 64 * TZ;
#pragma unroll
    for (int i = 0; i < TZ; ++i) pt[i * 64 + lane] = acc[i];
  }
}

// 2D spread: a work item is a tile of 64 positions on axis 1 by kTileZ on the last axis, one wave
// per item, lane y owning the kTileZ points of its position in registers.  The item's nodes are
// staged kSpreadBatch at a time in LDS, each as its axis-1 weight row (kWMax values, read whole),
// the offset of the tile's first axis-1 position in its support, its kTileZ last-axis weights at
// the tile's positions and its value; a lane looks its own axis-1 weight up in the row.  FP32
// accumulates with Kahan compensation.
template <typename T, bool KAHAN>
__global__ void __launch_bounds__(64) k_spread2d(C<T>* __restrict__ F, C<T>* __restrict__ partial,
                                                 const NodeRec<T>* __restrict__ nodes, const C<T>* __restrict__ g,
                                                 const int32_t* __restrict__ list,
                                                 const SpreadItem* __restrict__ items, int nf1, int nf2, int nt2,
                                                 int w1, int w2) {
  constexpr int TY = 64, TZ = kTileZ, NB = kSpreadBatch;
  __shared__ T srow[NB][kWMax];
  __shared__ T sz[NB][TZ];
  __shared__ C<T> sg[NB];
  __shared__ int soff[NB];
  const int lane = threadIdx.x;
  const SpreadItem it = items[blockIdx.x];
  if (it.tile < 0) return;                   // padding item
  const int tz = it.tile % nt2;
  const int ty = it.tile / nt2;              // the unit axis 0 has one tile
  const int y0 = ty * TY, z0 = tz * TZ;
  C<T> acc[TZ], cmp[TZ];
#pragma unroll
  for (int i = 0; i < TZ; ++i) {
    acc[i] = C<T>{0, 0};
    cmp[i] = C<T>{0, 0};
  }
  for (int base = 0; base < it.count; base += NB) {
    const int n = it.count - base < NB ? it.count - base : NB;
    if (lane < n) {
      const int q = list[it.start + base + lane];
      const NodeRec<T>* nd = nodes + q;
      int oy = y0 - nd->l0[1];               // support index of the tile's first axis-1 position
      if (oy < 0) oy += nf1;
      int dz = z0 - nd->l0[2];
      if (dz < 0) dz += nf2;
      soff[lane] = oy;
#pragma unroll
      for (int i = 0; i < kWMax; ++i) srow[lane][i] = nd->w[1][i];
#pragma unroll
      for (int i = 0; i < TZ; ++i) {
        int d = dz + i;
        if (d >= nf2) d -= nf2;
        const T v = nd->w[2][d < kWMax ? d : kWMax - 1];
        sz[lane][i] = d < w2 ? v : T(0);
      }
      sg[lane] = g[q];
    }
    __syncthreads();
#pragma unroll DDI_SPREAD_UNROLL
    for (int e = 0; e < n; ++e) {
      int d = soff[e] + lane;                // this lane's support index on axis 1
      if (d >= nf1) d -= nf1;
      const T wr = srow[e][d < w1 ? d : 0];
      const T wy = d < w1 ? wr : T(0);
      const C<T> gq = sg[e];
      const C<T> p = {gq.re * wy, gq.im * wy};
#pragma unroll
      for (int i = 0; i < TZ; ++i) {
        const T wz = sz[e][i];
        if (KAHAN) {
          T yr = p.re * wz - cmp[i].re;
          T tr = acc[i].re + yr;
          cmp[i].re = (tr - acc[i].re) - yr;
          acc[i].re = tr;
          T yi = p.im * wz - cmp[i].im;
          T ti = acc[i].im + yi;
          cmp[i].im = (ti - acc[i].im) - yi;
          acc[i].im = ti;
        } else {
          acc[i].re += p.re * wz;
          acc[i].im += p.im * wz;
        }
      }
    }
    __syncthreads();
  }
  if (it.slot < 0) {
    C<T>* row = F + static_cast<int64_t>(y0 + lane) * nf2 + z0;
#pragma unroll
    for (int i = 0; i < TZ; ++i) row[i] = acc[i];
  } else {
    C<T>* pt = partial + static_cast<int64_t>(it.slot) * 64 * TZ;
#pragma unroll
    for (int i = 0; i < TZ; ++i) pt[i * 64 + lane] = acc[i];
  }
}

// Cooperative weight loads of the matrix-core kernels.  For a block of 16 (tile, node)
// entries, lane (g, t) = (lane / 8, lane % 8) takes the entries 2 g and 2 g + 1 (one 16-byte
// load of their two records) and, for load j (0..5), the window of entry 2 g + j / 3 on axis
// j % 3 at tile position t: eight lanes read one contiguous run of a weight row.  The entry
// records and weight rows are read as raw buffers: a lane offset (32-bit) plus the block's
// uniform offset, with no per-lane 64-bit address arithmetic.  The entry table ends with
// kEntPad zero records, so a block may run past its item's entries; positions outside the
// node's weight row read the zero record at byte offset zrec of the rows.  The loaded
// weights are published to LDS as [entry][axis][8 tile positions].
typedef unsigned u32x2 __attribute__((ext_vector_type(2)));
constexpr int kBufferWord3 = 0x00020000;     // raw buffer descriptor word 3 (32-bit data, no swizzle)

template <typename X>
__device__ inline __amdgpu_buffer_rsrc_t raw_buffer(const X* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<X*>(p), 0, static_cast<int>(bytes), kBufferWord3);
}

struct CoopLanes {
  unsigned eo;                               // byte offset of the lane's two entry records in the block
  int tb;                                    // t - kOffBias
  int slot;                                  // LDS slot of load 0 (entry 2 g, axis 0, position t)
  __device__ explicit CoopLanes(int lane) {
    eo = static_cast<unsigned>(lane >> 3) * 2 * sizeof(int2);
    tb = (lane & 7) - kOffBias;
    slot = (lane >> 3) * 48 + (lane & 7);
  }
  // the lane's two entry records; blk = byte offset of the block's first record
  __device__ void entries(__amdgpu_buffer_rsrc_t ent, int blk, int2* en) const {
    const int4 v = __builtin_bit_cast(int4, __builtin_amdgcn_raw_buffer_load_b128(ent, eo, blk, 0));
    en[0] = make_int2(v.x, v.y);
    en[1] = make_int2(v.z, v.w);
  }
  // byte offset in the weight rows of load j's position, en = the lane's two entry records
  template <typename T>
  __device__ unsigned row_offset(const int2* en, int j, unsigned zrec) const {
    const int2 e = en[j / 3];
    const int a = j % 3;
    const int d = ((e.y >> (8 * a)) & 255) + tb;  // support index of this tile position
    const unsigned at = __umul24(static_cast<unsigned>(e.x), 3 * kRowLen) + static_cast<unsigned>(a * kRowLen + d);
    const unsigned off = at * static_cast<unsigned>(sizeof(T));
    return static_cast<unsigned>(d) < static_cast<unsigned>(kRowLen) ? off : zrec;
  }
  // LDS index of load j's value in the [entry][axis][8] weight buffer
  __device__ int wslot(int j) const { return slot + (j / 3) * 24 + (j % 3) * 8; }
};

template <typename T>
__device__ inline double row_load(__amdgpu_buffer_rsrc_t rows, unsigned off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rows, off, 0, 0));
  else
    return static_cast<double>(__builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rows, off, 0, 0)));
}

// LDS barrier of a one-wave workgroup: LDS operations of a wave complete in order; the fences
// keep the compiler from moving them across.
__device__ __forceinline__ void lds_sync_wave() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Matrix-core form of the spread (FP64, 3D, weight rows): for a tile
//   D[(y,z)][(x,p)] = sum_e A[e][(y,z)] Bs[e][(x,p)],  A[e][(y,z)] = wy_e[y] wz_e[z],
//   Bs[e][(x,p)] = wx_e[x] (part p of g_e),
// with K = entries (four per v_mfma_f64_16x16x4f64 step), four 16-row blocks of (y,z) rows
// and N = (x, p): the whole tile accumulates in registers.  The weights and node values of
// each stage of 16 entries are loaded cooperatively (eight lanes per contiguous run of a
// weight row) and published through LDS, the next stage's loads in flight during the
// current stage's products.  The tile goes through LDS and is written eight lanes per row
// along the last axis (or to its partial slot, in k_spread's slot layout).
template <typename T>
__global__ void __launch_bounds__(64, 4) k_spread_mfma(C<T>* __restrict__ F, C<T>* __restrict__ partial,
                                                    const T* __restrict__ pads, const C<T>* __restrict__ g,
                                                    const int2* __restrict__ ent,
                                                    const SpreadItem* __restrict__ items, int nf1, int nf2, int nt1,
                                                    int nt2, int64_t ent_bytes, int64_t rows_bytes, unsigned zrec) {
  typedef double dbl4s __attribute__((ext_vector_type(4)));
  const int lane = threadIdx.x;
  const SpreadItem it = items[blockIdx.x];
  if (it.tile < 0) return;                   // padding item
  const int tz = it.tile % nt2;
  const int ty = (it.tile / nt2) % nt1;
  const int tx = it.tile / (nt2 * nt1);
  if (it.count == 0) {                       // empty tile (never a chunk): zeros, eight lanes per row
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const int c = 8 * r + (lane >> 3);
      F[(static_cast<int64_t>(tx * 8 + (c >> 3)) * nf1 + (ty * 8 + (c & 7))) * nf2 + tz * kTileZ + (lane & 7)] =
          C<T>{0, 0};
    }
    return;
  }
  // one LDS buffer: the stage weights and node values while entries are accumulated, then the
  // output tile (after the last stage)
  constexpr int XS = 136;                    // x stride of the output staging (bank spread)
  constexpr int XH = 4;                      // x rows of the output staged at once (half the LDS of
                                             // the whole tile: more workgroups per CU)
  __shared__ double lds[XH * XS];
  double* wts = lds;                         // [entry of the stage][axis][8 tile positions]
  double* gv = lds + 16 * 24;                // [entry of the stage][part]
  double* tileO = lds;                       // [x][y][z][part]
  const int nst = (it.count + 15) / 16;
  // Weights by CoopLanes; entries past the item's count take finite weights (of other
  // entries, or the zero record) and a zero node value, so they add nothing.
  const CoopLanes cl(lane);
  const __amdgpu_buffer_rsrc_t ent_r = raw_buffer(ent, ent_bytes), rows_r = raw_buffer(pads, rows_bytes);
  const unsigned go = static_cast<unsigned>(lane >> 1) * sizeof(int2);
  auto load_stage = [&](int st, double* raw, double& graw) {
    const int blk = (it.start + 16 * st) * static_cast<int>(sizeof(int2));
    int2 en[2];
    cl.entries(ent_r, blk, en);
    const int2 eg = __builtin_bit_cast(int2, __builtin_amdgcn_raw_buffer_load_b64(ent_r, go, blk, 0));
#pragma unroll
    for (int j = 0; j < 6; ++j) raw[j] = row_load<T>(rows_r, cl.row_offset<T>(en, j, zrec));
    const bool valid = lane < 32 && 16 * st + (lane >> 1) < it.count;
    const C<T> gq = g[eg.x];
    graw = valid ? static_cast<double>((lane & 1) ? gq.im : gq.re) : 0.0;
  };
  auto publish = [&](const double* raw, double graw) {
#pragma unroll
    for (int j = 0; j < 6; ++j) wts[cl.wslot(j)] = raw[j];
    if (lane < 32) gv[lane] = graw;
  };
  double raw[6], graw = 0.0;
  if (nst > 0) {
    load_stage(0, raw, graw);
    publish(raw, graw);
  }
  lds_sync_wave();
  const int k = lane >> 4, i = lane & 15, x = i >> 1, p = i & 1;
  dbl4s acc[4];
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) acc[mb] = dbl4s{0.0, 0.0, 0.0, 0.0};
  for (int st = 0; st < nst; ++st) {
    const bool more = st + 1 < nst;
    if (more) load_stage(st + 1, raw, graw);  // in flight during this stage's products
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = 4 * q + k;               // entry of this lane's K index at step q
      const double* we = wts + e * 24;
      const double b = we[x] * gv[2 * e + p];
      const double wzv = we[16 + (i & 7)];
#pragma unroll
      for (int mb = 0; mb < 4; ++mb)
        acc[mb] = __builtin_amdgcn_mfma_f64_16x16x4f64(we[8 + 2 * mb + (i >> 3)] * wzv, b, acc[mb], 0, 0, 0);
    }
    if (more) {
      lds_sync_wave();                       // every lane has read this stage's weights
      publish(raw, graw);
      lds_sync_wave();
    }
  }
  // item t of block mb: row 4 t + k -> (y, z) = (2 mb + t / 2, 4 (t % 2) + k), column (x, p);
  // x rows [XH h, XH h + XH) go through LDS at a time and are written eight lanes per 128-byte
  // row along the last axis (or to the partial slot, in k_spread's slot layout)
  const int zl = lane & 7;
#pragma unroll
  for (int h = 0; h < 8 / XH; ++h) {
    lds_sync_wave();                         // earlier reads of the buffer are done
    if (x / XH == h) {
#pragma unroll
      for (int mb = 0; mb < 4; ++mb) {
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int y = 2 * mb + (t >> 1), z = 4 * (t & 1) + k;
          tileO[(x % XH) * XS + (y * 8 + z) * 2 + p] = acc[mb][t];
        }
      }
    }
    lds_sync_wave();
#pragma unroll
    for (int rr = 0; rr < XH; ++rr) {
      const int c = 8 * (XH * h + rr) + (lane >> 3), cx = c >> 3, cy = c & 7;
      const double* o = tileO + (cx % XH) * XS + (cy * 8 + zl) * 2;
      const C<T> v = C<T>{static_cast<T>(o[0]), static_cast<T>(o[1])};
      if (it.slot < 0)
        F[(static_cast<int64_t>(tx * 8 + cx) * nf1 + (ty * 8 + cy)) * nf2 + tz * kTileZ + zl] = v;
      else
        partial[static_cast<int64_t>(it.slot) * 64 * kTileZ + zl * 64 + c] = v;
    }
  }
}

// ------------------------------------------------------------------ tile-owned interpolation
__device__ inline int mod_fine(int d, int n) { return d < 0 ? d + n : d; }

// Lane-per-entry form (3D, 8 x 8 x kTileZ tiles): lane e of the wave takes entry e of the
// tile (64 at a time), holds the node's kernel weights at the tile's positions in registers,
// and walks the tile's 64 columns.  The tile is staged in LDS once per item (lane c loads
// column c, coalesced along the last axis); every lane then reads the same column, so each
// LDS read is a broadcast.  Per column a lane sums over z, then weights by y; per x row by x.
// No cross-lane reduction.  Arithmetic in FP64.
template <typename T>
__global__ void __launch_bounds__(64) k_interp_col(const C<T>* __restrict__ F, const NodeRec<T>* __restrict__ nodes,
                                                   const int32_t* __restrict__ list,
                                                   const SpreadItem* __restrict__ items, int nf0, int nf1, int nf2,
                                                   int nt1, int nt2, int w0, int w1, int w2,
                                                   C<double>* __restrict__ part) {
  constexpr int TX = 8, TY = 8, TZ = kTileZ;
  const int lane = threadIdx.x;
  const SpreadItem it = items[blockIdx.x];
  if (it.tile < 0 || it.count == 0) return;  // padding item or empty tile
  const int tz = it.tile % nt2;
  const int ty = (it.tile / nt2) % nt1;
  const int tx = it.tile / (nt2 * nt1);
  const int x0 = tx * TX, y0 = ty * TY, z0 = tz * TZ;
  __shared__ C<T> tileF[TX * TY * TZ];       // [x][y][z]
  {
    const C<T>* row = F + (static_cast<int64_t>(x0 + lane / TY) * nf1 + (y0 + lane % TY)) * nf2 + z0;
    C<T> v[TZ];
#pragma unroll
    for (int z = 0; z < TZ; ++z) v[z] = row[z];
#pragma unroll
    for (int z = 0; z < TZ; ++z) tileF[lane * TZ + z] = v[z];
  }
  __syncthreads();
  for (int base = 0; base < it.count; base += 64) {
    const int e = base + lane;
    const bool valid = e < it.count;
    const int q = list[it.start + (valid ? e : 0)];
    const NodeRec<T>* nd = nodes + q;
    // weight of tile position i on an axis: support index (tile origin + i - support origin)
    // mod n_fine, zero outside [0, w); i < tile extent <= n_fine, so one subtraction reduces
    auto weight = [&](int d0, int i, int n, int w, int a) {
      int d = d0 + i;
      if (d >= n) d -= n;
      const bool in = valid && d < w;
      const T v = nd->w[a][in ? d : 0];
      return in ? static_cast<double>(v) : 0.0;
    };
    const int dx = mod_fine(x0 - nd->l0[0], nf0);
    const int dy = mod_fine(y0 - nd->l0[1], nf1);
    const int dz = mod_fine(z0 - nd->l0[2], nf2);
    double wx[TX], wy[TY], wz[TZ];
#pragma unroll
    for (int i = 0; i < TX; ++i) wx[i] = weight(dx, i, nf0, w0, 0);
#pragma unroll
    for (int i = 0; i < TY; ++i) wy[i] = weight(dy, i, nf1, w1, 1);
#pragma unroll
    for (int i = 0; i < TZ; ++i) wz[i] = weight(dz, i, nf2, w2, 2);
    double ar = 0.0, ai = 0.0;
    for (int x = 0; x < TX; ++x) {
      const C<T>* plane = tileF + x * TY * TZ;
      double tr = 0.0, ti = 0.0;
#pragma unroll
      for (int y = 0; y < TY; ++y) {
        const C<T>* col = plane + y * TZ;
        double sr = 0.0, si = 0.0;
#pragma unroll
        for (int z = 0; z < TZ; ++z) {
          const C<T> f = col[z];
          sr += wz[z] * static_cast<double>(f.re);
          si += wz[z] * static_cast<double>(f.im);
        }
        tr += wy[y] * sr;
        ti += wy[y] * si;
      }
      ar += wx[x] * tr;
      ai += wx[x] * ti;
    }
    if (valid) part[static_cast<int64_t>(it.start) + e] = C<double>{ar, ai};
  }
}

// Matrix-core form of the same tile interpolation (FP64, 3D, weight rows).  For the
// entries of a tile the partials are a dense product followed by a short weighting:
//   G[e][(x,p)] = sum_{(y,z)} A[e][(y,z)] B[(y,z)][(x,p)],  A[e][(y,z)] = wy_e[y] wz_e[z],
//   B[(y,z)][(x,p)] = part p (re, im) of F[x][y][z],           partial_e,p = sum_x wx_e[x] G[e][(x,p)].
// v_mfma_f64_16x16x4f64 takes A[i][k] from lane i + 16k, B[k][j] from lane j + 16k and
// leaves D[i][j] in lane j + 16 (i % 4), item i / 4.  Rows are entries (16 per block), the
// 16 columns are (x, p), and K = (y, z) runs over 16 steps of 4: at step s lane group k
// covers y = 4 (k / 2) + s / 4, z = 4 (k % 2) + s % 4, so a lane needs four y and four z
// weights of its entry.  B is staged in LDS once per item in fragment order (each lane reads
// its own element); the weights of a row block are loaded cooperatively (eight lanes per
// contiguous run of a weight row) and published through LDS, their loads pipelined across
// the blocks' matrix products.
typedef double dbl4 __attribute__((ext_vector_type(4)));

template <typename T>
__global__ void __launch_bounds__(64) k_interp_mfma(const C<T>* __restrict__ F, const T* __restrict__ pads,
                                                    const int2* __restrict__ ent,
                                                    const SpreadItem* __restrict__ items, int nf1, int nf2, int nt1,
                                                    int nt2, int64_t ent_bytes, int64_t rows_bytes, unsigned zrec,
                                                    C<double>* __restrict__ part) {
  const int lane = threadIdx.x;
  const SpreadItem it = items[blockIdx.x];
  if (it.tile < 0 || it.count == 0) return;  // padding item or empty tile
  const int tz = it.tile % nt2;
  const int ty = (it.tile / nt2) % nt1;
  const int tx = it.tile / (nt2 * nt1);
  constexpr int SB = 65;                     // fragment step stride (one pad: conflict-free staging)
  __shared__ double fragB[16 * SB];
  __shared__ double wts[16 * 24];            // [entry of the block][axis][8 tile positions]
  const int nmb = (it.count + 15) / 16;
  // Weights of a row block are loaded cooperatively (CoopLanes).  Entries past the item's
  // count only fill rows of the product whose results are not stored.  The two dependent
  // loads are pipelined across blocks: entry records two blocks ahead, weight rows one ahead.
  const CoopLanes cl(lane);
  const __amdgpu_buffer_rsrc_t ent_r = raw_buffer(ent, ent_bytes), rows_r = raw_buffer(pads, rows_bytes);
  auto load_ent = [&](int mb, int2* en) { cl.entries(ent_r, (it.start + 16 * mb) * static_cast<int>(sizeof(int2)), en); };
  auto load_rows = [&](const int2* en, double* raw) {
#pragma unroll
    for (int j = 0; j < 6; ++j) raw[j] = row_load<T>(rows_r, cl.row_offset<T>(en, j, zrec));
  };
  int2 en_a[2], en_b[2];
  double raw[6];
  load_ent(0, en_a);
  if (nmb > 1) load_ent(1, en_b);
  {
    // the tile, eight lanes per 128-byte row: load r covers the row (x, y) = (r, lane / 8)
    const int cy = lane >> 3, z = lane & 7;
    const unsigned lo = static_cast<unsigned>(cy * nf2 + z);
    const int at = (4 * (cy & 3) + (z & 3)) * SB + (2 * (cy >> 2) + (z >> 2)) * 16;
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const C<T>* row = F + (static_cast<int64_t>(tx * 8 + r) * nf1 + ty * 8) * nf2 + tz * kTileZ;
      const C<T> v = row[lo];
      fragB[at + 2 * r] = static_cast<double>(v.re);
      fragB[at + 2 * r + 1] = static_cast<double>(v.im);
    }
  }
  load_rows(en_a, raw);
#pragma unroll
  for (int j = 0; j < 6; ++j) wts[cl.wslot(j)] = raw[j];
  __syncthreads();
  const int kk = lane >> 4, col = lane & 15, xo = col >> 1;
  const int yo = 4 * (kk >> 1), zo = 4 * (kk & 1);
  const bool b3 = (lane & 8) != 0, b2 = (lane & 4) != 0;
#if DDI_INTERP_BREG
  double bfr[16];                            // the lane's B fragments, the same for every block
#pragma unroll
  for (int st = 0; st < 16; ++st) bfr[st] = fragB[st * SB + lane];
#endif
  for (int mb = 0; mb < nmb; ++mb) {
    double wy[4], wz[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      wy[i] = wts[col * 24 + 8 + yo + i];
      wz[i] = wts[col * 24 + 16 + zo + i];
    }
    const double wxa = wts[col * 24 + 2 * kk], wxb = wts[col * 24 + 2 * kk + 1];
    // en_b holds block mb + 1's entry records: start its rows, and block mb + 2's records
    const bool more = mb + 1 < nmb;
    if (more) {
      load_rows(en_b, raw);
#pragma unroll
      for (int j = 0; j < 2; ++j) en_a[j] = en_b[j];
      if (mb + 2 < nmb) load_ent(mb + 2, en_b);
    }
    dbl4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int st = 0; st < 16; ++st)
#if DDI_INTERP_BREG
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wy[st >> 2] * wz[st & 3], bfr[st], acc, 0, 0, 0);
#else
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(wy[st >> 2] * wz[st & 3], fragB[st * SB + lane], acc, 0, 0, 0);
#endif
    // item i holds row 4 i + kk (entry 16 mb + 4 i + kk), an A row of lane (4 i + kk) + 16 (xo / 2)
    double v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int src = (4 * i + kk) + 16 * (xo >> 1);
      const double xa = __shfl(wxa, src, 64), xb = __shfl(wxb, src, 64);
      v[i] = acc[i] * ((xo & 1) ? xb : xa);
    }
    // sum over x (lane bits 1..3) for the four items at once: exchange halves across bit 3,
    // then bit 2, then add across bit 1; the lane ends with item b2 + 2 b3
    double u[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double send = b3 ? v[j] : v[j + 2], keep = b3 ? v[j + 2] : v[j];
      u[j] = keep + __shfl_xor(send, 8, 64);
    }
    double r;
    {
      const double send = b2 ? u[0] : u[1], keep = b2 ? u[1] : u[0];
      r = keep + __shfl_xor(send, 4, 64);
    }
    r += __shfl_xor(r, 2, 64);
    const int er = 4 * ((b2 ? 1 : 0) + (b3 ? 2 : 0)) + kk;   // entry of the block
    if ((lane & 2) == 0 && 16 * mb + er < it.count)
      reinterpret_cast<double*>(part + (static_cast<int64_t>(it.start) + 16 * mb))[2 * er + (lane & 1)] = r;
    if (more) {
      __syncthreads();                       // every lane has read this block's weights
#pragma unroll
      for (int j = 0; j < 6; ++j) wts[cl.wslot(j)] = raw[j];
      __syncthreads();
    }
  }
}

// Sum the partials of each node (its list positions, in list order) and apply the node scale.
template <typename T>
__global__ void __launch_bounds__(256) k_interp_gather(const C<double>* __restrict__ part,
                                                       const int32_t* __restrict__ gptr,
                                                       const int32_t* __restrict__ gpos, int64_t M,
                                                       const double* __restrict__ scale, double sscalar,
                                                       C<T>* __restrict__ out) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * 256 + threadIdx.x;
  if (q >= M) return;
  const int b = gptr[q], e = gptr[q + 1];
  if (b == e) return;                        // node outside the scheduled set
  // eight entries per round, all loads in flight, summed in list order
  double sr = 0.0, si = 0.0;
  for (int j0 = b; j0 < e; j0 += 8) {
    int pos[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) pos[j] = gpos[j0 + j < e ? j0 + j : b];
    C<double> v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = part[pos[j]];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (j0 + j < e) {
        sr += v[j].re;
        si += v[j].im;
      }
    }
  }
  const double s = scale ? scale[q] * sscalar : sscalar;
  out[q] = C<T>{static_cast<T>(s * sr), static_cast<T>(s * si)};
}

// Sum the partial tiles of each split tile (deterministic): kReduceSplit workgroups per tile
// (a hot tile's slots are then read by several CUs), each taking a part of the tile's points
// with kReduceGroups threads per point; thread group u sums the slots u, u + G, u + 2G, ... in
// order, sixteen loads in flight, and the G sums are added in group order.
constexpr int kReduceSplit = 4;
#ifndef DDI_REDUCE_GROUPS
#define DDI_REDUCE_GROUPS 4
#endif
constexpr int kReduceGroups = DDI_REDUCE_GROUPS;
constexpr int kReducePoints = 64 * kTileZ / kReduceSplit;   // points per workgroup
template <typename T, int TX, int TY>
__global__ void __launch_bounds__(kReducePoints * kReduceGroups) k_spread_reduce(C<T>* __restrict__ F,
                                                               const C<T>* __restrict__ partial,
                                                               const ReduceItem* __restrict__ red, int nf1, int nf2,
                                                               int nt1, int nt2) {
  constexpr int G = kReduceGroups;
  const int u = threadIdx.x / kReducePoints;
  const int pt = (blockIdx.x % kReduceSplit) * kReducePoints + threadIdx.x % kReducePoints;   // point of the tile
  const int lane = pt & 63;
  const int i = pt >> 6;
  const ReduceItem r = red[blockIdx.x / kReduceSplit];
  const int tz = r.tile % nt2;
  const int ty = (r.tile / nt2) % nt1;
  const int tx = r.tile / (nt2 * nt1);
  const int x = tx * TX + lane / TY, y = ty * TY + lane % TY, z = tz * kTileZ + i;
  const C<T>* src = partial + (static_cast<int64_t>(r.first_slot) * kTileZ + i) * 64 + lane;
  constexpr int64_t kSlot = 64 * kTileZ;     // elements per slot
  double sr = 0.0, si = 0.0;
  int s = u;
  for (; s + 15 * G < r.nslots; s += 16 * G) {
    C<T> v[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) v[j] = src[static_cast<int64_t>(s + j * G) * kSlot];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      sr += static_cast<double>(v[j].re);
      si += static_cast<double>(v[j].im);
    }
  }
  for (; s + 3 * G < r.nslots; s += 4 * G) {
    C<T> v[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) v[j] = src[static_cast<int64_t>(s + j * G) * kSlot];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      sr += static_cast<double>(v[j].re);
      si += static_cast<double>(v[j].im);
    }
  }
  for (; s < r.nslots; s += G) {
    const C<T> v = src[static_cast<int64_t>(s) * kSlot];
    sr += static_cast<double>(v.re);
    si += static_cast<double>(v.im);
  }
  if constexpr (G > 1) {
    __shared__ double part[G > 1 ? G - 1 : 1][kReducePoints][2];
    const int p = threadIdx.x % kReducePoints;
    if (u > 0) {
      part[u - 1][p][0] = sr;
      part[u - 1][p][1] = si;
    }
    __syncthreads();
    if (u > 0) return;
#pragma unroll
    for (int g = 0; g < G - 1; ++g) {
      sr += part[g][p][0];
      si += part[g][p][1];
    }
  }
  F[(static_cast<int64_t>(x) * nf1 + y) * nf2 + z] = C<T>{static_cast<T>(sr), static_cast<T>(si)};
}

// ------------------------------------------------------------------ drivers
// Sizes of the matrix-core kernels' raw buffers: the entry table and the weight rows (with
// the zero record that follows them, at byte offset zero_record).
static int64_t ent_bytes(const Schedule& S) { return static_cast<int64_t>(S.ent.size()) * sizeof(int32_t); }
template <typename T>
static unsigned zero_record(const HostTables& H) {
  return static_cast<unsigned>(H.M * 3 * kRowLen * static_cast<int64_t>(sizeof(T)));
}
template <typename T>
static int64_t rows_bytes(const HostTables& H) {
  return (H.M + 1) * 3 * kRowLen * static_cast<int64_t>(sizeof(T));
}

// ev (nullable): events recorded on s at the start (ev[0]) and after each stage:
// 1 last-axis FFT (pad), 2 axis-1 FFT, 3 axis-0 FFT, 4 interpolation, 5 spread,
// 6 spread reduce, 7 axis-0 FFT, 8 axis-1 FFT, 9 last-axis FFT (truncate).
#define DDI_REC(i)                                 \
  do {                                             \
    if (ev) DDI_CHECK(hipEventRecord(ev[(i)], s)); \
  } while (0)

// Forward transform of the padded, deconvolved density onto the fine grid (pruned:
// only lines that can hold non-zeros are transformed).
template <typename T, int SIGN>
static hipError_t type2_fft(DevicePlan& P, int which, const T* rho, hipStream_t s, hipEvent_t* ev) {
  const HostTables& H = P.H;
  const int z0 = H.sched[which].z0, nz = H.sched[which].nz;   // only the window is needed
  const int ny = H.sched[which].ny;                               // and on axis 1 only its lines
  const int ycut = ny < H.nf[1];
  C<T>* F = reinterpret_cast<C<T>*>(P.fine);
  const C<T>* tw2 = reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.nf[2])]);
  DDI_CHECK((launch_contig<T, SIGN, R2C_PAD>(H.nf[2], rho, F, H.N[0], H.N[1], H.nf[0], H.nf[1], H.N[2], z0, nz,
                                             P.deconv[0], P.deconv[1], P.deconv[2], tw2, s)));
  DDI_REC(1);
  DDI_CHECK((launch_strided<T, SIGN>(H.nf[1], F, 1, H.nf[0], H.nf[1], H.nf[2], H.N[0], 1, H.N[1], 1, ycut, ny, z0,
                                     nz, reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.nf[1])]), s)));
  DDI_REC(2);
  if (H.nf[0] > 1) {
    DDI_CHECK((launch_strided<T, SIGN>(H.nf[0], F, 0, H.nf[0], H.nf[1], H.nf[2], ny, ycut, H.N[0], 1, 0, H.N[0], z0,
                                       nz, reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.nf[0])]), s)));
  }
  DDI_REC(3);
  return hipSuccess;
}

// Inverse transform of the spread grid, keeping only the modes of the compact grid.
template <typename T, int SIGN>
static hipError_t type1_fft(DevicePlan& P, int which, T* phi, hipStream_t s, hipEvent_t* ev) {
  const HostTables& H = P.H;
  const int z0 = H.sched[which].z0, nz = H.sched[which].nz;   // the spread filled only the window
  const int ny = H.sched[which].ny;                               // and on axis 1 only its lines
  const int ycut = ny < H.nf[1];
  C<T>* F = reinterpret_cast<C<T>*>(P.fine);
  if (H.nf[0] > 1) {
    DDI_CHECK((launch_strided<T, SIGN>(H.nf[0], F, 0, H.nf[0], H.nf[1], H.nf[2], ny, ycut, H.N[0], 0, 1, H.N[0], z0,
                                       nz, reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.nf[0])]), s)));
  }
  DDI_REC(7);
  DDI_CHECK((launch_strided<T, SIGN>(H.nf[1], F, 1, H.nf[0], H.nf[1], H.nf[2], H.N[0], 1, ny, ycut, 1, H.N[1], z0,
                                     nz, reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.nf[1])]), s)));
  DDI_REC(8);
  const C<T>* tw2 = reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.nf[2])]);
  DDI_CHECK((launch_contig<T, SIGN, C2R_TRUNC>(H.nf[2], F, phi, H.N[0], H.N[1], H.nf[0], H.nf[1], H.N[2], z0, nz,
                                               P.deconv[0], P.deconv[1], P.deconv[2], tw2, s)));
  DDI_REC(9);
  return hipSuccess;
}

template <typename T, int W0, int W, int IB>
static hipError_t interp_w(DevicePlan& P, int which, C<T>* out, const double* scale, double sscalar,
                           hipStream_t s) {
  const HostTables& H = P.H;
  const Schedule& S = H.sched[which];
  const DevicePlan::DevSchedule& D = P.dsched[which];
  const int ng = static_cast<int>(S.interp_items.size());
  if (ng > 0) {
    constexpr int R = IB + W - 1;
    constexpr int R0 = W0 == 1 ? 1 : IB + W0 - 1;
    constexpr int NT = 512;   // 8 waves: the LDS region limits residency to two workgroups per CU
    const size_t shm = static_cast<size_t>(R0) * R * R * sizeof(C<T>);
    if (H.ib[1] != IB || H.ireg[1] != R || H.ireg[0] != R0) return hipErrorInvalidValue;
    if (!P.interp_lds_ready) {
      DDI_CHECK(hipFuncSetAttribute(reinterpret_cast<const void*>(&k_interp_lds<T, W0, W, IB, NT>),
                                    hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(shm)));
      P.interp_lds_ready = true;
    }
    hipLaunchKernelGGL((k_interp_lds<T, W0, W, IB, NT>), dim3(ng), dim3(NT), shm, s,
                       reinterpret_cast<const C<T>*>(P.fine), reinterpret_cast<const NodeRec<T>*>(P.nodes),
                       D.interp_items, H.nf[0], H.nf[1], H.nf[2], scale, sscalar, out);
    DDI_CHECK(hipGetLastError());
  }
  const int64_t nd = static_cast<int64_t>(S.interp_direct.size());
  if (nd > 0) {
    constexpr int per_block = 4 * InterpShape<W>::NS;
    const int blocks = static_cast<int>((nd + per_block - 1) / per_block);
    hipLaunchKernelGGL((k_interp<T, W0, W>), dim3(blocks), dim3(256), 0, s, reinterpret_cast<const C<T>*>(P.fine),
                       reinterpret_cast<const NodeRec<T>*>(P.nodes), D.interp_direct, nd, H.nf[0], H.nf[1], H.nf[2],
                       scale, sscalar, out);
    DDI_CHECK(hipGetLastError());
  }
  return hipSuccess;
}

template <typename T, int W>
static hipError_t interp_d(DevicePlan& P, int which, C<T>* out, const double* scale, double sscalar,
                           hipStream_t s) {
  if (P.H.W[0] == 1) return interp_w<T, 1, W, 8>(P, which, out, scale, sscalar, s);
  return interp_w<T, W, W, kInterpBlock3>(P, which, out, scale, sscalar, s);
}

template <typename T>
static hipError_t interp_tile_t(DevicePlan& P, int which, C<T>* out, const double* scale, double sscalar,
                                hipStream_t s) {
  const HostTables& H = P.H;
  const Schedule& S = H.sched[which];
  const DevicePlan::DevSchedule& D = P.dsched[which];
  const int nitems = static_cast<int>(S.items.size());
  if (nitems > 0 && !S.list.empty()) {
    if (kInterpMfma && H.row_windows)
      hipLaunchKernelGGL((k_interp_mfma<T>), dim3(nitems), dim3(64), 0, s, reinterpret_cast<const C<T>*>(P.fine),
                         reinterpret_cast<const T*>(P.pads), reinterpret_cast<const int2*>(D.ent), D.items, H.nf[1],
                         H.nf[2], H.ntiles[1], H.ntiles[2], ent_bytes(S), rows_bytes<T>(H), zero_record<T>(H),
                         reinterpret_cast<C<double>*>(P.ipartial));
    else
      hipLaunchKernelGGL((k_interp_col<T>), dim3(nitems), dim3(64), 0, s, reinterpret_cast<const C<T>*>(P.fine),
                         reinterpret_cast<const NodeRec<T>*>(P.nodes), D.list, D.items, H.nf[0], H.nf[1], H.nf[2],
                         H.ntiles[1], H.ntiles[2], H.W[0], H.W[1], H.W[2], reinterpret_cast<C<double>*>(P.ipartial));
    DDI_CHECK(hipGetLastError());
  }
  if (H.M > 0) {
    const int blocks = static_cast<int>((H.M + 255) / 256);
    hipLaunchKernelGGL((k_interp_gather<T>), dim3(blocks), dim3(256), 0, s,
                       reinterpret_cast<const C<double>*>(P.ipartial), D.gptr, D.gpos, H.M, scale, sscalar, out);
    DDI_CHECK(hipGetLastError());
  }
  return hipSuccess;
}

template <typename T>
static hipError_t interp(DevicePlan& P, int which, C<T>* out, const double* scale, double sscalar,
                         hipStream_t s) {
  if (interp_is_tiled(P.H, sizeof(T) == 8)) return interp_tile_t<T>(P, which, out, scale, sscalar, s);
  {
    switch (P.H.w) {
      case 2: return interp_d<T, 2>(P, which, out, scale, sscalar, s);
      case 3: return interp_d<T, 3>(P, which, out, scale, sscalar, s);
      case 4: return interp_d<T, 4>(P, which, out, scale, sscalar, s);
      case 5: return interp_d<T, 5>(P, which, out, scale, sscalar, s);
      case 6: return interp_d<T, 6>(P, which, out, scale, sscalar, s);
      case 7: return interp_d<T, 7>(P, which, out, scale, sscalar, s);
      case 8: return interp_d<T, 8>(P, which, out, scale, sscalar, s);
      case 9: return interp_d<T, 9>(P, which, out, scale, sscalar, s);
      case 10: return interp_d<T, 10>(P, which, out, scale, sscalar, s);
      case 11: return interp_d<T, 11>(P, which, out, scale, sscalar, s);
      case 12: return interp_d<T, 12>(P, which, out, scale, sscalar, s);
      case 13: return interp_d<T, 13>(P, which, out, scale, sscalar, s);
      case 14: return interp_d<T, 14>(P, which, out, scale, sscalar, s);
      case 15: return interp_d<T, 15>(P, which, out, scale, sscalar, s);
      case 16: return interp_d<T, 16>(P, which, out, scale, sscalar, s);
      default: return hipErrorInvalidValue;
    }
  }
}

template <typename T, int TX, int TY>
static hipError_t spread_t(DevicePlan& P, int which, const C<T>* g, hipStream_t s, hipEvent_t* ev) {
  const HostTables& H = P.H;
  const Schedule& S = H.sched[which];
  const DevicePlan::DevSchedule& D = P.dsched[which];
  C<T>* F = reinterpret_cast<C<T>*>(P.fine);
  const int nitems = static_cast<int>(S.items.size());
  constexpr bool kahan = sizeof(T) == 4;
  bool done = false;
  if constexpr (kSpreadMfma && TX == 8) {
    if (H.row_windows && P.pads) {
      hipLaunchKernelGGL((k_spread_mfma<T>), dim3(nitems), dim3(64), 0, s, F, reinterpret_cast<C<T>*>(P.partial),
                         reinterpret_cast<const T*>(P.pads), g, reinterpret_cast<const int2*>(D.ent), D.items, H.nf[1],
                         H.nf[2], H.ntiles[1], H.ntiles[2], ent_bytes(S), rows_bytes<T>(H), zero_record<T>(H));
      done = true;
    }
  }
  if constexpr (TX == 1) {
    if (!done) {
      hipLaunchKernelGGL((k_spread2d<T, kahan>), dim3(nitems), dim3(64), 0, s, F, reinterpret_cast<C<T>*>(P.partial),
                         reinterpret_cast<const NodeRec<T>*>(P.nodes), g, D.list, D.items, H.nf[1], H.nf[2],
                         H.ntiles[2], H.W[1], H.W[2]);
      done = true;
    }
  }
  if (!done)
    hipLaunchKernelGGL((k_spread<T, kahan, TX, TY>), dim3(nitems), dim3(64), 0, s, F,
                       reinterpret_cast<C<T>*>(P.partial), reinterpret_cast<const NodeRec<T>*>(P.nodes), g, D.list,
                       D.items, H.nf[0], H.nf[1], H.nf[2], H.ntiles[1], H.ntiles[2], H.W[0], H.W[1], H.W[2]);
  DDI_CHECK(hipGetLastError());
  DDI_REC(5);
  if (!S.reduces.empty()) {
    hipLaunchKernelGGL((k_spread_reduce<T, TX, TY>), dim3(static_cast<int>(S.reduces.size()) * kReduceSplit),
                       dim3(kReducePoints * kReduceGroups), 0,
                       s, F, reinterpret_cast<const C<T>*>(P.partial), D.reduces, H.nf[1], H.nf[2], H.ntiles[1],
                       H.ntiles[2]);
    DDI_CHECK(hipGetLastError());
  }
  DDI_REC(6);
  return hipSuccess;
}

template <typename T>
static hipError_t spread(DevicePlan& P, int which, const C<T>* g, hipStream_t s, hipEvent_t* ev) {
  if (P.H.tile[0] == 8 && P.H.tile[1] == 8) return spread_t<T, 8, 8>(P, which, g, s, ev);
  if (P.H.tile[0] == 1 && P.H.tile[1] == 64) return spread_t<T, 1, 64>(P, which, g, s, ev);
  return hipErrorInvalidValue;
}

template <typename T>
hipError_t run_type2(DevicePlan& P, int which, const T* rho, Complex<T>* out, const double* scale,
                     double cscalar, int sign, hipStream_t s, hipEvent_t* ev) {
  DDI_REC(0);
  if (sign < 0) DDI_CHECK((type2_fft<T, -1>(P, which, rho, s, ev)));
  else DDI_CHECK((type2_fft<T, +1>(P, which, rho, s, ev)));
  DDI_CHECK((interp<T>(P, which, out, scale, cscalar, s)));
  DDI_REC(4);
  return hipSuccess;
}

template <typename T>
hipError_t run_type1(DevicePlan& P, int which, const Complex<T>* g, T* phi, int sign, hipStream_t s,
                     hipEvent_t* ev) {
  DDI_CHECK(spread<T>(P, which, g, s, ev));
  if (sign > 0) return type1_fft<T, +1>(P, which, phi, s, ev);
  return type1_fft<T, -1>(P, which, phi, s, ev);
}

// Forward (sign = +1: exp(-ikx) to the nodes, exp(+ikx) back) or literal adjoint (sign = -1)
// of the operator on real grids: one node of each +-k pair is interpolated and spread, its
// weight carrying the factor 2 of the pair (the partner's term is the complex conjugate, and
// only the real part is kept).
template <typename T>
hipError_t run_apply(DevicePlan& P, const T* rho, T* phi, int sign, hipStream_t s, hipEvent_t* ev) {
  C<T>* g = reinterpret_cast<C<T>*>(P.gnodes);
  DDI_CHECK(run_type2<T>(P, kHalf, rho, g, P.c_half, 1.0, -sign, s, ev));
  return run_type1<T>(P, kHalf, g, phi, sign, s, ev);
}

// I_1 of the split (Eq. 3.9).  The box is zero-padded to the fine grid (2 N_i points,
// k_m = 2 pi m / (2 N_i h_i)); the density enters without deconvolution.  Only the modes
// m2 in [0, N2) are formed (a real field's half set; m2 = -N2 is a Nyquist plane).  3D: last-axis
// FFT with padding, axis-1 FFT, then one pass that transforms axis 0, multiplies by
// (1 - q) Uhat and transforms back, axis-1 inverse (front); last-axis inverse with truncation,
// real part and accumulation into phi (back).  2D (axes 1 and 2 of the internal layout): the
// padded last-axis FFT, then the pass along axis 1 with the multiplier (front); the same last
// pass (back).  Works in fine_short.
template <typename T>
hipError_t split_short_front(DevicePlan& P, const T* rho, hipStream_t s) {
  const HostTables& H = P.H;
  if (!H.split || !P.ones || !P.fine_short) return hipErrorInvalidValue;
  C<T>* F = reinterpret_cast<C<T>*>(P.fine_short);
  const int nz = H.N[2];
  const C<T>* tw1 = reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.nf[1])]);
  const C<T>* tw2 = reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.nf[2])]);
  SplitSymbol sp;
  for (int i = 0; i < 3; ++i) sp.dk[i] = 2.0 * M_PI / (H.nf[i] * H.h[i]);
  sp.inv_s2 = 1.0 / (H.split_s * H.split_s);
  sp.inv_s = 1.0 / H.split_s;
  sp.scale = 1.0 / (static_cast<double>(H.nf[0]) * H.nf[1] * H.nf[2]);
  sp.dim = H.dim;
  if (H.dim == 3) {
    for (int i = 0; i < 3; ++i) {
      sp.n[i] = H.nv[i];
      sp.m[i] = H.mv[i];
    }
    sp.nm = H.nv[0] * H.mv[0] + H.nv[1] * H.mv[1] + H.nv[2] * H.mv[2];
    sp.n3m3 = 0.0;
  } else {
    // the symbol pass runs along internal axis 1 (the paper's x) as the kernel's axis 0, with the
    // last axis (the paper's y) as its axis 2
    sp.n[0] = H.nv[0]; sp.n[1] = 0.0; sp.n[2] = H.nv[1];
    sp.m[0] = H.mv[0]; sp.m[1] = 0.0; sp.m[2] = H.mv[1];
    sp.dk[0] = sp.dk[1];
    sp.dk[1] = 0.0;
    sp.nm = 0.0;
    sp.n3m3 = H.nv[2] * H.mv[2];
  }
  DDI_CHECK((launch_contig<T, -1, R2C_PAD>(H.nf[2], rho, F, H.N[0], H.N[1], H.nf[0], H.nf[1], H.N[2], 0, nz, P.ones,
                                           P.ones, P.ones, tw2, s)));
  if (H.dim == 2) return launch_symbol<T>(H.nf[1], F, 1, H.nf[2], H.N[1], nz, sp, tw1, s);
  const C<T>* tw0 = reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.nf[0])]);
  DDI_CHECK((launch_strided<T, -1>(H.nf[1], F, 1, H.nf[0], H.nf[1], H.nf[2], H.N[0], 1, H.N[1], 1, 0, H.N[1], 0, nz,
                                   tw1, s)));
  DDI_CHECK((launch_symbol<T>(H.nf[0], F, H.nf[1], H.nf[2], H.N[0], nz, sp, tw0, s)));
  DDI_CHECK((launch_strided<T, 1>(H.nf[1], F, 1, H.nf[0], H.nf[1], H.nf[2], H.N[0], 1, H.N[1], 0, 1, H.N[1], 0, nz,
                                  tw1, s)));
  return hipSuccess;
}

template <typename T>
hipError_t split_short_back(DevicePlan& P, T* phi, hipStream_t s) {
  const HostTables& H = P.H;
  if (!H.split || !P.ones || !P.fine_short) return hipErrorInvalidValue;
  const C<T>* tw2 = reinterpret_cast<const C<T>*>(P.twiddles[tw_slot(H.nf[2])]);
  return launch_contig<T, 1, C2R_ADD>(H.nf[2], P.fine_short, phi, H.N[0], H.N[1], H.nf[0], H.nf[1], H.N[2], 0,
                                      H.N[2], P.ones, P.ones, P.ones, tw2, s);
}

// The operator of the plan.  Split: I_1's front runs on the plan's own stream while I_2 runs on
// s; I_1's last pass adds into phi once I_2 has written it, and s waits for it (I_1 is its own
// transpose, so the adjoint takes the same I_1).
template <typename T>
hipError_t run_ddi(DevicePlan& P, const T* rho, T* phi, int sign, hipStream_t s, hipEvent_t* ev) {
  if (!P.H.split) return run_apply<T>(P, rho, phi, sign, s, ev);
  DDI_CHECK(hipEventRecord(P.ev_fork, s));
  DDI_CHECK(hipStreamWaitEvent(P.aux, P.ev_fork, 0));
  DDI_CHECK(split_short_front<T>(P, rho, P.aux));
  DDI_CHECK(run_apply<T>(P, rho, phi, sign, s, ev));
  DDI_CHECK(hipEventRecord(P.ev_long, s));
  DDI_CHECK(hipStreamWaitEvent(P.aux, P.ev_long, 0));
  DDI_CHECK(split_short_back<T>(P, phi, P.aux));
  DDI_CHECK(hipEventRecord(P.ev_join, P.aux));
  return hipStreamWaitEvent(s, P.ev_join, 0);
}

// ------------------------------------------------------------------ dipole axes
// c = base * Uhat(k; n, m) for every node (Eq. DipKer; two axes: Eq. dipmn), in plan order.
__global__ void __launch_bounds__(256) k_dipole_coeffs(int64_t M, int dim, const double* __restrict__ kq,
                                                       const double* __restrict__ bs, const double* __restrict__ bh,
                                                       double n0, double n1, double n2, double m0, double m1,
                                                       double m2, double* __restrict__ cs, double* __restrict__ ch) {
  const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (q >= M) return;
  const double k0 = kq[3 * q], k1 = kq[3 * q + 1], k2 = kq[3 * q + 2];
  const double kk = k0 * k0 + k1 * k1 + k2 * k2;
  double U;
  if (dim == 3) {
    U = 3.0 * (k0 * n0 + k1 * n1 + k2 * n2) * (k0 * m0 + k1 * m1 + k2 * m2) / kk - (n0 * m0 + n1 * m1 + n2 * m2);
  } else {
    U = 3.0 * ((k0 * n0 + k1 * n1) * (k0 * m0 + k1 * m1) - n2 * m2 * kk) / (2.0 * sqrt(kk));
  }
  cs[q] = bs[q] * U;
  ch[q] = bh[q] * U;
}

hipError_t run_set_dipole(DevicePlan& P, const double* n, const double* m, hipStream_t s) {
  const int64_t M = P.H.M;
  if (!P.kq || !P.base_scaled || !P.base_half || M <= 0) return hipErrorInvalidValue;
  const int blocks = static_cast<int>((M + 255) / 256);
  hipLaunchKernelGGL(k_dipole_coeffs, dim3(blocks), dim3(256), 0, s, M, P.H.dim, P.kq, P.base_scaled, P.base_half,
                     n[0], n[1], n[2], m[0], m[1], m[2], P.c_scaled, P.c_half);
  return hipGetLastError();
}

template hipError_t split_short_front<double>(DevicePlan&, const double*, hipStream_t);
template hipError_t split_short_front<float>(DevicePlan&, const float*, hipStream_t);
template hipError_t split_short_back<double>(DevicePlan&, double*, hipStream_t);
template hipError_t split_short_back<float>(DevicePlan&, float*, hipStream_t);
template hipError_t run_ddi<double>(DevicePlan&, const double*, double*, int, hipStream_t, hipEvent_t*);
template hipError_t run_ddi<float>(DevicePlan&, const float*, float*, int, hipStream_t, hipEvent_t*);
template hipError_t run_type2<double>(DevicePlan&, int, const double*, Complex<double>*, const double*, double,
                                      int, hipStream_t, hipEvent_t*);
template hipError_t run_type2<float>(DevicePlan&, int, const float*, Complex<float>*, const double*, double, int,
                                     hipStream_t, hipEvent_t*);
template hipError_t run_type1<double>(DevicePlan&, int, const Complex<double>*, double*, int, hipStream_t,
                                      hipEvent_t*);
template hipError_t run_type1<float>(DevicePlan&, int, const Complex<float>*, float*, int, hipStream_t,
                                     hipEvent_t*);
template hipError_t run_apply<double>(DevicePlan&, const double*, double*, int, hipStream_t, hipEvent_t*);
template hipError_t run_apply<float>(DevicePlan&, const float*, float*, int, hipStream_t, hipEvent_t*);

}  // namespace ddi
