// Internal declarations shared by the plan builder, the kernels and the C ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ddi.h"

namespace ddi {

constexpr int kWMax = 16;          // largest kernel width
constexpr int kTwSlots = 20;       // twiddle tables: lengths 2^0..2^10 and 3 * 2^0..3 * 2^8
constexpr int kTileZ = 8;          // spread tile extent along the last axis (registers per lane)
#ifndef DDI_INTERP_BLOCK3
#define DDI_INTERP_BLOCK3 4
#endif
#ifndef DDI_INTERP_MIN_GROUP
#define DDI_INTERP_MIN_GROUP 6
#endif
// interpolation groups: block of cells per axis (3D) and smallest group staged in LDS
constexpr int kInterpBlock3 = DDI_INTERP_BLOCK3;
constexpr int kInterpMinGroup = DDI_INTERP_MIN_GROUP;
#ifndef DDI_SPREAD_BATCH
#define DDI_SPREAD_BATCH 64
#endif
// spread: nodes staged in LDS per batch (LDS per wave ~ batch * 26 values)
constexpr int kSpreadBatch = DDI_SPREAD_BATCH;
#ifndef DDI_SPREAD_CHUNK
#define DDI_SPREAD_CHUNK 256
#endif
#ifndef DDI_SPREAD_CHUNK_MFMA
#define DDI_SPREAD_CHUNK_MFMA 512
#endif
// spread: a tile with more nodes is split into chunks of this many (partial tiles + reduce);
// the matrix-core kernels take longer chunks (cheaper per node)
constexpr int kSpreadChunk = DDI_SPREAD_CHUNK;
#ifndef DDI_INTERP_BREG
#define DDI_INTERP_BREG 1      // the interpolation's tile fragments held in registers across blocks
#endif
#ifndef DDI_SPREAD_CHUNK_2D
#define DDI_SPREAD_CHUNK_2D 32
#endif
// shortest chunk of the 2D spread (hot tiles are split into chunks of at least this many nodes)
constexpr int kSpreadChunk2d = DDI_SPREAD_CHUNK_2D;
constexpr int kSpreadChunkMfma = DDI_SPREAD_CHUNK_MFMA;
#ifndef DDI_SPREAD_WAVES
#define DDI_SPREAD_WAVES 4096
#endif
// matrix-core chunks are shortened until the entries fill about this many items (resident waves)
constexpr int kSpreadWaves = DDI_SPREAD_WAVES;
#ifndef DDI_SPREAD_XCD_ORDER
#define DDI_SPREAD_XCD_ORDER 1
#endif
#ifndef DDI_SPREAD_UNROLL
#define DDI_SPREAD_UNROLL 4
#endif
constexpr int kRowLen = kWMax;    // weight row of the matrix-core kernels: w weights, then zeros
constexpr int kOffBias = 8;       // entry offsets are stored biased by this (non-negative bytes)
constexpr int kEntPad = 32;       // zero entries after the last one (blocks of 16 may read past an item)
#ifndef DDI_INTERP_TILE
#define DDI_INTERP_TILE 1
#endif
// FP64 interpolation in 3D: 1 = tile-owned (each fine-grid tile read once by a wave whose
// lanes are (tile, node) entries; one partial per entry, gathered per node); 0 = node-owned
// (LDS-staged groups plus direct reads of the fine grid), which FP32 and 2D always use
constexpr bool kInterpTile = DDI_INTERP_TILE != 0;
#ifndef DDI_INTERP_MFMA
#define DDI_INTERP_MFMA 1
#endif
// tile-owned FP64 interpolation on the matrix cores where the plan has row windows
constexpr bool kInterpMfma = DDI_INTERP_MFMA != 0;
#ifndef DDI_SPREAD_MFMA
#define DDI_SPREAD_MFMA 1
#endif
// spread on the matrix cores where the plan has row windows
constexpr bool kSpreadMfma = DDI_SPREAD_MFMA != 0;


// One quadrature node as seen by the spread / interpolation kernels: the first
// fine-grid index of its support on each axis (already reduced mod n_fine) and
// the separable kernel weights psi(l0 + i - tau) for i < w on each axis.
template <typename T>
struct alignas(16) NodeRec {
  int32_t l0[3];
  int32_t pad;
  T w[3][kWMax];
};

// A unit of spread work: the nodes list[start, start+count) are summed into
// the tile `tile`; slot < 0 writes the tile directly, otherwise a partial
// tile is written to partial slot `slot` and summed by a reduce item.
struct SpreadItem {
  int32_t tile;
  int32_t start;
  int32_t count;
  int32_t slot;
};

// A group of nodes (plan-order range) whose supports start in one block of ib^3
// cells; their supports lie in the region org + [0, ireg) (mod n_fine), staged in LDS.
struct InterpItem {
  int32_t start;
  int32_t count;
  int32_t org[3];
  int32_t pad[3];
};

struct ReduceItem {
  int32_t tile;
  int32_t first_slot;
  int32_t nslots;
  int32_t pad;
};

// Interpolation and spread work lists over one subset of the nodes.
struct Schedule {
  std::vector<InterpItem> interp_items;   // grouped nodes (LDS-staged region)
  std::vector<int32_t> interp_direct;     // nodes interpolated straight from the grid
  std::vector<int32_t> list;              // spread: node indices per tile, concatenated
  std::vector<SpreadItem> items;
  std::vector<ReduceItem> reduces;
  int32_t nslots = 0;
  // tile-owned interpolation: one partial sum per list entry; the list positions of node q
  // are gpos[gptr[q] .. gptr[q+1]) (increasing)
  std::vector<int32_t> gptr;
  std::vector<int32_t> gpos;
  // row-window form (see HostTables::row_windows): per list entry i, ent[2i] = node and
  // ent[2i+1] = kOffBias + s_a packed as bytes x | y << 8 | z << 16, where s_a in [-7, w-1]
  // is the tile origin minus the support origin on axis a; kEntPad zero entries follow
  std::vector<int32_t> ent;
  // Last-axis window: every fine position that a scheduled node's support touches lies in
  // [z0, z0 + nz) (mod n_fine[2]); z0 and nz are multiples of HostTables::zalign.  The FFT passes of
  // this schedule read and write only the window, and the spread writes only its tiles.
  int32_t z0 = 0;
  int32_t nz = 0;
  // Axis-1 window (3D): every scheduled support lies at signed fine positions [-ny/2, ny/2) on
  // axis 1 (ny even; n_fine[1] when the supports reach the whole axis).  The axis-0 passes
  // transform only those lines and the axis-1 passes write (type-2) or read (type-1) only them.
  int32_t ny = 0;
};

// The two node subsets a plan schedules.  kAll: every node (the type-2 / type-1 entry
// points, whose node values are arbitrary).  kHalf: one node of each +-k pair (the
// operator on real grids, where the pair's terms are complex conjugates).
enum { kAll = 0, kHalf = 1 };

// Host-side tables built by build_tables() (all FP64).
struct HostTables {
  int dim = 3;
  int N[3] = {1, 1, 1};        // grid sizes on the internal 3-axis layout (N[0] = 1 in 2D)
  int nf[3] = {1, 1, 1};       // oversampled FFT sizes
  int W[3] = {1, 1, 1};        // kernel width per axis (1 on the unused 2D axis)
  int tile[3] = {1, 1, 1};     // spread tile extents
  int ntiles[3] = {1, 1, 1};
  int ib[3] = {1, 1, 1};       // interpolation group block extents
  int ireg[3] = {1, 1, 1};     // region extents ib + W - 1
  double h[3] = {1, 1, 1};
  double L[3] = {0, 0, 0};
  double cell = 1.0;           // prod(h)
  int w = 0;
  double es_beta = 0.0;
  double kmax = 0.0;
  int64_t m_nominal = 0;
  int64_t M = 0;               // nodes kept
  // per node, plan (sorted) order
  std::vector<int32_t> index;  // [M][3]
  std::vector<double> k;       // [M][3]
  std::vector<double> c;       // [M]  W Uhat / (2 pi)^d (times q for a split plan), for the axes nv, mv
  std::vector<double> base;    // [M]  W / (2 pi)^d (times q): c without the symbol
  bool c_stale = false;        // the axes changed (ddi_set_dipole): c is recomputed when read
  std::vector<int32_t> l0;     // [M][3]
  std::vector<double> wts;     // [M][3][kWMax]
  std::vector<double> deconv[3];   // 1/phihat per compact index, length N[a]
  // per node: 2 for the kept member of a complete +-k pair, 1 for a node whose partner
  // was masked out, 0 for the partner that is not kept in the half set
  std::vector<double> half_factor;
  // 3D with 8 x 8 x 8 tiles and n_fine >= w + 8 on every axis: a node's weights at a tile's
  // positions are one contiguous run of its weight row (no periodic wrap inside a tile); and
  // the weight rows fit 32-bit byte offsets (2 GiB)
  bool row_windows = false;
  // granularity of the schedules' last-axis windows: a multiple of kTileZ; 8 in FP64, 16 in FP32
  // (the strided FFT passes cover a window in blocks of lines that divide it: 128-byte rows)
  int zalign = 16;
  Schedule sched[2];
  // split of Eq. 3.9 (3D): c holds the I_2 weights (times q); I_1 uses the axes and s
  bool split = false;
  double split_s = 0.0;
  double nv[3] = {0, 0, 1};
  double mv[3] = {0, 0, 1};
};

// Kernel selection shared by the plan upload and the drivers.
inline bool uses_weight_rows(const HostTables& H) { return H.row_windows && ((kInterpTile && kInterpMfma) || kSpreadMfma); }
// (FP64 only: for the FP32 plans' narrower kernel the node-owned interpolation measured faster)
inline bool interp_is_tiled(const HostTables& H, bool fp64) { return kInterpTile && H.tile[0] == 8 && fp64; }

// Builds every host table of a plan.  Returns an empty string on success or an error message.
std::string build_tables(const ddi_params& p, HostTables& t, int* status);

// Accurate e^{-2 pi i k / n}, k in [0, n), interleaved (re, im).
std::vector<double> twiddle_table(int n);

// ---------------------------------------------------------------- device side
template <typename T>
struct Complex {
  T re, im;
};

// Remap a block index so that consecutive logical blocks run on the same XCD:
// blocks are dispatched round-robin over the 8 XCDs, each with its own L2.
__device__ inline int xcd_remap(int b, int nb) {
  constexpr int X = 8;
  const int x = b % X, local = b / X;
  const int base = nb / X, rem = nb % X;
  return x * base + (x < rem ? x : rem) + local;
}

#define DDI_CHECK(x)                 \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) return e_; \
  } while (0)

// Workspace of the GPE kernels on an N0 x N1 x N2 grid of the plan's real type T.
struct GpeWork {
  void* rho = nullptr;           // T[N]
  void* phi = nullptr;           // T[N]
  void* phit = nullptr;          // T[N]
  void* c1 = nullptr;            // Complex<T>[N]
  void* c2 = nullptr;            // Complex<T>[N] (gradient flow only)
  double* red = nullptr;         // reduction scratch: gpe_red_doubles(red_blocks) doubles
  int red_blocks = 0;
};
// Doubles of the reduction scratch: 4 slots per block for two reductions, then 8 scalars (the
// gradient flow's alpha), then the 5 energies (at offset 8 nb + 8).
inline size_t gpe_red_doubles(int nb) { return 8 * static_cast<size_t>(nb) + 16; }

// Device-resident plan state.
struct DevicePlan {
  HostTables H;
  bool mixed = false;
  int device = 0;
  // tables
  void* nodes = nullptr;         // NodeRec<T>[M]
  double* c_scaled = nullptr;    // c_q * prod(h) [M]
  double* deconv[3] = {nullptr, nullptr, nullptr};
  double* c_half = nullptr;       // half_factor * c_q * prod(h) [M]
  double* ones = nullptr;         // [max N]: unit factors for the split's padded FFT passes
  // split: I_1 runs on its own stream (default priority) into its own padded grid, overlapping
  // I_2; events fork it from and join it to the caller's stream
  void* fine_short = nullptr;     // Complex<T>[nf0*nf1*nf2]
  // ddi_set_dipole (allocated on its first call): node coordinates and the weights without the
  // symbol, scaled as c_scaled and c_half
  double* kq = nullptr;           // [M][3]
  double* base_scaled = nullptr;  // base * prod(h) [M]
  double* base_half = nullptr;    // half_factor * base * prod(h) [M]
  hipStream_t aux = nullptr;
  hipEvent_t ev_fork = nullptr, ev_long = nullptr, ev_join = nullptr;
  struct DevSchedule {
    int32_t* list = nullptr;
    SpreadItem* items = nullptr;
    ReduceItem* reduces = nullptr;
    InterpItem* interp_items = nullptr;
    int32_t* interp_direct = nullptr;
    int32_t* gptr = nullptr;
    int32_t* gpos = nullptr;
    int32_t* ent = nullptr;
  } dsched[2];
  bool interp_lds_ready = false;
  void* twiddles[kTwSlots] = {}; // per FFT length n (slot tw_slot(n) of fft.h): Complex<T>[n]
  // workspace
  void* fine = nullptr;          // Complex<T>[nf0*nf1*nf2]
  void* gnodes = nullptr;        // Complex<T>[M]
  void* partial = nullptr;       // Complex<T>[nslots][tile volume]
  void* ipartial = nullptr;      // Complex<double>[spread entries]: interpolation partial sums
  void* pads = nullptr;          // T[M + 1][3][kRowLen]: weight rows (one 128-byte line per row in
                                 // FP64), then a zero record that positions outside a window read
  int64_t workspace_bytes = 0;
  // GPE workspace (allocated on first use)
  GpeWork gpe;
};

// Kernel launchers (kernels.hip), templated on the real type.
template <typename T>
hipError_t run_type2(DevicePlan& P, int which, const T* rho, Complex<T>* out, const double* scale,
                     double cscalar, int sign, hipStream_t s, hipEvent_t* ev);
template <typename T>
hipError_t run_type1(DevicePlan& P, int which, const Complex<T>* g, T* phi, int sign, hipStream_t s,
                     hipEvent_t* ev);
template <typename T>
hipError_t run_apply(DevicePlan& P, const T* rho, T* phi, int sign, hipStream_t s, hipEvent_t* ev);
// I_1 of the split (Eq. 3.9): padded FFT, (1 - q) Uhat, inverse FFT into fine_short (front),
// then the last inverse pass added to phi (back).
template <typename T>
hipError_t split_short_front(DevicePlan& P, const T* rho, hipStream_t s);
template <typename T>
hipError_t split_short_back(DevicePlan& P, T* phi, hipStream_t s);
// Re-evaluate c_scaled and c_half for new dipole axes from kq, base_scaled and base_half.
hipError_t run_set_dipole(DevicePlan& P, const double* n, const double* m, hipStream_t s);
// The operator of the plan: run_apply, plus I_1 for a split plan (I_1 is its own transpose).
template <typename T>
hipError_t run_ddi(DevicePlan& P, const T* rho, T* phi, int sign, hipStream_t s, hipEvent_t* ev);
constexpr int kStages = 9;
template <typename T>
hipError_t run_gpe_energy_grad(DevicePlan& P, const GpeWork& W, const gpe_params& gp, const Complex<T>* psi,
                               double* E_dev, Complex<T>* grad, hipStream_t s);
template <typename T>
hipError_t run_gf_step(DevicePlan& P, const gpe_params& gp, double dt, int n_inner, const Complex<T>* psi_in,
                       Complex<T>* psi_out, double* residual, hipStream_t s);
template <typename T>
hipError_t run_ts_step(DevicePlan& P, const gpe_params& gp, double dt, double delta, double q,
                       const Complex<T>* psi_in, Complex<T>* psi_out, hipStream_t s);
template <typename T>
int gpe_reduction_blocks(const DevicePlan& P);

}  // namespace ddi
