// Plan-time tables (host, FP64): quadrature of Eq. DDI-Trun1, Nyquist mask,
// dipolar symbol (Eqs. DipKer, dipmn), exponential-of-semicircle kernel and
// its Fourier transform, node binning and the tiled spread schedule.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>

#include "ddi_internal.h"

namespace ddi {

namespace {

constexpr long double kPiL = 3.141592653589793238462643383279502884L;

bool is_pow2(int64_t v) { return v > 0 && (v & (v - 1)) == 0; }
// grid sizes the FFT passes take: 2^a, or 3 * 2^a (radix 3 in the first pass)
bool fft_size(int64_t v) { return is_pow2(v) || (v % 3 == 0 && is_pow2(v / 3)); }

// n-point Gauss-Legendre rule on [-1, 1]: Newton's method on P_n evaluated by
// the three-term recurrence, carried in long double.
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    long double z = cosl(kPiL * (i + 0.75L) / (n + 0.5L));
    long double dp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = z;
      for (int j = 1; j < n; ++j) {
        long double p2 = ((2 * j + 1) * z * p1 - j * p0) / (j + 1);
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) { p0 = 1.0L; p1 = z; }
      dp = n * (z * p1 - p0) / (z * z - 1.0L);
      long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    long double p0 = 1.0L, p1 = z;
    for (int j = 1; j < n; ++j) {
      long double p2 = ((2 * j + 1) * z * p1 - j * p0) / (j + 1);
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0L);
    // nodes in increasing order
    x[n - 1 - i] = static_cast<double>(z);
    w[n - 1 - i] = static_cast<double>(2.0L / ((1.0L - z * z) * dp * dp));
  }
}

// Exponential-of-semicircle kernel psi(z) = exp(beta (sqrt(1 - (2z/w)^2) - 1)), |z| < w/2: the
// spreading kernel of Barnett, Magland & af Klinteberg, "A parallel nonuniform fast Fourier
// transform library based on an 'exponential of semicircle' kernel", SIAM J. Sci. Comput. 41(5),
// C479-C504 (2019), with their shape parameter beta = 2.30 w for upsampling factor 2.
double es_kernel(double z, int w, double beta) {
  double a = 2.0 * z / w;
  double s = 1.0 - a * a;
  if (s <= 0.0) return 0.0;
  return std::exp(beta * (std::sqrt(s) - 1.0));
}

// phihat(m) = int psi(z) cos(2 pi m z / nf) dz over [-w/2, w/2], by a 128-point
// Gauss-Legendre rule on each half (the integrand is even).
double es_fourier(double m, int nf, int w, double beta, const std::vector<double>& gx,
                  const std::vector<double>& gw) {
  double half = 0.5 * w;
  long double acc = 0.0L;
  for (size_t i = 0; i < gx.size(); ++i) {
    double z = 0.5 * half * (gx[i] + 1.0);
    acc += (long double)gw[i] * es_kernel(z, w, beta) * std::cos(2.0 * M_PI * m * z / nf);
  }
  return static_cast<double>(2.0L * 0.5L * half * acc);
}

// Dispatch order for work items that are listed in spatial order: cut the list into
// kXcd contiguous segments of about equal work and interleave them, so that with the
// round-robin assignment of workgroups to XCDs (workgroup b runs on XCD b mod kXcd)
// each XCD works through one compact region of the grid and its L2 sees the reuse.
// Shorter segments are padded with `pad` items, which the kernels skip.
template <typename Item, typename Work>
std::vector<Item> xcd_order(const std::vector<Item>& items_in, Work work, const Item& pad, bool heavy_first = false) {
  constexpr int kXcd = 8;
  if (items_in.size() < 2 * kXcd) return items_in;
  std::vector<Item> items = items_in;
  double total = 0.0;
  for (const Item& it : items) total += work(it);
  std::vector<size_t> cut(kXcd + 1, items.size());
  cut[0] = 0;
  double acc = 0.0;
  int seg = 1;
  for (size_t i = 0; i < items.size() && seg < kXcd; ++i) {
    acc += work(items[i]);
    if (acc >= total * seg / kXcd) cut[seg++] = i + 1;
  }
  if (heavy_first)   // inside each region, the heaviest items first (the long ones start early)
    for (int x = 0; x < kXcd; ++x)
      std::stable_sort(items.begin() + cut[x], items.begin() + cut[x + 1],
                       [&](const Item& a, const Item& b) { return work(a) > work(b); });
  size_t longest = 0;
  for (int x = 0; x < kXcd; ++x) longest = std::max(longest, cut[x + 1] - cut[x]);
  std::vector<Item> out(longest * kXcd, pad);
  for (int x = 0; x < kXcd; ++x)
    for (size_t j = 0; j < cut[x + 1] - cut[x]; ++j) out[j * kXcd + x] = items[cut[x] + j];
  return out;
}

// Morton (Z-order) key of a 3D block coordinate (each coordinate < 2^20): consecutive
// keys stay compact in all three directions, so work that runs at the same time on one
// XCD touches nearby grid rows and its L2 sees the reuse.
uint64_t morton3(uint32_t x, uint32_t y, uint32_t z) {
  auto spread = [](uint64_t v) {
    v &= 0xFFFFF;
    v = (v | (v << 32)) & 0x1F00000000FFFFull;
    v = (v | (v << 16)) & 0x1F0000FF0000FFull;
    v = (v | (v << 8)) & 0x100F00F00F00F00Full;
    v = (v | (v << 4)) & 0x10C30C30C30C30C3ull;
    v = (v | (v << 2)) & 0x1249249249249249ull;
    return v;
  };
  return (spread(x) << 2) | (spread(y) << 1) | spread(z);
}

}  // namespace

namespace {

// Interpolation work over the nodes selected by `used` (a prefix of every group block in
// plan order): blocks with at least kInterpMinGroup selected nodes become LDS-staged items
// (split into chunks), the other selected nodes are interpolated directly.
template <typename Used>
std::string build_interp_schedule(const HostTables& t, const std::vector<uint64_t>& key, Used used, Schedule& S) {
  const int64_t M = t.M;
  const int chunk_i = 256;
  S.interp_items.clear();
  S.interp_direct.clear();
  for (int64_t b = 0; b < M;) {
    int64_t e = b;
    while (e < M && key[e] == key[b]) ++e;
    int64_t ue = b;
    while (ue < e && used(ue)) ++ue;
    if (ue - b >= kInterpMinGroup) {
      int org[3];
      for (int a = 0; a < 3; ++a) org[a] = (t.l0[3 * b + a] / t.ib[a]) * t.ib[a];
      for (int64_t c = b; c < ue; c += chunk_i) {
        InterpItem it{};
        it.start = static_cast<int32_t>(c);
        it.count = static_cast<int32_t>(std::min<int64_t>(chunk_i, ue - c));
        for (int a = 0; a < 3; ++a) it.org[a] = org[a];
        S.interp_items.push_back(it);
      }
    } else {
      for (int64_t c = b; c < ue; ++c) S.interp_direct.push_back(static_cast<int32_t>(c));
    }
    b = e;
  }
  // heaviest items first so that the long ones start early
  std::stable_sort(S.interp_items.begin(), S.interp_items.end(),
                   [](const InterpItem& x, const InterpItem& y) { return x.count > y.count; });
  return "";
}

// Spread work over the nodes selected by `used`: for every tile of the fine grid, the
// selected nodes whose support meets it (tiles in Morton order); tiles with more than
// `chunk` nodes are split into chunks whose partial tiles are summed by reduce items.
template <typename Used>
std::string build_spread_schedule(const HostTables& t, const std::vector<int64_t>& tile_order, Used used,
                                  Schedule& S) {
  const int64_t M = t.M;
  const int64_t ntile_total = static_cast<int64_t>(t.ntiles[0]) * t.ntiles[1] * t.ntiles[2];
  auto touched = [&](int64_t s, int a, int* out) {
    int cnt = 0;
    for (int i = 0; i < t.W[a]; ++i) {
      int pos = (t.l0[3 * s + a] + i) % t.nf[a];
      int tl = pos / t.tile[a];
      bool seen = false;
      for (int j = 0; j < cnt; ++j) seen = seen || out[j] == tl;
      if (!seen) out[cnt++] = tl;
    }
    return cnt;
  };
  // last-axis window: the complement of the longest circular run of zalign-blocks that no
  // support touches (the whole axis when that run is empty or the axis is short)
  {
    const int n = t.nf[2], za = t.zalign;
    S.z0 = 0;
    S.nz = n;
    if (n % za == 0 && n >= 4 * za) {
      const int nb = n / za;
      std::vector<char> hit(nb, 0);
      for (int64_t s = 0; s < M; ++s) {
        if (!used(s)) continue;
        for (int i = 0; i < t.W[2]; ++i) hit[((t.l0[3 * s + 2] + i) % n) / za] = 1;
      }
      int best = 0, best_end = 0;
      for (int i = 0, run = 0; i < 2 * nb; ++i) {   // twice round: runs that wrap
        run = hit[i % nb] ? 0 : std::min(run + 1, nb);
        if (run > best) { best = run; best_end = i % nb; }
      }
      if (best > 0 && best < nb) {
        S.z0 = ((best_end + 1) % nb) * za;
        S.nz = (nb - best) * za;
      }
    }
  }
  // axis-1 window, centred on mode 0 (3D only): the smallest ny with every support inside the
  // signed positions [-ny/2, ny/2) and ny/2 a multiple of the tile extent, so that a tile lies
  // wholly inside or outside (the matrix-core interpolation multiplies whole tiles, and rows
  // outside the window are never transformed)
  {
    const int n = t.nf[1];
    S.ny = n;
    if (t.dim == 3) {
      int need = 2;
      for (int64_t s = 0; s < M; ++s) {
        if (!used(s)) continue;
        for (int i = 0; i < t.W[1]; ++i) {
          const int pos = (t.l0[3 * s + 1] + i) % n;
          const int sp = pos < n / 2 ? pos : pos - n;
          need = std::max(need, sp >= 0 ? 2 * (sp + 1) : -2 * sp);
        }
      }
      const int half = (need / 2 + t.tile[1] - 1) / t.tile[1] * t.tile[1];
      S.ny = std::min(n, 2 * half);
    }
  }
  auto in_window = [&](int z) { return ((z - S.z0) % t.nf[2] + t.nf[2]) % t.nf[2] < S.nz; };
  std::vector<int64_t> count(ntile_total + 1, 0);
  int tx[kWMax], ty[kWMax], tz[kWMax];
  for (int pass = 0; pass < 2; ++pass) {
    if (pass == 1) {
      for (int64_t i = 0, run = 0; i <= ntile_total; ++i) { int64_t c = count[i]; count[i] = run; run += c; }
      if (count[ntile_total] > (int64_t(1) << 31) - 1) return "spread schedule too large";
      S.list.assign(count[ntile_total], 0);
    }
    std::vector<int64_t> fill;
    if (pass == 1) fill.assign(count.begin(), count.end());
    for (int64_t s = 0; s < M; ++s) {
      if (!used(s)) continue;
      int nx = touched(s, 0, tx), ny = touched(s, 1, ty), nz = touched(s, 2, tz);
      for (int i = 0; i < nx; ++i)
        for (int j = 0; j < ny; ++j)
          for (int k = 0; k < nz; ++k) {
            int64_t tid = (static_cast<int64_t>(tx[i]) * t.ntiles[1] + ty[j]) * t.ntiles[2] + tz[k];
            if (pass == 0) count[tid]++;
            else S.list[fill[tid]++] = static_cast<int32_t>(s);
          }
    }
  }
  // chunk length of the matrix-core kernels: the tuned maximum, or shorter when the entries
  // would otherwise fill fewer items than the 4096 waves the spread keeps resident (a small
  // ball of nodes crowds a few tiles, and one wave per long chunk then sets the duration)
  int chunk = kSpreadChunk;
  const int64_t per_wave = (count[ntile_total] + kSpreadWaves - 1) / kSpreadWaves;
  if (t.row_windows && kSpreadMfma) {
    chunk = static_cast<int>(std::min<int64_t>(kSpreadChunkMfma, std::max<int64_t>(32, (per_wave + 15) / 16 * 16)));
  } else if (t.dim == 2) {
    // 2D: a few thousand tiles hold all the entries, one wave each, so the hot tiles (many nodes near
    // k = 0) set the duration; chunks of about entries / resident waves (at least kSpreadChunk2d)
    chunk = static_cast<int>(std::min<int64_t>(kSpreadChunk, std::max<int64_t>(kSpreadChunk2d, per_wave)));
  }
  S.items.clear();
  S.reduces.clear();
  int32_t slot = 0;
  for (int64_t tord = 0; tord < ntile_total; ++tord) {
    const int64_t tid = tile_order[tord];
    int64_t beg = count[tid], n = count[tid + 1] - count[tid];
    if (!in_window(static_cast<int>(tid % t.ntiles[2]) * t.tile[2])) {
      if (n > 0) return "internal: a node support outside the last-axis window";
      continue;                              // never read: no item
    }
    if (n <= chunk) {
      S.items.push_back({static_cast<int32_t>(tid), static_cast<int32_t>(beg), static_cast<int32_t>(n), -1});
    } else {
      int nch = static_cast<int>((n + chunk - 1) / chunk);
      S.reduces.push_back({static_cast<int32_t>(tid), slot, nch, 0});
      for (int c = 0; c < nch; ++c) {
        int64_t b = beg + static_cast<int64_t>(c) * chunk;
        int64_t e = std::min(beg + n, b + chunk);
        S.items.push_back({static_cast<int32_t>(tid), static_cast<int32_t>(b), static_cast<int32_t>(e - b), slot++});
      }
    }
  }
#if DDI_SPREAD_XCD_ORDER
  // items are in tile (Morton) order; each XCD gets one contiguous region of equal work, so its
  // L2 holds the weight rows its tiles share; inside a region the heaviest items go first when
  // items are long (about 32 entries or more on average), else the Morton order is kept
  {
    const bool heavy_first = count[ntile_total] >= 32 * static_cast<int64_t>(S.items.size());
    S.items = xcd_order(S.items, [](const SpreadItem& it) { return 16.0 + it.count; }, SpreadItem{-1, 0, 0, -1},
                        heavy_first);
  }
#else
  // heaviest items first so that the long ones start early
  std::stable_sort(S.items.begin(), S.items.end(),
                   [](const SpreadItem& x, const SpreadItem& y) { return x.count > y.count; });
#endif
  S.nslots = slot;
  // weight-row offsets of every (tile, node) entry
  S.ent.clear();
  if (t.row_windows) {
    // kEntPad zero entries at the end: a kernel's block of 16 may read past its item's entries
    // (the kernels address the table with 32-bit byte offsets)
    if (static_cast<int64_t>(S.list.size() + kEntPad) * 2 * static_cast<int64_t>(sizeof(int32_t)) >= (int64_t(1) << 31))
      return "spread schedule too large";
    S.ent.assign(2 * (S.list.size() + kEntPad), 0);
    for (int64_t tid = 0; tid < ntile_total; ++tid) {
      const int64_t org[3] = {(tid / (static_cast<int64_t>(t.ntiles[2]) * t.ntiles[1])) * t.tile[0],
                              ((tid / t.ntiles[2]) % t.ntiles[1]) * t.tile[1], (tid % t.ntiles[2]) * t.tile[2]};
      for (int64_t i = count[tid]; i < count[tid + 1]; ++i) {
        const int32_t q = S.list[i];
        int32_t packed = 0;
        for (int a = 0; a < 3; ++a) {
          int64_t d = (org[a] - t.l0[3 * q + a]) % t.nf[a];
          if (d < 0) d += t.nf[a];
          if (d > t.nf[a] - t.tile[a]) d -= t.nf[a];     // the tile starts before the support
          if (d < -(t.tile[a] - 1) || d > t.W[a] - 1) return "entry offset outside the weight row";
          packed |= static_cast<int32_t>(kOffBias + d) << (8 * a);
        }
        S.ent[2 * i] = q;
        S.ent[2 * i + 1] = packed;
      }
    }
  }
  // per node, the positions of its entries in the list (in list order)
  S.gptr.assign(M + 1, 0);
  for (int32_t q : S.list) S.gptr[q + 1]++;
  for (int64_t q = 0; q < M; ++q) S.gptr[q + 1] += S.gptr[q];
  S.gpos.assign(S.list.size(), 0);
  {
    std::vector<int32_t> fillg(S.gptr.begin(), S.gptr.end() - 1);
    for (size_t i = 0; i < S.list.size(); ++i) S.gpos[fillg[S.list[i]]++] = static_cast<int32_t>(i);
  }
  return "";
}

}  // namespace

std::vector<double> twiddle_table(int n) {
  std::vector<double> t(2 * n);
  for (int k = 0; k < n; ++k) {
    long double a = 2.0L * kPiL * k / n;
    t[2 * k] = static_cast<double>(cosl(a));
    t[2 * k + 1] = static_cast<double>(-sinl(a));
  }
  return t;
}

std::string build_tables(const ddi_params& p, HostTables& t, int* status) {
  *status = DDI_EINVAL;
  if (p.dim != 2 && p.dim != 3) return "dim must be 2 or 3";
  const int d = p.dim;
  for (int a = 0; a < d; ++a) {
    if (!fft_size(p.n[a])) return "grid sizes must be powers of two or three times a power of two";
    if (!(p.L[a] > 0.0) || !std::isfinite(p.L[a])) return "L must be positive and finite";
  }
  double nn = std::sqrt(p.dip_n[0] * p.dip_n[0] + p.dip_n[1] * p.dip_n[1] + p.dip_n[2] * p.dip_n[2]);
  double nm = std::sqrt(p.dip_m[0] * p.dip_m[0] + p.dip_m[1] * p.dip_m[1] + p.dip_m[2] * p.dip_m[2]);
  if (!(nn > 0.0) || !std::isfinite(nn)) return "dipole axis n must be a non-zero finite vector";
  if (!std::isfinite(nm)) return "dipole axis m must be finite";
  if (p.n_rad < 1 || p.n_azi < 1 || (d == 3 && p.n_pol < 1)) return "quadrature sizes must be positive";
  if (p.n_rad > 65536 || p.n_azi > 65536 || (d == 3 && p.n_pol > 65536)) return "quadrature sizes too large";
  if (p.prec != DDI_FP64 && p.prec != DDI_MIXED) return "prec must be DDI_FP64 or DDI_MIXED";
  int w = p.kernel_width;
  if (w == 0) {
    if (!(p.tol > 0.0) || !(p.tol < 1.0)) return "tol must lie in (0, 1) when kernel_width is 0";
    w = static_cast<int>(std::ceil(-std::log10(p.tol))) + 1;
    w = std::min(kWMax, std::max(4, w));
  }
  if (w < 2 || w > kWMax) return "kernel_width must lie in [2, 16]";
  if (p.split != 0 && p.split != 1) return "split must be 0 or 1";
  if (p.split && !std::isfinite(p.split_s)) return "split_s must be finite";
  for (int a = 0; a < 3; ++a)
    if (!std::isfinite(p.stretch[a])) return "stretch must be finite";

  *status = DDI_ENOTSUP;
  // internal 3-axis layout: 2D grids live on axes 1 and 2
  const int off = 3 - d;
  for (int a = 0; a < 3; ++a) { t.N[a] = 1; t.nf[a] = 1; t.W[a] = 1; t.h[a] = 1.0; t.L[a] = 0.5; }
  for (int a = 0; a < d; ++a) {
    int64_t n = p.n[a];
    if (n < (d == 3 ? 8 : 32) || n > 512) return "grid size per axis must lie in [8, 512] (3D) or [32, 512] (2D)";
    t.N[off + a] = static_cast<int>(n);
    t.nf[off + a] = static_cast<int>(2 * n);
    t.W[off + a] = w;
    t.L[off + a] = p.L[a];
    t.h[off + a] = 2.0 * p.L[a] / n;
    if (t.nf[off + a] < 2 * w) return "grid too small for the kernel width";
  }
  t.dim = d;
  t.w = w;
  t.es_beta = 2.30 * w;     // the published choice for sigma = 2 (see es_kernel)
  t.cell = 1.0;
  for (int a = 0; a < 3; ++a) t.cell *= (a >= off ? t.h[a] : 1.0);
  if (d == 3) { t.tile[0] = 8; t.tile[1] = 8; t.tile[2] = kTileZ; }
  else { t.tile[0] = 1; t.tile[1] = 64; t.tile[2] = kTileZ; }
  for (int a = 0; a < 3; ++a) {
    t.ib[a] = t.N[a] == 1 ? 1 : (d == 3 ? kInterpBlock3 : 8);
    t.ireg[a] = t.ib[a] + t.W[a] - 1;
  }
  for (int a = 0; a < 3; ++a) {
    if (t.nf[a] % t.tile[a] != 0)   // (only for 3 * 2^a: the fine grid of a 2D axis below 96 points)
      return "the oversampled grid must be a multiple of the spread tile (64 on the first axis of a 2D grid)";
    t.ntiles[a] = t.nf[a] / t.tile[a];
  }

  // ---------------------------------------------------------------- quadrature
  double hp[3] = {0, 0, 0};      // h in paper axes
  for (int a = 0; a < d; ++a) hp[a] = 2.0 * p.L[a] / p.n[a];
  // split (Eq. 3.9): I_1's kernel, the inverse transform of (1 - q) Uhat, decays like
  // exp(-s^2 r^2 / 4) and the nearest image of the zero-padded box lies 2 L_min away, so
  // s^2 L_min^2 = ln(1/tol); q rhohat falls below tol at |k| = s sqrt(ln(1/tol)).
  double split_s = 0.0, ln_tol = 0.0;
  if (p.split) {
    const double tol_eff = (p.tol > 0.0 && p.tol < 1.0) ? p.tol : std::pow(10.0, -(w - 1));
    ln_tol = std::log(1.0 / tol_eff);
    double lmin = p.L[0];
    for (int a = 1; a < d; ++a) lmin = std::min(lmin, p.L[a]);
    split_s = p.split_s > 0.0 ? p.split_s : std::sqrt(ln_tol) / lmin;
  }
  t.split = p.split != 0;
  t.split_s = split_s;
  // stretched rule (anisotropic boxes): k = S k', W = W' det S; kmax is the radius in k'
  double S[3] = {1.0, 1.0, 1.0};
  double detS = 1.0;
  for (int a = 0; a < d; ++a) {
    S[a] = p.stretch[a] > 0.0 ? p.stretch[a] : 1.0;
    detS *= S[a];
  }
  double kmax = p.kmax;
  if (!(kmax > 0.0)) {
    if (p.split) {
      double smin = S[0];
      for (int a = 1; a < d; ++a) smin = std::min(smin, S[a]);
      kmax = split_s * std::sqrt(ln_tol) / smin;   // the ellipsoid holds the ball where q matters
    } else {
      double s = 0.0;
      for (int a = 0; a < d; ++a) s += 1.0 / (hp[a] * S[a] * hp[a] * S[a]);
      kmax = M_PI * std::sqrt(s);
    }
  }
  t.kmax = kmax;
  double nv[3], mv[3];
  // the axes are used as given: the paper prints its unit vectors to five digits
  for (int i = 0; i < 3; ++i) nv[i] = p.dip_n[i];
  if (nm > 0.0) for (int i = 0; i < 3; ++i) mv[i] = p.dip_m[i];
  else for (int i = 0; i < 3; ++i) mv[i] = nv[i];
  for (int i = 0; i < 3; ++i) { t.nv[i] = nv[i]; t.mv[i] = mv[i]; }

  std::vector<double> tr, wr, tu, wu;
  gauss_legendre(static_cast<int>(p.n_rad), tr, wr);
  const int npol = d == 3 ? static_cast<int>(p.n_pol) : 1;
  if (d == 3) gauss_legendre(npol, tu, wu);
  const int nazi = static_cast<int>(p.n_azi);
  std::vector<double> cphi(nazi), sphi(nazi);
  for (int c = 0; c < nazi; ++c) {
    double ph = 2.0 * M_PI * c / nazi;
    cphi[c] = std::cos(ph);
    sphi[c] = std::sin(ph);
  }
  const double wphi = 2.0 * M_PI / nazi;
  const double inv2pid = 1.0 / std::pow(2.0 * M_PI, d);
  t.m_nominal = static_cast<int64_t>(p.n_rad) * npol * nazi;

  std::vector<int32_t> idx_nat;
  std::vector<double> k_nat, c_nat, base_nat;
  for (int ia = 0; ia < p.n_rad; ++ia) {
    double r = 0.5 * kmax * (1.0 + tr[ia]);
    double wrad = 0.5 * kmax * wr[ia];
    for (int ib = 0; ib < npol; ++ib) {
      double u = d == 3 ? tu[ib] : 0.0;
      double su = d == 3 ? std::sqrt(1.0 - u * u) : 1.0;
      for (int ic = 0; ic < nazi; ++ic) {
        double k[3];
        double W;
        if (d == 3) {
          k[0] = r * su * cphi[ic];
          k[1] = r * su * sphi[ic];
          k[2] = r * u;
          W = wrad * r * r * wu[ib] * wphi;
        } else {
          k[0] = r * cphi[ic];
          k[1] = r * sphi[ic];
          k[2] = 0.0;
          W = wrad * r * wphi;
        }
        for (int a = 0; a < d; ++a) k[a] *= S[a];
        W *= detS;
        if (p.nyquist_mask) {
          bool inside = true;
          for (int a = 0; a < d; ++a) inside = inside && (std::fabs(k[a]) <= M_PI / hp[a]);
          if (!inside) continue;
        }
        double U;
        double kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
        if (d == 3) {
          double kn = k[0] * nv[0] + k[1] * nv[1] + k[2] * nv[2];
          double km = k[0] * mv[0] + k[1] * mv[1] + k[2] * mv[2];
          U = 3.0 * kn * km / kk - (nv[0] * mv[0] + nv[1] * mv[1] + nv[2] * mv[2]);
        } else {
          double kn = k[0] * nv[0] + k[1] * nv[1];
          double km = k[0] * mv[0] + k[1] * mv[1];
          U = 3.0 * (kn * km - nv[2] * mv[2] * kk) / (2.0 * std::sqrt(kk));
        }
        idx_nat.push_back(ia);
        idx_nat.push_back(d == 3 ? ib : 0);
        idx_nat.push_back(ic);
        k_nat.push_back(k[0]);
        k_nat.push_back(k[1]);
        k_nat.push_back(k[2]);
        // split: I_2 carries q(k) = exp(-|k|^2/s^2) (3D) or erfc(|k|/s) (2D)
        const double qk = !t.split ? 1.0
                          : (d == 3 ? std::exp(-kk / (split_s * split_s)) : std::erfc(std::sqrt(kk) / split_s));
        c_nat.push_back(W * U * inv2pid * qk);
        base_nat.push_back(W * inv2pid * qk);
      }
    }
  }
  const int64_t M = static_cast<int64_t>(c_nat.size());
  if (M == 0) { *status = DDI_EINVAL; return "no quadrature node lies inside the Nyquist box"; }
  if (M > (int64_t(1) << 30)) return "too many quadrature nodes";
  t.M = M;

  // ---------------------------------------------------------------- kernel geometry per node
  std::vector<int32_t> l0_nat(3 * M);
  std::vector<double> w_nat(static_cast<size_t>(3 * kWMax) * M, 0.0);
  std::vector<uint64_t> home(M);
  for (int64_t q = 0; q < M; ++q) {
    uint32_t hb[3] = {0, 0, 0};
    for (int a = 0; a < 3; ++a) {
      int l0 = 0;
      double* wq = &w_nat[(q * 3 + a) * kWMax];
      if (t.N[a] == 1) {
        wq[0] = 1.0;
      } else {
        int pa = a - off;                       // paper axis
        double tq = k_nat[3 * q + pa] * t.h[a]; // in [-pi, pi] when masked
        double tau = tq * t.nf[a] / (2.0 * M_PI);
        l0 = static_cast<int>(std::ceil(tau - 0.5 * w));
        for (int i = 0; i < w; ++i) wq[i] = es_kernel(l0 + i - tau, w, t.es_beta);
        l0 %= t.nf[a];
        if (l0 < 0) l0 += t.nf[a];
      }
      l0_nat[3 * q + a] = l0;
      hb[a] = static_cast<uint32_t>(l0 / t.ib[a]);
    }
    home[q] = morton3(hb[0], hb[1], hb[2]);
  }
  // ---------------------------------------------------------------- +-k pairs
  // The tensor rule is symmetric under k -> -k: (a, b, c) pairs with (a, n_pol-1-b,
  // c + n_azi/2) (2D: (a, c + n_azi/2)), with equal weight and symbol.  On real grids the two
  // terms of a pair are complex conjugates, so one member carries factor 2 and the other 0;
  // a node whose partner the mask removed (or any node when n_azi is odd) keeps factor 1.
  std::vector<double> hf_nat(M, 1.0);
  if (nazi % 2 == 0) {
    std::vector<int64_t> pos(static_cast<size_t>(p.n_rad) * npol * nazi, -1);
    for (int64_t q = 0; q < M; ++q)
      pos[(static_cast<size_t>(idx_nat[3 * q]) * npol + idx_nat[3 * q + 1]) * nazi + idx_nat[3 * q + 2]] = q;
    for (int64_t q = 0; q < M; ++q) {
      const int a = idx_nat[3 * q], b = idx_nat[3 * q + 1], c = idx_nat[3 * q + 2];
      const int bp = d == 3 ? npol - 1 - b : 0;
      const int cp = (c + nazi / 2) % nazi;
      const int64_t pq = pos[(static_cast<size_t>(a) * npol + bp) * nazi + cp];
      if (pq >= 0 && pq != q) hf_nat[q] = q < pq ? 2.0 : 0.0;
    }
  }

  // sort nodes by the interpolation group (the block of ib^3 cells holding the start of
  // their support), members of the half set first inside a group; stable otherwise
  std::vector<int64_t> perm(M);
  std::iota(perm.begin(), perm.end(), 0);
  std::stable_sort(perm.begin(), perm.end(), [&](int64_t x, int64_t y) {
    if (home[x] != home[y]) return home[x] < home[y];
    return (hf_nat[x] > 0.0) > (hf_nat[y] > 0.0);
  });
  t.index.resize(3 * M);
  t.k.resize(3 * M);
  t.c.resize(M);
  t.base.resize(M);
  t.half_factor.resize(M);
  t.l0.resize(3 * M);
  t.wts.resize(static_cast<size_t>(3 * kWMax) * M);
  std::vector<uint64_t> key(M);
  for (int64_t s = 0; s < M; ++s) {
    int64_t q = perm[s];
    for (int a = 0; a < 3; ++a) {
      t.index[3 * s + a] = idx_nat[3 * q + a];
      t.k[3 * s + a] = k_nat[3 * q + a];
      t.l0[3 * s + a] = l0_nat[3 * q + a];
    }
    t.c[s] = c_nat[q];
    t.base[s] = base_nat[q];
    t.half_factor[s] = hf_nat[q];
    key[s] = home[q];
    std::memcpy(&t.wts[static_cast<size_t>(s) * 3 * kWMax], &w_nat[static_cast<size_t>(q) * 3 * kWMax],
                sizeof(double) * 3 * kWMax);
  }

  // ---------------------------------------------------------------- deconvolution 1/phihat
  {
    std::vector<double> gx, gw;
    gauss_legendre(128, gx, gw);
    for (int a = 0; a < 3; ++a) {
      t.deconv[a].assign(t.N[a], 1.0);
      if (t.N[a] == 1) continue;
      for (int c = 0; c < t.N[a]; ++c) {
        double m = c - t.N[a] / 2;
        t.deconv[a][c] = 1.0 / es_fourier(m, t.nf[a], w, t.es_beta, gx, gw);
      }
    }
  }

  // ---------------------------------------------------------------- schedules
  const int64_t ntile_total = static_cast<int64_t>(t.ntiles[0]) * t.ntiles[1] * t.ntiles[2];
  if (ntile_total > (int64_t(1) << 30)) return "fine grid too large";
  std::vector<int64_t> tile_order(ntile_total);
  {
    std::vector<uint64_t> tkey(ntile_total);
    for (int64_t tid = 0; tid < ntile_total; ++tid) {
      const uint32_t tz = static_cast<uint32_t>(tid % t.ntiles[2]);
      const uint32_t ty = static_cast<uint32_t>((tid / t.ntiles[2]) % t.ntiles[1]);
      const uint32_t tx = static_cast<uint32_t>(tid / (static_cast<int64_t>(t.ntiles[2]) * t.ntiles[1]));
      tkey[tid] = morton3(tx, ty, tz);
      tile_order[tid] = tid;
    }
    std::stable_sort(tile_order.begin(), tile_order.end(),
                     [&](int64_t x, int64_t y) { return tkey[x] < tkey[y]; });
  }
  // (the matrix-core kernels address the weight rows with 32-bit byte offsets)
  t.zalign = p.prec == DDI_FP64 ? 8 : 16;
  t.row_windows = t.dim == 3 && (t.M + 1) * 3 * kRowLen * static_cast<int64_t>(sizeof(double)) < (int64_t(1) << 31);
  for (int a = 0; a < 3; ++a) t.row_windows = t.row_windows && t.tile[a] == 8 && t.nf[a] >= t.W[a] + 8;
  for (int which = 0; which < 2; ++which) {
    Schedule& S = t.sched[which];
    auto used = [&](int64_t s2) { return which == kAll || t.half_factor[s2] > 0.0; };
    std::string err = build_interp_schedule(t, key, used, S);
    if (err.empty()) err = build_spread_schedule(t, tile_order, used, S);
    if (!err.empty()) return err;
  }
  *status = DDI_OK;
  return "";
}

}  // namespace ddi
