// C ABI of libddi (declared in include/ddi.h): plan construction, device
// uploads, argument checks and dispatch on the precision.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <string>

#include "alloc_group.h"
#include "ddi_internal.h"
#include "fft.h"

struct ddi_plan_s {
  ddi::DevicePlan P;
};

namespace {

thread_local std::string g_err;

ddi_status fail(ddi_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

ddi_status hip_fail(hipError_t e, const char* what) {
  g_err = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? DDI_ENOMEM : DDI_EDEVICE;
}

#define HIP_TRY(call, what)                        \
  do {                                             \
    hipError_t e_ = (call);                        \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

template <typename X>
hipError_t upload(X** dst, const X* src, size_t count, hipStream_t s, int64_t& bytes) {
  if (count == 0) { *dst = nullptr; return hipSuccess; }
  hipError_t e = hipMalloc(reinterpret_cast<void**>(dst), count * sizeof(X));
  if (e != hipSuccess) return e;
  bytes += static_cast<int64_t>(count * sizeof(X));
  return hipMemcpyAsync(*dst, src, count * sizeof(X), hipMemcpyHostToDevice, s);
}

void free_plan(ddi::DevicePlan& P) {
  if (P.aux) (void)hipStreamSynchronize(P.aux);
  for (hipEvent_t e : {P.ev_fork, P.ev_long, P.ev_join})
    if (e) (void)hipEventDestroy(e);
  if (P.aux) (void)hipStreamDestroy(P.aux);
  void* ptrs[] = {P.nodes, P.c_scaled, P.c_half, P.ones, P.fine_short, P.kq, P.base_scaled, P.base_half,
                  P.deconv[0], P.deconv[1], P.deconv[2],
                  P.fine, P.gnodes, P.partial, P.ipartial, P.pads, P.gpe.rho, P.gpe.phi, P.gpe.phit, P.gpe.c1, P.gpe.c2, P.gpe.red};
  for (auto& d : P.dsched) {
    void* sp[] = {d.list, d.items, d.reduces, d.interp_items, d.interp_direct, d.gptr, d.gpos, d.ent};
    for (void* p : sp)
      if (p) (void)hipFree(p);
  }
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  for (void* p : P.twiddles)
    if (p) (void)hipFree(p);
}

template <typename T>
ddi_status build_device(ddi::DevicePlan& P, hipStream_t s, std::vector<ddi::NodeRec<T>>& recs,
                        std::vector<std::vector<ddi::Complex<T>>>& tws, std::vector<T>& padrows) {
  const ddi::HostTables& H = P.H;
  int64_t& bytes = P.workspace_bytes;
  recs.resize(H.M);
  for (int64_t q = 0; q < H.M; ++q) {
    ddi::NodeRec<T>& r = recs[q];
    std::memset(&r, 0, sizeof(r));
    for (int a = 0; a < 3; ++a) {
      r.l0[a] = H.l0[3 * q + a];
      for (int i = 0; i < ddi::kWMax; ++i) r.w[a][i] = static_cast<T>(H.wts[(q * 3 + a) * ddi::kWMax + i]);
    }
  }
  ddi::NodeRec<T>* dn = nullptr;
  HIP_TRY(upload(&dn, recs.data(), recs.size(), s, bytes), "upload node table");
  P.nodes = dn;
  std::vector<double> cs(H.M), cs_half(H.M);
  for (int64_t q = 0; q < H.M; ++q) cs[q] = H.c[q] * H.cell;
  HIP_TRY(upload(&P.c_scaled, cs.data(), cs.size(), s, bytes), "upload weights");
  for (int64_t q = 0; q < H.M; ++q) cs_half[q] = H.half_factor[q] * H.c[q] * H.cell;
  HIP_TRY(upload(&P.c_half, cs_half.data(), cs_half.size(), s, bytes), "upload weights");
  for (int a = 0; a < 3; ++a)
    HIP_TRY(upload(&P.deconv[a], H.deconv[a].data(), H.deconv[a].size(), s, bytes), "upload deconvolution");
  if (H.split) {
    const std::vector<double> ones(std::max(H.N[0], std::max(H.N[1], H.N[2])), 1.0);
    HIP_TRY(upload(&P.ones, ones.data(), ones.size(), s, bytes), "upload unit factors");
  }
  // tile-owned interpolation (FP64 in 3D) and the weight rows of the matrix-core kernels
  const bool tile_interp = ddi::interp_is_tiled(H, sizeof(T) == 8);
  const bool use_pads = ddi::uses_weight_rows(H);
  for (int w = 0; w < 2; ++w) {
    const ddi::Schedule& S = H.sched[w];
    auto& D = P.dsched[w];
    HIP_TRY(upload(&D.list, S.list.data(), S.list.size(), s, bytes), "upload spread lists");
    HIP_TRY(upload(&D.items, S.items.data(), S.items.size(), s, bytes), "upload spread items");
    HIP_TRY(upload(&D.reduces, S.reduces.data(), S.reduces.size(), s, bytes), "upload spread reduces");
    HIP_TRY(upload(&D.interp_items, S.interp_items.data(), S.interp_items.size(), s, bytes), "upload interp groups");
    HIP_TRY(upload(&D.interp_direct, S.interp_direct.data(), S.interp_direct.size(), s, bytes),
            "upload interp list");
    if (tile_interp) {
      HIP_TRY(upload(&D.gptr, S.gptr.data(), S.gptr.size(), s, bytes), "upload interp gather");
      HIP_TRY(upload(&D.gpos, S.gpos.data(), S.gpos.size(), s, bytes), "upload interp gather");
    }
    if (use_pads) HIP_TRY(upload(&D.ent, S.ent.data(), S.ent.size(), s, bytes), "upload entry table");
  }
  if (use_pads) {
    padrows.assign(static_cast<size_t>(H.M + 1) * 3 * ddi::kRowLen, T(0));   // + the zero record
    for (int64_t q = 0; q < H.M; ++q)
      for (int a = 0; a < 3; ++a)
        for (int i = 0; i < ddi::kWMax; ++i)
          padrows[(q * 3 + a) * ddi::kRowLen + i] = static_cast<T>(H.wts[(q * 3 + a) * ddi::kWMax + i]);
    T* dp = nullptr;
    HIP_TRY(upload(&dp, padrows.data(), padrows.size(), s, bytes), "upload weight rows");
    P.pads = dp;
  }
  // twiddles for every FFT length used: fine grid sizes and the unpadded sizes
  tws.assign(ddi::kTwSlots, {});
  for (int a = 0; a < 3; ++a) {
    for (int n : {H.nf[a], H.N[a]}) {
      if (n < 2) continue;
      const int l = ddi::tw_slot(n);
      if (P.twiddles[l]) continue;
      std::vector<double> t = ddi::twiddle_table(n);
      tws[l].resize(n);
      for (int k = 0; k < n; ++k) tws[l][k] = {static_cast<T>(t[2 * k]), static_cast<T>(t[2 * k + 1])};
      ddi::Complex<T>* d = nullptr;
      HIP_TRY(upload(&d, tws[l].data(), tws[l].size(), s, bytes), "upload twiddles");
      P.twiddles[l] = d;
    }
  }
  const int64_t nfine = static_cast<int64_t>(H.nf[0]) * H.nf[1] * H.nf[2];
  HIP_TRY(hipMalloc(&P.fine, nfine * sizeof(ddi::Complex<T>)), "allocate fine grid");
  bytes += nfine * static_cast<int64_t>(sizeof(ddi::Complex<T>));
  if (H.split) {
    // I_1 of the split runs beside I_2: its own padded grid, stream (default priority) and events
    HIP_TRY(hipMalloc(&P.fine_short, nfine * sizeof(ddi::Complex<T>)), "allocate the split's padded grid");
    bytes += nfine * static_cast<int64_t>(sizeof(ddi::Complex<T>));
    HIP_TRY(hipStreamCreateWithFlags(&P.aux, hipStreamNonBlocking), "create the split's stream");
    HIP_TRY(hipEventCreateWithFlags(&P.ev_fork, hipEventDisableTiming), "create the split's events");
    HIP_TRY(hipEventCreateWithFlags(&P.ev_long, hipEventDisableTiming), "create the split's events");
    HIP_TRY(hipEventCreateWithFlags(&P.ev_join, hipEventDisableTiming), "create the split's events");
  }
  HIP_TRY(hipMalloc(&P.gnodes, H.M * sizeof(ddi::Complex<T>)), "allocate node values");
  bytes += H.M * static_cast<int64_t>(sizeof(ddi::Complex<T>));
  const size_t nentries = std::max(H.sched[0].list.size(), H.sched[1].list.size());
  if (nentries > 0 && tile_interp) {
    const int64_t ib = static_cast<int64_t>(nentries) * sizeof(ddi::Complex<double>);
    HIP_TRY(hipMalloc(&P.ipartial, ib), "allocate interpolation partial sums");
    bytes += ib;
  }
  const int32_t nslots = std::max(H.sched[0].nslots, H.sched[1].nslots);
  if (nslots > 0) {
    const int64_t pbytes = static_cast<int64_t>(nslots) * 64 * ddi::kTileZ * sizeof(ddi::Complex<T>);
    HIP_TRY(hipMalloc(&P.partial, pbytes), "allocate spread partial tiles");
    bytes += pbytes;
  }
  return DDI_OK;
}

// The GPE workspace (allocated on the first GPE call): all of it or none, so that a call after a
// failed allocation allocates again instead of running on missing buffers.
template <typename T>
ddi_status ensure_gpe(ddi::DevicePlan& P) {
  if (P.gpe.rho) return DDI_OK;
  const int64_t n = static_cast<int64_t>(P.H.N[0]) * P.H.N[1] * P.H.N[2];
  const int nb = ddi::gpe_reduction_blocks<T>(P);
  ddi::GpeWork& W = P.gpe;
  void** ptrs[] = {&W.rho, &W.phi, &W.phit, &W.c1, &W.c2, reinterpret_cast<void**>(&W.red)};
  const size_t bytes[] = {n * sizeof(T), n * sizeof(T), n * sizeof(T), n * sizeof(ddi::Complex<T>),
                          n * sizeof(ddi::Complex<T>), ddi::gpe_red_doubles(nb) * sizeof(double)};
  const int e = ddi::alloc_group(
      ptrs, bytes, 6, [](void** p, size_t b) { return hipMalloc(p, b); }, [](void* p) { (void)hipFree(p); });
  if (e != 0) return hip_fail(static_cast<hipError_t>(e), "allocate GPE workspace");
  W.red_blocks = nb;
  for (size_t b : bytes) P.workspace_bytes += static_cast<int64_t>(b);
  return DDI_OK;
}

ddi_status ts_step_impl(ddi_plan_t plan, const gpe_params& gp, double dt, double delta, double q, const void* in,
                        void* out, void* stream, const char* what) {
  ddi::DevicePlan& P = plan->P;
  ddi_status st = P.mixed ? ensure_gpe<float>(P) : ensure_gpe<double>(P);
  if (st != DDI_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = P.mixed ? ddi::run_ts_step<float>(P, gp, dt, delta, q, static_cast<const ddi::Complex<float>*>(in),
                                                   static_cast<ddi::Complex<float>*>(out), s)
                         : ddi::run_ts_step<double>(P, gp, dt, delta, q, static_cast<const ddi::Complex<double>*>(in),
                                                    static_cast<ddi::Complex<double>*>(out), s);
  if (e != hipSuccess) return hip_fail(e, what);
  return DDI_OK;
}

// Static workspace of gpe_energy_grad_noalloc: one copy of this array per GPU, resident from the
// module's load until the process ends.  Host code never uses the array's name as an address:
// each device's copy is located once with hipGetSymbolAddress and only that pointer is used.
constexpr size_t kScratchBytes = size_t(96) << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
void* g_scratch_ptr[kMaxDevices] = {};

// The device address of the current device's copy of `scratch` (looked up on the first call per
// device, with that device current).
ddi_status scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(DDI_ENOTSUP, "device index beyond the static workspace table");
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    if (!ptr) return fail(DDI_EDEVICE, "hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return DDI_OK;
}

// Carves the GPE workspace of an n-point grid of real type T out of a static workspace of
// kScratchBytes at base (256-byte aligned pieces); fails if it does not fit.
template <typename T>
ddi_status scratch_gpe_work(const ddi::DevicePlan& P, void* base, ddi::GpeWork& W) {
  const int64_t n = static_cast<int64_t>(P.H.N[0]) * P.H.N[1] * P.H.N[2];
  const int nb = ddi::gpe_reduction_blocks<T>(P);
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t real = up(n * sizeof(T)), cplx = up(n * sizeof(ddi::Complex<T>));
  const size_t need = 3 * real + cplx + up(ddi::gpe_red_doubles(nb) * sizeof(double));
  if (need > kScratchBytes)
    return fail(DDI_EINVAL, "gpe_energy_grad_noalloc: the grid needs " + std::to_string(need) +
                                " bytes of workspace, the static workspace holds " + std::to_string(kScratchBytes));
  unsigned char* b = static_cast<unsigned char*>(base);
  W.rho = b;
  W.phi = b + real;
  W.phit = b + 2 * real;
  W.c1 = b + 3 * real;
  W.c2 = nullptr;
  W.red = reinterpret_cast<double*>(b + 3 * real + cplx);
  W.red_blocks = nb;
  return DDI_OK;
}

ddi_status check_plan(ddi_plan_t plan) {
  if (!plan) return fail(DDI_EINVAL, "plan is NULL");
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess) return fail(DDI_EDEVICE, "hipGetDevice failed");
  if (dev != plan->P.device) return fail(DDI_EINVAL, "the current device differs from the plan's device");
  return DDI_OK;
}

}  // namespace

extern "C" {

const char* ddi_last_error(void) { return g_err.c_str(); }

ddi_status ddi_plan(const ddi_params* params, void* stream, ddi_plan_t* out) {
  g_err.clear();
  if (!out) return fail(DDI_EINVAL, "out is NULL");
  *out = nullptr;
  if (!params) return fail(DDI_EINVAL, "params is NULL");
  ddi_plan_s* plan = new (std::nothrow) ddi_plan_s();
  if (!plan) return fail(DDI_ENOMEM, "host allocation failed");
  ddi::DevicePlan& P = plan->P;
  int st = DDI_OK;
  std::string msg;
  try {
    msg = ddi::build_tables(*params, P.H, &st);
  } catch (const std::bad_alloc&) {
    delete plan;
    return fail(DDI_ENOMEM, "host allocation failed while building plan tables");
  } catch (...) {
    delete plan;
    return fail(DDI_EINTERNAL, "unexpected error while building plan tables");
  }
  if (st != DDI_OK) {
    delete plan;
    return fail(static_cast<ddi_status>(st), msg);
  }
  P.mixed = params->prec == DDI_MIXED;
  if (hipGetDevice(&P.device) != hipSuccess) {
    delete plan;
    return fail(DDI_EDEVICE, "no HIP device");
  }
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  {
    // grouped interpolation stages its region in LDS; without room for it, every node goes direct
    int max_lds = 0;
    if (hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, P.device) != hipSuccess) max_lds = 0;
    const size_t elem = P.mixed ? 2 * sizeof(float) : 2 * sizeof(double);
    const size_t need = static_cast<size_t>(P.H.ireg[0]) * P.H.ireg[1] * P.H.ireg[2] * elem;
    if (need > static_cast<size_t>(max_lds)) {
      for (ddi::Schedule& S : P.H.sched) {
        for (const ddi::InterpItem& it : S.interp_items)
          for (int32_t c = 0; c < it.count; ++c) S.interp_direct.push_back(it.start + c);
        S.interp_items.clear();
      }
    }
  }
  ddi_status ds;
  std::vector<ddi::NodeRec<double>> rd;
  std::vector<ddi::NodeRec<float>> rf;
  std::vector<std::vector<ddi::Complex<double>>> td;
  std::vector<std::vector<ddi::Complex<float>>> tf;
  std::vector<double> pd;
  std::vector<float> pf;
  try {
    ds = P.mixed ? build_device<float>(P, s, rf, tf, pf) : build_device<double>(P, s, rd, td, pd);
  } catch (const std::bad_alloc&) {
    ds = fail(DDI_ENOMEM, "host allocation failed while uploading plan tables");
  }
  if (ds == DDI_OK) {
    hipError_t e = hipStreamSynchronize(s);   // host staging buffers die at return
    if (e != hipSuccess) ds = hip_fail(e, "plan upload");
  }
  if (ds != DDI_OK) {
    (void)hipStreamSynchronize(s);
    free_plan(P);
    delete plan;
    return ds;
  }
  *out = plan;
  return DDI_OK;
}

void ddi_destroy(ddi_plan_t plan) {
  if (!plan) return;
  free_plan(plan->P);
  delete plan;
}

ddi_status ddi_plan_info(ddi_plan_t plan, ddi_plan_info_t* info) {
  if (!plan || !info) return fail(DDI_EINVAL, "plan or info is NULL");
  const ddi::HostTables& H = plan->P.H;
  info->m_eff = H.M;
  info->m_nominal = H.m_nominal;
  info->m_half = 0;
  for (double f : H.half_factor) info->m_half += f > 0.0 ? 1 : 0;
  info->apply_window = H.sched[ddi::kHalf].nz;
  for (int a = 0; a < 3; ++a) info->n_fine[a] = H.nf[a];
  info->width = H.w;
  info->es_beta = H.es_beta;
  info->kmax = H.kmax;
  info->spread_items = static_cast<int64_t>(H.sched[ddi::kHalf].items.size());
  info->spread_entries = static_cast<int64_t>(H.sched[ddi::kHalf].list.size());
  info->workspace_bytes = plan->P.workspace_bytes;
  info->split = H.split ? 1 : 0;
  info->split_s = H.split_s;
  return DDI_OK;
}

ddi_status ddi_plan_nodes(ddi_plan_t plan, int32_t* index_host, double* k_host, double* c_host) {
  if (!plan) return fail(DDI_EINVAL, "plan is NULL");
  ddi::HostTables& H = plan->P.H;
  if (H.c_stale) {
    // the axes were changed by ddi_set_dipole: the same symbol as the plan builder, new axes
    for (int64_t q = 0; q < H.M; ++q) {
      const double* k = &H.k[3 * q];
      const double kk = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
      double U;
      if (H.dim == 3) {
        const double kn = k[0] * H.nv[0] + k[1] * H.nv[1] + k[2] * H.nv[2];
        const double km = k[0] * H.mv[0] + k[1] * H.mv[1] + k[2] * H.mv[2];
        U = 3.0 * kn * km / kk - (H.nv[0] * H.mv[0] + H.nv[1] * H.mv[1] + H.nv[2] * H.mv[2]);
      } else {
        const double kn = k[0] * H.nv[0] + k[1] * H.nv[1];
        const double km = k[0] * H.mv[0] + k[1] * H.mv[1];
        U = 3.0 * (kn * km - H.nv[2] * H.mv[2] * kk) / (2.0 * std::sqrt(kk));
      }
      H.c[q] = H.base[q] * U;
    }
    H.c_stale = false;
  }
  if (index_host) std::memcpy(index_host, H.index.data(), H.index.size() * sizeof(int32_t));
  if (k_host) std::memcpy(k_host, H.k.data(), H.k.size() * sizeof(double));
  if (c_host) std::memcpy(c_host, H.c.data(), H.c.size() * sizeof(double));
  return DDI_OK;
}

ddi_status ddi_set_dipole(ddi_plan_t plan, const double* dip_n, const double* dip_m, void* stream) {
  ddi_status st = check_plan(plan);
  if (st != DDI_OK) return st;
  if (!dip_n) return fail(DDI_EINVAL, "dip_n is NULL");
  double n[3], m[3];
  double nn = 0.0, mm = 0.0;
  for (int i = 0; i < 3; ++i) {
    n[i] = dip_n[i];
    m[i] = dip_m ? dip_m[i] : 0.0;
    nn += n[i] * n[i];
    mm += m[i] * m[i];
  }
  if (!(nn > 0.0) || !std::isfinite(nn)) return fail(DDI_EINVAL, "dipole axis n must be a non-zero finite vector");
  if (!std::isfinite(mm)) return fail(DDI_EINVAL, "dipole axis m must be finite");
  if (!(mm > 0.0)) for (int i = 0; i < 3; ++i) m[i] = n[i];
  ddi::DevicePlan& P = plan->P;
  const ddi::HostTables& H = P.H;
  if (!P.kq) {
    // first call: the node coordinates and the weights without the symbol (synchronous upload)
    std::vector<double> bs(H.M), bh(H.M);
    for (int64_t q = 0; q < H.M; ++q) {
      bs[q] = H.base[q] * H.cell;
      bh[q] = H.half_factor[q] * H.base[q] * H.cell;
    }
    double* d[3] = {nullptr, nullptr, nullptr};
    const void* src[3] = {H.k.data(), bs.data(), bh.data()};
    const size_t cnt[3] = {H.k.size(), bs.size(), bh.size()};
    for (int i = 0; i < 3; ++i) {
      hipError_t e = hipMalloc(reinterpret_cast<void**>(&d[i]), cnt[i] * sizeof(double));
      if (e == hipSuccess) e = hipMemcpy(d[i], src[i], cnt[i] * sizeof(double), hipMemcpyHostToDevice);
      if (e != hipSuccess) {
        for (double* x : d)
          if (x) (void)hipFree(x);
        return hip_fail(e, "ddi_set_dipole tables");
      }
    }
    P.kq = d[0];
    P.base_scaled = d[1];
    P.base_half = d[2];
    P.workspace_bytes += static_cast<int64_t>((cnt[0] + cnt[1] + cnt[2]) * sizeof(double));
  }
  hipError_t e = ddi::run_set_dipole(P, n, m, reinterpret_cast<hipStream_t>(stream));
  if (e != hipSuccess) return hip_fail(e, "ddi_set_dipole launch");
  for (int i = 0; i < 3; ++i) {
    P.H.nv[i] = n[i];
    P.H.mv[i] = m[i];
  }
  P.H.c_stale = true;
  return DDI_OK;
}

ddi_status ddi_apply(ddi_plan_t plan, const void* rho_dev, void* phi_dev, void* stream) {
  ddi_status st = check_plan(plan);
  if (st != DDI_OK) return st;
  if (!rho_dev || !phi_dev) return fail(DDI_EINVAL, "NULL buffer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ddi::DevicePlan& P = plan->P;
  hipError_t e = P.mixed ? ddi::run_ddi<float>(P, static_cast<const float*>(rho_dev), static_cast<float*>(phi_dev), +1, s, nullptr)
                         : ddi::run_ddi<double>(P, static_cast<const double*>(rho_dev), static_cast<double*>(phi_dev), +1, s, nullptr);
  if (e != hipSuccess) return hip_fail(e, "ddi_apply launch");
  return DDI_OK;
}

ddi_status ddi_apply_adjoint(ddi_plan_t plan, const void* phibar_dev, void* rhobar_dev, void* stream) {
  ddi_status st = check_plan(plan);
  if (st != DDI_OK) return st;
  if (!phibar_dev || !rhobar_dev) return fail(DDI_EINVAL, "NULL buffer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ddi::DevicePlan& P = plan->P;
  hipError_t e = P.mixed ? ddi::run_ddi<float>(P, static_cast<const float*>(phibar_dev), static_cast<float*>(rhobar_dev), -1, s, nullptr)
                         : ddi::run_ddi<double>(P, static_cast<const double*>(phibar_dev), static_cast<double*>(rhobar_dev), -1, s, nullptr);
  if (e != hipSuccess) return hip_fail(e, "ddi_apply_adjoint launch");
  return DDI_OK;
}

ddi_status ddi_profile_apply(ddi_plan_t plan, const void* in_dev, void* out_dev, int32_t sign, int32_t reps,
                             double* stage_ms, void* stream) {
  ddi_status st = check_plan(plan);
  if (st != DDI_OK) return st;
  if (!in_dev || !out_dev || !stage_ms) return fail(DDI_EINVAL, "NULL argument");
  if (sign != 1 && sign != -1) return fail(DDI_EINVAL, "sign must be +1 or -1");
  if (reps < 1 || reps > 100000) return fail(DDI_EINVAL, "reps must lie in [1, 100000]");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ddi::DevicePlan& P = plan->P;
  hipEvent_t ev[ddi::kStages + 1];
  for (int i = 0; i <= ddi::kStages; ++i) {
    hipError_t e = hipEventCreate(&ev[i]);
    if (e != hipSuccess) {
      for (int j = 0; j < i; ++j) (void)hipEventDestroy(ev[j]);
      return hip_fail(e, "hipEventCreate");
    }
  }
  for (int i = 0; i < ddi::kStages; ++i) stage_ms[i] = 0.0;
  ddi_status result = DDI_OK;
  for (int r = 0; r < reps && result == DDI_OK; ++r) {
    hipError_t e = P.mixed ? ddi::run_ddi<float>(P, static_cast<const float*>(in_dev), static_cast<float*>(out_dev), sign, s, ev)
                           : ddi::run_ddi<double>(P, static_cast<const double*>(in_dev), static_cast<double*>(out_dev), sign, s, ev);
    if (e == hipSuccess) e = hipEventSynchronize(ev[ddi::kStages]);
    if (e != hipSuccess) { result = hip_fail(e, "ddi_profile_apply"); break; }
    for (int i = 0; i < ddi::kStages; ++i) {
      float ms = 0.0f;
      e = hipEventElapsedTime(&ms, ev[i], ev[i + 1]);
      if (e != hipSuccess) { result = hip_fail(e, "hipEventElapsedTime"); break; }
      stage_ms[i] += ms;
    }
  }
  for (int i = 0; i <= ddi::kStages; ++i) (void)hipEventDestroy(ev[i]);
  if (result == DDI_OK)
    for (int i = 0; i < ddi::kStages; ++i) stage_ms[i] /= reps;
  return result;
}

ddi_status ddi_type2(ddi_plan_t plan, const void* rho_dev, void* rhohat_dev, void* stream) {
  ddi_status st = check_plan(plan);
  if (st != DDI_OK) return st;
  if (!rho_dev || !rhohat_dev) return fail(DDI_EINVAL, "NULL buffer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ddi::DevicePlan& P = plan->P;
  hipError_t e;
  if (P.mixed)
    e = ddi::run_type2<float>(P, ddi::kAll, static_cast<const float*>(rho_dev), static_cast<ddi::Complex<float>*>(rhohat_dev),
                              nullptr, P.H.cell, -1, s, nullptr);
  else
    e = ddi::run_type2<double>(P, ddi::kAll, static_cast<const double*>(rho_dev), static_cast<ddi::Complex<double>*>(rhohat_dev),
                               nullptr, P.H.cell, -1, s, nullptr);
  if (e != hipSuccess) return hip_fail(e, "ddi_type2 launch");
  return DDI_OK;
}

ddi_status ddi_type1(ddi_plan_t plan, const void* g_dev, void* phi_dev, void* stream) {
  ddi_status st = check_plan(plan);
  if (st != DDI_OK) return st;
  if (!g_dev || !phi_dev) return fail(DDI_EINVAL, "NULL buffer");
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  ddi::DevicePlan& P = plan->P;
  hipError_t e = P.mixed ? ddi::run_type1<float>(P, ddi::kAll, static_cast<const ddi::Complex<float>*>(g_dev), static_cast<float*>(phi_dev), +1, s, nullptr)
                         : ddi::run_type1<double>(P, ddi::kAll, static_cast<const ddi::Complex<double>*>(g_dev), static_cast<double*>(phi_dev), +1, s, nullptr);
  if (e != hipSuccess) return hip_fail(e, "ddi_type1 launch");
  return DDI_OK;
}

ddi_status gpe_energy_grad(ddi_plan_t plan, const gpe_params* gp, const void* psi_dev, double E_out[5],
                           void* grad_dev, void* stream) {
  ddi_status st = check_plan(plan);
  if (st != DDI_OK) return st;
  if (!gp || !psi_dev || !E_out) return fail(DDI_EINVAL, "NULL argument");
  if (!std::isfinite(gp->beta) || !std::isfinite(gp->lambda)) return fail(DDI_EINVAL, "beta and lambda must be finite");
  ddi::DevicePlan& P = plan->P;
  st = P.mixed ? ensure_gpe<float>(P) : ensure_gpe<double>(P);
  if (st != DDI_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double* E_dev = P.gpe.red + 8 * P.gpe.red_blocks + 8;
  hipError_t e = P.mixed ? ddi::run_gpe_energy_grad<float>(P, P.gpe, *gp, static_cast<const ddi::Complex<float>*>(psi_dev), E_dev,
                                                           static_cast<ddi::Complex<float>*>(grad_dev), s)
                         : ddi::run_gpe_energy_grad<double>(P, P.gpe, *gp, static_cast<const ddi::Complex<double>*>(psi_dev), E_dev,
                                                            static_cast<ddi::Complex<double>*>(grad_dev), s);
  if (e != hipSuccess) return hip_fail(e, "gpe_energy_grad launch");
  HIP_TRY(hipMemcpyAsync(E_out, E_dev, 5 * sizeof(double), hipMemcpyDeviceToHost, s), "copy energies");
  HIP_TRY(hipStreamSynchronize(s), "gpe_energy_grad");
  return DDI_OK;
}

ddi_status gpe_energy_grad_noalloc(ddi_plan_t plan, const gpe_params* gp, const void* psi_dev, double* E_dev,
                                   void* grad_dev, void* stream) {
  ddi_status st = check_plan(plan);
  if (st != DDI_OK) return st;
  if (!gp || !psi_dev || !E_dev) return fail(DDI_EINVAL, "NULL argument");
  if (!std::isfinite(gp->beta) || !std::isfinite(gp->lambda)) return fail(DDI_EINVAL, "beta and lambda must be finite");
  ddi::DevicePlan& P = plan->P;
  void* base = nullptr;
  st = scratch_address(P.device, &base);
  if (st != DDI_OK) return st;
  ddi::GpeWork W;
  st = P.mixed ? scratch_gpe_work<float>(P, base, W) : scratch_gpe_work<double>(P, base, W);
  if (st != DDI_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = P.mixed ? ddi::run_gpe_energy_grad<float>(P, W, *gp, static_cast<const ddi::Complex<float>*>(psi_dev), E_dev,
                                                           static_cast<ddi::Complex<float>*>(grad_dev), s)
                         : ddi::run_gpe_energy_grad<double>(P, W, *gp, static_cast<const ddi::Complex<double>*>(psi_dev), E_dev,
                                                            static_cast<ddi::Complex<double>*>(grad_dev), s);
  if (e != hipSuccess) return hip_fail(e, "gpe_energy_grad_noalloc launch");
  return DDI_OK;
}

ddi_status gpe_gf_step(ddi_plan_t plan, const gpe_params* gp, double dt, int32_t n_inner, const void* psi_in_dev,
                       void* psi_out_dev, double* residual_dev, void* stream) {
  ddi_status st = check_plan(plan);
  if (st != DDI_OK) return st;
  if (!gp || !psi_in_dev || !psi_out_dev) return fail(DDI_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DDI_EINVAL, "dt must be positive");
  if (n_inner < 0 || n_inner > 10000) return fail(DDI_EINVAL, "n_inner must lie in [0, 10000]");
  ddi::DevicePlan& P = plan->P;
  st = P.mixed ? ensure_gpe<float>(P) : ensure_gpe<double>(P);
  if (st != DDI_OK) return st;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  hipError_t e = P.mixed ? ddi::run_gf_step<float>(P, *gp, dt, n_inner, static_cast<const ddi::Complex<float>*>(psi_in_dev),
                                                   static_cast<ddi::Complex<float>*>(psi_out_dev), residual_dev, s)
                         : ddi::run_gf_step<double>(P, *gp, dt, n_inner, static_cast<const ddi::Complex<double>*>(psi_in_dev),
                                                    static_cast<ddi::Complex<double>*>(psi_out_dev), residual_dev, s);
  if (e != hipSuccess) return hip_fail(e, "gpe_gf_step launch");
  return DDI_OK;
}

ddi_status gpe_ts_step(ddi_plan_t plan, const gpe_params* gp, double dt, double delta, const void* psi_in_dev,
                       void* psi_out_dev, void* stream) {
  ddi_status st = check_plan(plan);
  if (st != DDI_OK) return st;
  if (!gp || !psi_in_dev || !psi_out_dev) return fail(DDI_EINVAL, "NULL argument");
  if (dt == 0.0 || !std::isfinite(dt)) return fail(DDI_EINVAL, "dt must be finite and non-zero");
  if (!(delta >= 0.0) || !std::isfinite(delta)) return fail(DDI_EINVAL, "delta must be finite and >= 0");
  return ts_step_impl(plan, *gp, dt, delta, 0.0, psi_in_dev, psi_out_dev, stream, "gpe_ts_step launch");
}

ddi_status gpe_ts_step_loss(ddi_plan_t plan, const gpe_params* gp, double dt, double delta, double q,
                            const void* psi_in_dev, void* psi_out_dev, void* stream) {
  ddi_status st = check_plan(plan);
  if (st != DDI_OK) return st;
  if (!gp || !psi_in_dev || !psi_out_dev) return fail(DDI_EINVAL, "NULL argument");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(DDI_EINVAL, "dt must be finite and positive");
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(DDI_EINVAL, "delta must be finite and > 0");
  if (!(q > 0.0) || !std::isfinite(q)) return fail(DDI_EINVAL, "q must be finite and > 0");
  return ts_step_impl(plan, *gp, dt, delta, q, psi_in_dev, psi_out_dev, stream, "gpe_ts_step_loss launch");
}

}  // extern "C"
