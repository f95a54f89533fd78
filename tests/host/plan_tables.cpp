// Host-only driver of the plan builder, for the CPU tests: reads one ddi_params struct (its raw
// bytes, written by the Python binding's ctypes structure) from a file, runs ddi::build_tables,
// and writes the status, the message and every host table and schedule as named arrays:
//   per array: u32 name length, name, u8 type ('i' int32, 'd' float64), i64 count, data.
// It touches no device: the tables are what a plan uploads.
#include <cstdio>
#include <string>
#include <vector>

#include "../../paper_1504_02897_amd/csrc/ddi_internal.h"

namespace {

FILE* out = nullptr;

void put(const std::string& name, char type, const void* data, int64_t count) {
  const uint32_t n = static_cast<uint32_t>(name.size());
  std::fwrite(&n, sizeof n, 1, out);
  std::fwrite(name.data(), 1, n, out);
  std::fwrite(&type, 1, 1, out);
  std::fwrite(&count, sizeof count, 1, out);
  const size_t elem = type == 'i' ? sizeof(int32_t) : sizeof(double);
  if (count > 0) std::fwrite(data, elem, static_cast<size_t>(count), out);
}
void put_i(const std::string& name, const std::vector<int32_t>& v) { put(name, 'i', v.data(), static_cast<int64_t>(v.size())); }
void put_d(const std::string& name, const std::vector<double>& v) { put(name, 'd', v.data(), static_cast<int64_t>(v.size())); }
void put_i(const std::string& name, const int* v, int n) { put_i(name, std::vector<int32_t>(v, v + n)); }
void put_d(const std::string& name, const double* v, int n) { put_d(name, std::vector<double>(v, v + n)); }

}  // namespace

int main(int argc, char** argv) {
  if (argc != 3) {
    std::fprintf(stderr, "usage: %s params.bin tables.bin\n", argv[0]);
    return 2;
  }
  ddi_params p{};
  FILE* in = std::fopen(argv[1], "rb");
  if (!in) return 2;
  const size_t got = std::fread(&p, 1, sizeof p, in);
  const bool extra = std::fgetc(in) != EOF;
  std::fclose(in);
  if (got != sizeof p || extra) {
    std::fprintf(stderr, "params file holds %zu bytes, ddi_params is %zu\n", got, sizeof p);
    return 3;
  }
  ddi::HostTables t;
  int status = DDI_EINTERNAL;
  const std::string err = ddi::build_tables(p, t, &status);
  out = std::fopen(argv[2], "wb");
  if (!out) return 2;
  put_i("status", &status, 1);
  if (!err.empty()) {
    std::vector<int32_t> chars(err.begin(), err.end());
    put_i("message_chars", chars);
  }
  if (err.empty()) {
    const int sc[] = {t.dim, t.w, t.zalign, t.row_windows ? 1 : 0, ddi::kWMax, t.split ? 1 : 0};
    put_i("dim_w_zalign_rows_wmax_split", sc, 6);
    put_i("N", t.N, 3);
    put_i("nf", t.nf, 3);
    put_i("W", t.W, 3);
    put_i("tile", t.tile, 3);
    put_i("ntiles", t.ntiles, 3);
    put_i("ib", t.ib, 3);
    put_d("h", t.h, 3);
    put_d("L", t.L, 3);
    const double sd[] = {t.cell, t.es_beta, t.kmax, static_cast<double>(t.m_nominal), t.split_s};
    put_d("cell_beta_kmax_mnom_splits", sd, 5);
    put_i("index", t.index);
    put_d("k", t.k);
    put_d("c", t.c);
    put_d("base", t.base);
    put_d("half_factor", t.half_factor);
    put_i("l0", t.l0);
    put_d("wts", t.wts);
    for (int a = 0; a < 3; ++a) put_d("deconv" + std::to_string(a), t.deconv[a]);
    for (int s = 0; s < 2; ++s) {
      const ddi::Schedule& S = t.sched[s];
      const std::string pre = "s" + std::to_string(s) + "_";
      std::vector<int32_t> v;
      for (const ddi::InterpItem& it : S.interp_items) v.insert(v.end(), {it.start, it.count, it.org[0], it.org[1], it.org[2]});
      put_i(pre + "interp_items", v);
      put_i(pre + "interp_direct", S.interp_direct);
      put_i(pre + "list", S.list);
      v.clear();
      for (const ddi::SpreadItem& it : S.items) v.insert(v.end(), {it.tile, it.start, it.count, it.slot});
      put_i(pre + "items", v);
      v.clear();
      for (const ddi::ReduceItem& it : S.reduces) v.insert(v.end(), {it.tile, it.first_slot, it.nslots});
      put_i(pre + "reduces", v);
      put_i(pre + "gptr", S.gptr);
      put_i(pre + "gpos", S.gpos);
      put_i(pre + "ent", S.ent);
      const int win[] = {S.nslots, S.z0, S.nz, S.ny};
      put_i(pre + "nslots_z0_nz_ny", win, 4);
    }
  }
  for (int n : {4, 64, 256, 1024, 12, 96, 192, 768}) put_d("twiddle" + std::to_string(n), ddi::twiddle_table(n));
  std::fclose(out);
  return 0;
}
