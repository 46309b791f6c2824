// C ABI of libpyjac_mi355x: mechanism handles, argument checking, variant
// selection and kernel launches.  Declarations and contracts: include/pyjac.h.
#include <hip/hip_runtime.h>

#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pyjac.h"
#include "tables.hpp"
#include "chemkin.hpp"

namespace pyjac {

size_t tile_lds_bytes(int N, int NR, int NG, int TS, int NT, bool jac);
size_t conc_lds_bytes(int N, int NR, int NG, int TS, int NT);
hipError_t launch_tile_multi(int TS, int NT, int kpt, bool split, const WorkList& wl, int64_t tiles, size_t lds,
                             hipStream_t st);
hipError_t launch_cs_jacobian(const MechDev& md, int64_t n, int64_t ld, const double* phi, const double* p,
                              double step, double* jac, hipStream_t st);
hipError_t launch_mix_pairs(const MechDev& md, int64_t n, int64_t ld, const double* phi, const int* partner, double w,
                            double* out, hipStream_t st);
hipError_t launch_conc(int TS, int NT, const MechDev& md, int64_t n, int64_t ld, const double* phi, double* out,
                       size_t lds, hipStream_t st);
hipError_t launch_tile(bool jac_mode, int TS, int NT, const MechDev& md, int64_t n, int64_t ld,
                       const double* phi, const double* p, double* rop_f, double* rop_r, double* pmod,
                       double* wdot, double* dphi, double* jac, size_t lds, hipStream_t st);

thread_local std::string g_last_error;

pyjac_status fail(pyjac_status code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

struct Variant { int ts = 0, nt = 0; };

size_t fd_bytes_per_state(int N);
hipError_t fd_perturb(int N, int64_t m, int64_t ld, const double* phi, const double* p, int64_t s0, double* phi2,
                      double* p2, int64_t ld2, double* inc, hipStream_t st);
hipError_t fd_diff(int N, int64_t m, const double* f2, int64_t ld2, const double* inc, int64_t s0, double* jac,
                   int64_t ld, hipStream_t st);

}  // namespace pyjac

struct pyjac_mech {
  pyjac::PackedMech host;
  pyjac::MechDev dev{};
  void* dmem = nullptr;
  int device = 0;
  size_t max_lds = 65536;
  pyjac::Variant jac_var, rates_var, conc_var;
  // per launch shape: species-list chunk bounds, built when the shape is chosen
  struct VarDev {
    int ts = 0, nt = 0;
    bool jac = false;
    void* mem = nullptr;
    const int* chunk = nullptr;
  };
  std::vector<VarDev> vars;
};

namespace pyjac {
namespace {

template <class T>
void append(std::vector<char>& blob, const std::vector<T>& v, std::vector<size_t>& offs) {
  size_t off = (blob.size() + 255) & ~size_t(255);
  blob.resize(off + v.size() * sizeof(T));
  std::memcpy(blob.data() + off, v.data(), v.size() * sizeof(T));
  offs.push_back(off);
}

int kpt_of(int N, int ts, int nt) { int g = nt / ts; return (N + g - 1) / g; }

// Candidate launch shapes, most preferred first; the first that fits the
// device's LDS and keeps <= 8 species per thread is used.
Variant pick(const PackedMech& P, bool jac, size_t max_lds) {
  static const int jac_c[][2] = {{16, 1024}, {8, 1024}, {8, 512}, {4, 1024}, {4, 512}, {2, 1024}, {2, 512}};
  static const int rate_c[][2] = {{64, 1024}, {32, 1024}, {16, 1024}, {16, 512}, {8, 1024}, {8, 512},
                                  {4, 1024}, {2, 1024}};   // all compiled shapes
  const auto* list = jac ? jac_c : rate_c;
  int cnt = jac ? 7 : 8;
  for (int c = 0; c < cnt; ++c) {
    int ts = list[c][0], nt = list[c][1];
    if (kpt_of(P.N, ts, nt) > 8) continue;
    if (tile_lds_bytes(P.N, P.NR, P.NG, ts, nt, jac) <= max_lds) return {ts, nt};
  }
  return {0, 0};
}

// Shapes compiled for the concentration-form Jacobian, most preferred first.
const int kConcShapes[][2] = {{16, 1024}, {8, 1024}, {8, 512}, {4, 1024}, {4, 512}, {2, 512}, {8, 256}, {4, 256}};

bool conc_fits(const PackedMech& P, Variant v, size_t max_lds) {
  return kpt_of(P.N, v.ts, v.nt) <= 8 && conc_lds_bytes(P.N, P.NR, P.NG, v.ts, v.nt) <= max_lds;
}

Variant pick_conc(const PackedMech& P, size_t max_lds) {
  for (auto& q : kConcShapes)
    if (conc_fits(P, Variant{q[0], q[1]}, max_lds)) return {q[0], q[1]};
  return {0, 0};
}

size_t kind_lds(const pyjac_mech* m, int which, Variant v) {
  const PackedMech& P = m->host;
  return which == 2 ? conc_lds_bytes(P.N, P.NR, P.NG, v.ts, v.nt)
                    : tile_lds_bytes(P.N, P.NR, P.NG, v.ts, v.nt, which == 1);
}

pyjac_status upload(pyjac_mech* m) {
  PackedMech& P = m->host;
  std::vector<char> blob;
  std::vector<size_t> o;
  append(blob, P.W, o); append(blob, P.invW, o); append(blob, P.nasa, o); append(blob, P.tmid, o);
  append(blob, P.vcol.empty() ? std::vector<double>{0.0} : P.vcol, o);
  append(blob, P.rx, o);
  append(blob, P.eff_sp, o); append(blob, P.eff_am1, o); append(blob, P.plog, o); append(blob, P.cheb, o);
  append(blob, P.spg_ent, o);
  append(blob, P.col_start, o); append(blob, P.colrec, o); append(blob, P.col_order, o);
  append(blob, P.col_flags, o);
  append(blob, P.col_item, o); append(blob, P.col_join, o);
  append(blob, P.cv_col_start, o); append(blob, P.cv_colrec, o); append(blob, P.cv_col_order, o);
  append(blob, P.cv_colptr, o);
  if (hipMalloc(&m->dmem, blob.size()) != hipSuccess) return fail(PYJAC_E_NOMEM, "hipMalloc of mechanism tables failed");
  if (hipMemcpy(m->dmem, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess)
    return fail(PYJAC_E_DEVICE, "copy of mechanism tables failed");
  char* b = static_cast<char*>(m->dmem);
  size_t q = 0;
  auto D = [&](auto ptr_type) { return reinterpret_cast<decltype(ptr_type)>(b + o[q++]); };
  MechDev& d = m->dev;
  d.N = P.N; d.NR = P.NR; d.NG = P.NG; d.col_split = P.col_split;
  d.W = D((const double*)0); d.invW = D((const double*)0); d.nasa = D((const double*)0);
  d.tmid = D((const double*)0); d.vcol = D((const double*)0);
  d.rx = D((const RxnRec*)0);
  d.eff_sp = D((const int*)0); d.eff_am1 = D((const double*)0); d.plog = D((const double*)0);
  d.cheb = D((const double*)0);
  d.spg_ent = D((const int*)0);
  d.col_start = D((const int*)0); d.colrec = D((const ColRec*)0); d.col_order = D((const int*)0);
  d.col_flags = D((const uint32_t*)0);
  d.col_item = D((const ColItem*)0); d.col_join = D((const ColJoin*)0);
  d.n_col_item = (int)P.col_item.size(); d.n_col_join = (int)P.col_join.size();
  d.cv_col_start = D((const int*)0); d.cv_colrec = D((const ColRec*)0); d.cv_col_order = D((const int*)0);
  d.cv_colptr = D((const int*)0);
  d.spg_chunk = nullptr;
  return PYJAC_OK;
}

// Device data of one launch shape (built once per shape and kernel family).
pyjac_status ensure_var(pyjac_mech* m, Variant v, bool jac) {
  for (auto& e : m->vars) if (e.ts == v.ts && e.nt == v.nt && e.jac == jac) return PYJAC_OK;
  pyjac_mech::VarDev vd;
  vd.ts = v.ts; vd.nt = v.nt; vd.jac = jac;
  std::vector<char> blob;
  std::vector<size_t> o;
  append(blob, species_chunk_bounds(m->host, v.nt / v.ts), o);
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(m->device);
  hipError_t e1 = hipMalloc(&vd.mem, blob.size());
  hipError_t e2 = e1 == hipSuccess ? hipMemcpy(vd.mem, blob.data(), blob.size(), hipMemcpyHostToDevice) : e1;
  hipSetDevice(prev);
  if (e1 != hipSuccess) return fail(PYJAC_E_NOMEM, "hipMalloc of launch tables failed");
  if (e2 != hipSuccess) { hipFree(vd.mem); return fail(PYJAC_E_DEVICE, "copy of launch tables failed"); }
  char* b = static_cast<char*>(vd.mem);
  vd.chunk = reinterpret_cast<const int*>(b + o[0]);
  m->vars.push_back(vd);
  return PYJAC_OK;
}

MechDev launch_view(const pyjac_mech* m, Variant v, bool jac) {
  MechDev md = m->dev;
  for (auto& e : m->vars)
    if (e.ts == v.ts && e.nt == v.nt && e.jac == jac) md.spg_chunk = e.chunk;
  return md;
}

bool misaligned(const void* p) { return p && (reinterpret_cast<uintptr_t>(p) & 7u); }

pyjac_status check_common(const pyjac_mech* m, int64_t n, int64_t ld, const double* phi, const double* p) {
  if (!m) return fail(PYJAC_E_INVALID, "mechanism handle is NULL");
  if (n < 0) return fail(PYJAC_E_INVALID, "n_states is negative");
  if (ld < n) return fail(PYJAC_E_INVALID, "ld is smaller than n_states");
  if (n > 0 && (!phi || !p)) return fail(PYJAC_E_INVALID, "phi and p are required");
  if (misaligned(phi) || misaligned(p)) return fail(PYJAC_E_INVALID, "input pointer not 8-byte aligned");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(PYJAC_E_DEVICE, "hipGetDevice failed");
  if (cur != m->device) return fail(PYJAC_E_INVALID, "current HIP device differs from the mechanism's device");
  if (ld > (int64_t)1 << 40) return fail(PYJAC_E_INVALID, "ld too large");
  return PYJAC_OK;
}

}  // namespace
}  // namespace pyjac

using namespace pyjac;

extern "C" {

pyjac_status pyjac_mech_load_string(const char* text, int32_t hip_device, pyjac_mech** out) {
  if (!out) return fail(PYJAC_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!text) return fail(PYJAC_E_INVALID, "text is NULL");
  auto* m = new pyjac_mech();
  std::string msg;
  int rc = build_tables(text, m->host, msg);
  if (rc != PYJAC_OK) { delete m; return fail(rc, msg); }
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || hip_device < 0 || hip_device >= ndev) {
    delete m;
    return fail(PYJAC_E_DEVICE, "no such HIP device");
  }
  m->device = hip_device;
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(hip_device);
  int lds = 0;
  if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, hip_device) == hipSuccess && lds > 0)
    m->max_lds = (size_t)lds;
  rc = upload(m);
  hipSetDevice(prev);
  if (rc != PYJAC_OK) {
    if (m->dmem) hipFree(m->dmem);
    delete m;
    return rc;
  }
  m->jac_var = pick(m->host, true, m->max_lds);
  m->rates_var = pick(m->host, false, m->max_lds);
  if (!m->jac_var.ts || !m->rates_var.ts) {
    hipFree(m->dmem);
    delete m;
    return fail(PYJAC_E_UNSUPPORTED, "mechanism too large for the per-tile LDS budget");
  }
  m->conc_var = pick_conc(m->host, m->max_lds);   // {0, 0}: the concentration form does not fit
  rc = ensure_var(m, m->jac_var, true);
  if (rc == PYJAC_OK) rc = ensure_var(m, m->rates_var, false);
  if (rc == PYJAC_OK && m->conc_var.ts) rc = ensure_var(m, m->conc_var, true);
  if (rc != PYJAC_OK) {
    pyjac_mech_free(m);
    return rc;
  }
  *out = m;
  return PYJAC_OK;
}

pyjac_status pyjac_mech_load(const char* path, int32_t hip_device, pyjac_mech** out) {
  if (!out) return fail(PYJAC_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!path) return fail(PYJAC_E_INVALID, "path is NULL");
  std::ifstream f(path, std::ios::binary);
  if (!f) return fail(PYJAC_E_IO, std::string("cannot read ") + path);
  std::stringstream ss;
  ss << f.rdbuf();
  return pyjac_mech_load_string(ss.str().c_str(), hip_device, out);
}

pyjac_status pyjac_chemkin_to_text(const char* mech_text, const char* thermo_text, char* out, size_t out_capacity,
                                   size_t* out_len) {
  if (!mech_text) return fail(PYJAC_E_INVALID, "mech_text is NULL");
  if (!out_len) return fail(PYJAC_E_INVALID, "out_len is NULL");
  std::string th = thermo_text ? thermo_text : "", tokens, msg;
  const int rc = chemkin_to_tokens(mech_text, thermo_text ? &th : nullptr, tokens, msg);
  if (rc != PYJAC_OK) return fail(rc, msg);
  *out_len = tokens.size() + 1;
  if (!out) return PYJAC_OK;
  if (out_capacity < tokens.size() + 1) return fail(PYJAC_E_INVALID, "output buffer too small");
  std::memcpy(out, tokens.c_str(), tokens.size() + 1);
  return PYJAC_OK;
}

pyjac_status pyjac_mech_load_chemkin(const char* mech_path, const char* thermo_path, int32_t hip_device,
                                     pyjac_mech** out) {
  if (!out) return fail(PYJAC_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!mech_path) return fail(PYJAC_E_INVALID, "mech_path is NULL");
  auto slurp = [](const char* path, std::string& s) {
    std::ifstream f(path, std::ios::binary);
    if (!f) return false;
    std::stringstream ss;
    ss << f.rdbuf();
    s = ss.str();
    return true;
  };
  std::string mech, thermo, tokens, msg;
  if (!slurp(mech_path, mech)) return fail(PYJAC_E_IO, std::string("cannot read ") + mech_path);
  if (thermo_path && !slurp(thermo_path, thermo)) return fail(PYJAC_E_IO, std::string("cannot read ") + thermo_path);
  const int rc = chemkin_to_tokens(mech, thermo_path ? &thermo : nullptr, tokens, msg);
  if (rc != PYJAC_OK) return fail(rc, msg);
  return pyjac_mech_load_string(tokens.c_str(), hip_device, out);
}

pyjac_status pyjac_mech_info(const pyjac_mech* m, int32_t* ns, int32_t* nr, uint64_t* hash) {
  if (!m) return fail(PYJAC_E_INVALID, "mechanism handle is NULL");
  if (ns) *ns = m->host.N;
  if (nr) *nr = m->host.NR;
  if (hash) *hash = m->host.hash;
  return PYJAC_OK;
}

pyjac_status pyjac_mech_free(pyjac_mech* m) {
  if (!m) return PYJAC_OK;
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(m->device);
  hipDeviceSynchronize();
  if (m->dmem) hipFree(m->dmem);
  for (auto& e : m->vars) hipFree(e.mem);
  hipSetDevice(prev);
  delete m;
  return PYJAC_OK;
}

pyjac_status pyjac_eval_rates(const pyjac_mech* m, int64_t n, int64_t ld, const double* phi, const double* p,
                              double* rop_f, double* rop_r, double* pres_mod, double* wdot, double* dphi,
                              void* stream) {
  pyjac_status rc = check_common(m, n, ld, phi, p);
  if (rc != PYJAC_OK) return rc;
  for (const double* q : {rop_f, rop_r, pres_mod, wdot, dphi})
    if (misaligned(q)) return fail(PYJAC_E_INVALID, "output pointer not 8-byte aligned");
  if (n == 0) return PYJAC_OK;
  const Variant v = m->rates_var;
  size_t lds = tile_lds_bytes(m->host.N, m->host.NR, m->host.NG, v.ts, v.nt, false);
  const MechDev md = launch_view(m, v, false);
  hipError_t e = launch_tile(false, v.ts, v.nt, md, n, ld, phi, p, rop_f, rop_r, pres_mod, wdot, dphi,
                             nullptr, lds, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(PYJAC_E_DEVICE, std::string("rates launch failed: ") + hipGetErrorString(e));
  return PYJAC_OK;
}

pyjac_status pyjac_eval_jacobian(const pyjac_mech* m, int64_t n, int64_t ld, const double* phi, const double* p,
                                 double* jac, void* stream) {
  pyjac_status rc = check_common(m, n, ld, phi, p);
  if (rc != PYJAC_OK) return rc;
  if (n > 0 && !jac) return fail(PYJAC_E_INVALID, "jac is NULL");
  if (misaligned(jac)) return fail(PYJAC_E_INVALID, "jac not 8-byte aligned");
  if (n == 0) return PYJAC_OK;
  const Variant v = m->jac_var;
  size_t lds = tile_lds_bytes(m->host.N, m->host.NR, m->host.NG, v.ts, v.nt, true);
  const MechDev md = launch_view(m, v, true);
  hipError_t e = launch_tile(true, v.ts, v.nt, md, n, ld, phi, p, nullptr, nullptr, nullptr, nullptr,
                             nullptr, jac, lds, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(PYJAC_E_DEVICE, std::string("jacobian launch failed: ") + hipGetErrorString(e));
  return PYJAC_OK;
}

pyjac_status pyjac_eval_jacobian_multi(int32_t n_items, const pyjac_work_item* items, void* stream) {
  if (n_items < 0 || (n_items > 0 && !items)) return fail(PYJAC_E_INVALID, "bad item list");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess) return fail(PYJAC_E_DEVICE, "hipGetDevice failed");
  // validate every item first, so that nothing is enqueued on an error
  Variant v{0, 0};
  int split = -1;
  for (int32_t i = 0; i < n_items; ++i) {
    const pyjac_work_item& it = items[i];
    pyjac_status rc = check_common(it.mech, it.n_states, it.ld, it.phi, it.p);
    if (rc != PYJAC_OK) return rc;
    if (it.n_states > 0 && !it.jac) return fail(PYJAC_E_INVALID, "jac is NULL");
    if (misaligned(it.jac)) return fail(PYJAC_E_INVALID, "jac not 8-byte aligned");
    if (it.n_states == 0) continue;
    const Variant w = it.mech->jac_var;
    if (!v.ts) { v = w; split = it.mech->host.col_split; }
    if (w.ts != v.ts || w.nt != v.nt || it.mech->host.col_split != split)
      return fail(PYJAC_E_UNSUPPORTED, "items of one launch need the same Jacobian launch shape and stream form");
  }
  if (!v.ts) return PYJAC_OK;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  for (int32_t i0 = 0; i0 < n_items;) {
    WorkList wl{};
    int64_t tiles = 0;
    size_t lds = 0;
    int kpt = 1;
    int c = 0;
    for (; i0 < n_items && c < kMaxWorkItems; ++i0) {
      const pyjac_work_item& it = items[i0];
      if (it.n_states == 0) continue;
      const PackedMech& P = it.mech->host;
      WorkItem& w = wl.item[c++];
      w.md = launch_view(it.mech, v, true);
      w.phi = it.phi;
      w.p = it.p;
      w.jac = it.jac;
      w.n = it.n_states;
      w.ld = it.ld;
      w.tile0 = tiles;
      tiles += (it.n_states + v.ts - 1) / v.ts;
      lds = std::max(lds, tile_lds_bytes(P.N, P.NR, P.NG, v.ts, v.nt, true));
      kpt = std::max(kpt, kpt_of(P.N, v.ts, v.nt));
    }
    if (!c) break;
    wl.n_items = c;
    if (tiles >= ((int64_t)1 << 31)) return fail(PYJAC_E_INVALID, "work list too large for one launch");
    hipError_t e = launch_tile_multi(v.ts, v.nt, kpt, split == 1, wl, tiles, lds, st);
    if (e != hipSuccess) return fail(PYJAC_E_DEVICE, std::string("work-list launch failed: ") + hipGetErrorString(e));
  }
  return PYJAC_OK;
}

pyjac_status pyjac_conc_pattern(const pyjac_mech* m, int32_t* colptr, int32_t* rowidx, int64_t* nnz) {
  if (!m) return fail(PYJAC_E_INVALID, "mechanism handle is NULL");
  const PackedMech& P = m->host;
  if (nnz) *nnz = (int64_t)P.cv_rowidx.size();
  if (colptr) std::memcpy(colptr, P.cv_colptr.data(), P.cv_colptr.size() * sizeof(int32_t));
  if (rowidx && !P.cv_rowidx.empty())
    std::memcpy(rowidx, P.cv_rowidx.data(), P.cv_rowidx.size() * sizeof(int32_t));
  return PYJAC_OK;
}

pyjac_status pyjac_eval_jacobian_conc(const pyjac_mech* m, int64_t n, int64_t ld, const double* phi_c, double* jac,
                                      void* stream) {
  if (!m) return fail(PYJAC_E_INVALID, "mechanism handle is NULL");
  if (n < 0) return fail(PYJAC_E_INVALID, "n_states is negative");
  if (ld < n) return fail(PYJAC_E_INVALID, "ld is smaller than n_states");
  if (n == 0) return PYJAC_OK;
  if (!phi_c || !jac) return fail(PYJAC_E_INVALID, "phi_c and jac are required");
  if (misaligned(phi_c) || misaligned(jac)) return fail(PYJAC_E_INVALID, "pointer not 8-byte aligned");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != m->device)
    return fail(PYJAC_E_INVALID, "current HIP device differs from the mechanism's device");
  if (ld > (int64_t)1 << 40) return fail(PYJAC_E_INVALID, "ld too large");
  const Variant v = m->conc_var;
  if (!v.ts) return fail(PYJAC_E_UNSUPPORTED, "mechanism too large for the concentration-form tile");
  const size_t lds = conc_lds_bytes(m->host.N, m->host.NR, m->host.NG, v.ts, v.nt);
  const MechDev md = launch_view(m, v, true);
  hipError_t e = launch_conc(v.ts, v.nt, md, n, ld, phi_c, jac, lds, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(PYJAC_E_DEVICE, std::string("jacobian launch failed: ") + hipGetErrorString(e));
  return PYJAC_OK;
}

pyjac_status pyjac_eval_jacobian_cs(const pyjac_mech* m, int64_t n, int64_t ld, const double* phi, const double* p,
                                    double step, double* jac, void* stream) {
  pyjac_status rc = check_common(m, n, ld, phi, p);
  if (rc != PYJAC_OK) return rc;
  if (n > 0 && !jac) return fail(PYJAC_E_INVALID, "jac is NULL");
  if (misaligned(jac)) return fail(PYJAC_E_INVALID, "jac not 8-byte aligned");
  if (!(step > 0.0) || !(step <= 1e-6)) return fail(PYJAC_E_INVALID, "step must lie in (0, 1e-6]");
  if (m->host.N > 384) return fail(PYJAC_E_UNSUPPORTED, "complex-step Jacobian limited to 384 species");
  if (n == 0) return PYJAC_OK;
  hipError_t e = launch_cs_jacobian(m->dev, n, ld, phi, p, step, jac, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(PYJAC_E_DEVICE, std::string("complex-step launch failed: ") + hipGetErrorString(e));
  return PYJAC_OK;
}

pyjac_status pyjac_mix_pairs(const pyjac_mech* m, int64_t n, int64_t ld, const double* phi, const int32_t* partner,
                             double weight, double* phi_out, void* stream) {
  if (!m) return fail(PYJAC_E_INVALID, "mechanism handle is NULL");
  if (n < 0 || ld < n) return fail(PYJAC_E_INVALID, "bad n_states / ld");
  if (!(weight >= 0.0 && weight <= 0.5)) return fail(PYJAC_E_INVALID, "weight must lie in [0, 1/2]");
  if (n == 0) return PYJAC_OK;
  if (!phi || !partner || !phi_out) return fail(PYJAC_E_INVALID, "NULL array argument");
  if (phi_out == phi) return fail(PYJAC_E_INVALID, "phi_out may not alias phi");
  if (misaligned(phi) || misaligned(phi_out) || (reinterpret_cast<uintptr_t>(partner) & 3u))
    return fail(PYJAC_E_INVALID, "pointer not aligned");
  if (m->host.N > 1024) return fail(PYJAC_E_UNSUPPORTED, "more than 1024 species");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != m->device)
    return fail(PYJAC_E_INVALID, "current HIP device differs from the mechanism's device");
  hipError_t e = launch_mix_pairs(m->dev, n, ld, phi, partner, weight, phi_out, static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return fail(PYJAC_E_DEVICE, std::string("mixing launch failed: ") + hipGetErrorString(e));
  return PYJAC_OK;
}

size_t pyjac_fd_workspace_bytes(const pyjac_mech* m, int64_t chunk_states) {
  if (!m || chunk_states < 1) return 0;
  return (size_t)chunk_states * fd_bytes_per_state(m->host.N) + 1024;
}

pyjac_status pyjac_eval_jacobian_fd(const pyjac_mech* m, int64_t n, int64_t ld, const double* phi, const double* p,
                                    double* jac, void* workspace, size_t workspace_bytes, void* stream) {
  pyjac_status rc = check_common(m, n, ld, phi, p);
  if (rc != PYJAC_OK) return rc;
  if (n > 0 && !jac) return fail(PYJAC_E_INVALID, "jac is NULL");
  if (misaligned(jac) || misaligned(workspace)) return fail(PYJAC_E_INVALID, "pointer not 8-byte aligned");
  if (n == 0) return PYJAC_OK;
  const int N = m->host.N;
  const size_t per = fd_bytes_per_state(N);
  if (!workspace || workspace_bytes < per + 1024) return fail(PYJAC_E_WORKSPACE, "workspace smaller than one state");
  const int64_t chunk = std::min<int64_t>(n, (int64_t)((workspace_bytes - 1024) / per));
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const Variant v = m->rates_var;
  const size_t lds = tile_lds_bytes(N, m->host.NR, m->host.NG, v.ts, v.nt, false);
  const MechDev md = launch_view(m, v, false);
  auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
  for (int64_t s0 = 0; s0 < n; s0 += chunk) {
    const int64_t mm = std::min(chunk, n - s0), ld2 = mm * (N + 1);
    char* w = static_cast<char*>(workspace);
    double* phi2 = reinterpret_cast<double*>(w);
    w += al((size_t)N * ld2 * 8);
    double* f2 = reinterpret_cast<double*>(w);
    w += al((size_t)N * ld2 * 8);
    double* p2 = reinterpret_cast<double*>(w);
    w += al((size_t)ld2 * 8);
    double* inc = reinterpret_cast<double*>(w);
    hipError_t e = fd_perturb(N, mm, ld, phi, p, s0, phi2, p2, ld2, inc, st);
    if (e == hipSuccess)
      e = launch_tile(false, v.ts, v.nt, md, ld2, ld2, phi2, p2, nullptr, nullptr, nullptr, nullptr, f2, nullptr,
                      lds, st);
    if (e == hipSuccess) e = fd_diff(N, mm, f2, ld2, inc, s0, jac, ld, st);
    if (e != hipSuccess) return fail(PYJAC_E_DEVICE, std::string("finite-difference launch failed: ") + hipGetErrorString(e));
  }
  return PYJAC_OK;
}

// Tuning hook: force the launch shape of one kernel family (which = 0 rates,
// 1 Jacobian).  ts = 0 restores the automatic choice.  Returns
// PYJAC_E_UNSUPPORTED when the shape does not fit the device or the mechanism.
pyjac_status pyjac_mech_set_variant(pyjac_mech* m, int32_t which, int32_t ts, int32_t nt) {
  if (!m || which < 0 || which > 2) return fail(PYJAC_E_INVALID, "bad handle or kernel id");
  if (which == 2) {
    Variant v{ts, nt};
    if (ts == 0) v = pick_conc(m->host, m->max_lds);
    else {
      bool found = false;
      for (auto& q : kConcShapes) found |= (q[0] == ts && q[1] == nt);
      if (!found) return fail(PYJAC_E_UNSUPPORTED, "variant not compiled");
      if (!conc_fits(m->host, v, m->max_lds)) return fail(PYJAC_E_UNSUPPORTED, "variant does not fit");
    }
    if (v.ts) {
      pyjac_status rc = ensure_var(m, v, true);
      if (rc != PYJAC_OK) return rc;
    }
    m->conc_var = v;
    return PYJAC_OK;
  }
  const bool jac = which == 1;
  Variant v{ts, nt};
  if (ts == 0) v = pick(m->host, jac, m->max_lds);
  else {
    if (ts <= 0 || nt <= 0 || nt % ts) return fail(PYJAC_E_INVALID, "bad variant");
    if (kpt_of(m->host.N, ts, nt) > 8 || tile_lds_bytes(m->host.N, m->host.NR, m->host.NG, ts, nt, jac) > m->max_lds)
      return fail(PYJAC_E_UNSUPPORTED, "variant does not fit");
    static const int ok[][2] = {{16, 512}, {16, 1024}, {8, 512}, {8, 1024}, {4, 512}, {4, 1024},
                                {2, 512},  {2, 1024}, {32, 1024}, {64, 1024}, {8, 256}, {4, 256}};
    bool found = false;
    for (auto& q : ok) found |= (q[0] == ts && q[1] == nt);
    if (!found) return fail(PYJAC_E_UNSUPPORTED, "variant not compiled");
  }
  pyjac_status rc = ensure_var(m, v, jac);
  if (rc != PYJAC_OK) return rc;
  (jac ? m->jac_var : m->rates_var) = v;
  return PYJAC_OK;
}

pyjac_status pyjac_mech_autotune(pyjac_mech* m, int32_t which, int64_t n, int64_t ld, const double* phi,
                                 const double* p, double* out, int32_t reps, int32_t* shapes, float* ms,
                                 int32_t max_entries, int32_t* n_entries, void* stream) {
  if (!m || which < 0 || which > 2) return fail(PYJAC_E_INVALID, "bad handle or kernel id");
  if (reps < 1 || n < 1) return fail(PYJAC_E_INVALID, "reps and n_states must be positive");
  // the concentration form takes no pressure array (p may be NULL)
  pyjac_status rc = check_common(m, n, ld, phi, which == 2 ? phi : p);
  if (rc != PYJAC_OK) return rc;
  if (!out || misaligned(out)) return fail(PYJAC_E_INVALID, "out is NULL or not 8-byte aligned");
  if (n_entries) *n_entries = 0;
  const bool jac = which == 1;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  static const int shapes_all[][2] = {{16, 1024}, {16, 512}, {32, 1024}, {64, 1024}, {8, 512}, {8, 1024},
                                      {4, 512},   {4, 1024}, {2, 512},   {2, 1024},  {8, 256}, {4, 256}};
  int prev = 0;
  hipGetDevice(&prev);
  hipSetDevice(m->device);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) {
    if (e0) hipEventDestroy(e0);
    hipSetDevice(prev);
    return fail(PYJAC_E_DEVICE, "hipEventCreate failed");
  }
  Variant best{0, 0};
  float best_ms = 0.0f;
  int count = 0;
  rc = PYJAC_OK;
  const bool conc = which == 2;
  const int n_shapes = conc ? (int)(sizeof(kConcShapes) / sizeof(kConcShapes[0]))
                            : (int)(sizeof(shapes_all) / sizeof(shapes_all[0]));
  for (int si = 0; si < n_shapes; ++si) {
    const Variant v = conc ? Variant{kConcShapes[si][0], kConcShapes[si][1]}
                           : Variant{shapes_all[si][0], shapes_all[si][1]};
    if (kpt_of(m->host.N, v.ts, v.nt) > 8) continue;
    const size_t lds = kind_lds(m, which, v);
    if (lds > m->max_lds) continue;
    if ((rc = ensure_var(m, v, jac || conc)) != PYJAC_OK) break;
    const MechDev md = launch_view(m, v, jac || conc);
    auto launch = [&]() {
      if (conc) return launch_conc(v.ts, v.nt, md, n, ld, phi, out, lds, st);
      return jac ? launch_tile(true, v.ts, v.nt, md, n, ld, phi, p, nullptr, nullptr, nullptr, nullptr,
                               nullptr, out, lds, st)
                 : launch_tile(false, v.ts, v.nt, md, n, ld, phi, p, nullptr, nullptr, nullptr, nullptr,
                               out, nullptr, lds, st);
    };
    std::vector<float> t;
    hipError_t err = launch();
    for (int r = 0; r < reps && err == hipSuccess; ++r) {
      hipEventRecord(e0, st);
      err = launch();
      hipEventRecord(e1, st);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float x = 0.0f;
      if (err == hipSuccess) err = hipEventElapsedTime(&x, e0, e1);
      t.push_back(x);
    }
    if (err != hipSuccess) {
      rc = fail(PYJAC_E_DEVICE, std::string("autotune launch failed: ") + hipGetErrorString(err));
      break;
    }
    std::sort(t.begin(), t.end());
    const float med = t[t.size() / 2];
    if (shapes && ms && count < max_entries) {
      shapes[2 * count] = v.ts;
      shapes[2 * count + 1] = v.nt;
      ms[count] = med;
    }
    ++count;
    // a later shape must be clearly faster (2 %) to replace an earlier,
    // preferred one, so that timing noise does not flip the choice
    if (!best.ts || med < 0.98f * best_ms) { best = v; best_ms = med; }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  hipSetDevice(prev);
  if (rc != PYJAC_OK) return rc;
  if (!best.ts) return fail(PYJAC_E_UNSUPPORTED, "no launch shape fits");
  (conc ? m->conc_var : jac ? m->jac_var : m->rates_var) = best;
  if (n_entries) *n_entries = count < max_entries ? count : max_entries;
  return PYJAC_OK;
}

pyjac_status pyjac_mech_get_variant(const pyjac_mech* m, int32_t which, int32_t* ts, int32_t* nt,
                                    size_t* lds_bytes) {
  if (!m || which < 0 || which > 2) return fail(PYJAC_E_INVALID, "bad handle or kernel id");
  const Variant v = which == 2 ? m->conc_var : which ? m->jac_var : m->rates_var;
  if (ts) *ts = v.ts;
  if (nt) *nt = v.nt;
  if (lds_bytes) *lds_bytes = v.ts ? kind_lds(m, which, v) : 0;
  return PYJAC_OK;
}

}  // extern "C"

namespace pyjac {
int mech_device(const pyjac_mech* m) { return m->device; }
int mech_species(const pyjac_mech* m) { return m->host.N; }
}  // namespace pyjac

extern "C" {

const char* pyjac_status_string(pyjac_status s) {
  switch (s) {
    case PYJAC_OK: return "ok";
    case PYJAC_E_INVALID: return "invalid argument";
    case PYJAC_E_PARSE: return "mechanism parse error";
    case PYJAC_E_UNSUPPORTED: return "unsupported feature";
    case PYJAC_E_DEVICE: return "HIP device error";
    case PYJAC_E_NOMEM: return "out of memory";
    case PYJAC_E_IO: return "I/O error";
    case PYJAC_E_UNBALANCED: return "reaction not element-balanced";
    case PYJAC_E_WORKSPACE: return "workspace too small";
    default: return "unknown status";
  }
}

const char* pyjac_last_error(void) { return g_last_error.c_str(); }

}  // extern "C"
