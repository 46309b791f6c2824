// One implicit integrator step per state: the three-stage, L-stable, stiffly
// accurate SDIRK method of order 3 (Alexander, 1977) whose diagonal
// coefficient is the gamma = 0.43586652150845899942 of the Newton matrix
// I - h gamma J that motivates fast Jacobians (Sec. 1).
//
// Stage i solves z_i = h sum_{j<i} a_ij F_j + h gamma f(y + z_i), F_j =
// f(y + z_j), by simplified Newton with the matrix I - h gamma J(y) from
// z_i = 0 for a fixed number of iterations; y_next = y + z_3.  The RHS, the
// Jacobian and the Newton solves are the library's own kernels (the matrix is
// factored once per step where the Newton path keeps its factor); the kernels
// here only combine per-state vectors, element-major with the state fastest
// like every other array (coalesced, HBM-bound, no reductions across states).
#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>

#include "../../include/pyjac.h"

namespace pyjac {
pyjac_status fail(pyjac_status code, const std::string& msg);
int mech_species(const pyjac_mech* m);

namespace {

constexpr double kG = 0.43586652150845899942;
constexpr double kA21 = (1.0 - kG) / 2.0;
constexpr double kB1 = -(6.0 * kG * kG - 16.0 * kG + 1.0) / 4.0;
constexpr double kB2 = (6.0 * kG * kG - 20.0 * kG + 5.0) / 4.0;

// rhs = h (a1 F1 + a2 F2 + gamma fz) - z  (the negated stage residual);
// F1 / F2 unused when their coefficient is zero
__global__ void stage_rhs_kernel(int N, int64_t n, int64_t ld, const double* __restrict__ h, double a1,
                                 const double* __restrict__ F1, double a2, const double* __restrict__ F2,
                                 const double* __restrict__ fz, const double* __restrict__ z,
                                 double* __restrict__ rhs) {
  const int64_t total = (int64_t)N * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / n, s = i - e * n, o = e * ld + s;
    double acc = kG * fz[o];
    if (a1 != 0.0) acc += a1 * F1[o];
    if (a2 != 0.0) acc += a2 * F2[o];
    rhs[o] = h[s] * acc - z[o];
  }
}

// z += d (when d is given; z = 0 otherwise) and Y = y + z
__global__ void stage_update_kernel(int N, int64_t n, int64_t ld, const double* __restrict__ y,
                                    const double* __restrict__ d, double* __restrict__ z, double* __restrict__ Y) {
  const int64_t total = (int64_t)N * n;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t e = i / n, s = i - e * n, o = e * ld + s;
    const double zn = d ? z[o] + d[o] : 0.0;
    z[o] = zn;
    Y[o] = y[o] + zn;
  }
}

// out[s] = max_e |d[e][s]|
__global__ void max_abs_kernel(int N, int64_t n, int64_t ld, const double* __restrict__ d, double* __restrict__ out) {
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
    double m = 0.0;
    for (int e = 0; e < N; ++e) m = fmax(m, fabs(d[(int64_t)e * ld + s]));
    out[s] = m;
  }
}

unsigned grid_for(int64_t work) {
  const int64_t b = (work + 255) / 256;
  return (unsigned)(b < 1 ? 1 : (b > 65535 ? 65535 : b));
}

}  // namespace

// Stage coefficients a_ij (j < i) of stage i.
void sdirk_stage_coeffs(int i, double& a1, double& a2) {
  a1 = i == 1 ? kA21 : (i == 2 ? kB1 : 0.0);
  a2 = i == 2 ? kB2 : 0.0;
}

hipError_t sdirk_stage_rhs(int N, int64_t n, int64_t ld, const double* h, double a1, const double* F1, double a2,
                           const double* F2, const double* fz, const double* z, double* rhs, hipStream_t st) {
  hipLaunchKernelGGL(stage_rhs_kernel, dim3(grid_for((int64_t)N * n)), dim3(256), 0, st, N, n, ld, h, a1, F1, a2,
                     F2, fz, z, rhs);
  return hipGetLastError();
}

hipError_t sdirk_stage_update(int N, int64_t n, int64_t ld, const double* y, const double* d, double* z, double* Y,
                              hipStream_t st) {
  hipLaunchKernelGGL(stage_update_kernel, dim3(grid_for((int64_t)N * n)), dim3(256), 0, st, N, n, ld, y, d, z, Y);
  return hipGetLastError();
}

hipError_t sdirk_max_abs(int N, int64_t n, int64_t ld, const double* d, double* out, hipStream_t st) {
  hipLaunchKernelGGL(max_abs_kernel, dim3(grid_for(n)), dim3(256), 0, st, N, n, ld, d, out);
  return hipGetLastError();
}

namespace {

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct SdirkLayout {
  size_t J, vec, info, nws, total;   // byte offsets / sizes
};

SdirkLayout sdirk_layout(const pyjac_mech* m, int64_t n, int64_t ld, int32_t mode) {
  const int N = mech_species(m);
  SdirkLayout L;
  L.J = 0;
  L.vec = align256((size_t)N * N * ld * sizeof(double));
  L.info = L.vec + 7 * align256((size_t)N * ld * sizeof(double));
  L.nws = L.info + align256((size_t)ld * sizeof(int32_t));
  L.total = L.nws + align256(pyjac_newton_workspace_bytes(m, n, mode | PYJAC_NEWTON_KEEP_FACTOR));
  return L;
}

}  // namespace
}  // namespace pyjac

extern "C" {

size_t pyjac_sdirk3_workspace_bytes(const pyjac_mech* m, int64_t n, int64_t ld, int32_t mode) {
  if (!m || n < 0 || ld < n || (mode != 0 && mode != 1)) return 0;
  return pyjac::sdirk_layout(m, n, ld, mode).total;
}

pyjac_status pyjac_sdirk3_step(const pyjac_mech* m, int64_t n, int64_t ld, const double* phi, const double* p,
                               const double* h, int32_t newton_iters, int32_t mode, double* phi_out,
                               double* dnorm, void* workspace, size_t workspace_bytes, void* stream) {
  using namespace pyjac;
  if (!m) return fail(PYJAC_E_INVALID, "mechanism handle is NULL");
  if (n < 0 || ld < n) return fail(PYJAC_E_INVALID, "need 0 <= n_states <= ld");
  if (newton_iters < 1 || newton_iters > 16) return fail(PYJAC_E_INVALID, "newton_iters must be in [1, 16]");
  if (mode != 0 && mode != 1) return fail(PYJAC_E_INVALID, "mode must be 0 or 1");
  if (n == 0) return PYJAC_OK;         // empty batch: the arrays may be NULL
  if (!phi || !p || !h || !phi_out) return fail(PYJAC_E_INVALID, "NULL array argument");
  const SdirkLayout L = sdirk_layout(m, n, ld, mode);
  if (!workspace || workspace_bytes < L.total)
    return fail(PYJAC_E_WORKSPACE, "workspace smaller than pyjac_sdirk3_workspace_bytes");
  hipStream_t st = (hipStream_t)stream;
  const int N = mech_species(m);
  char* w = static_cast<char*>(workspace);
  double* J = reinterpret_cast<double*>(w + L.J);
  double* v[7];
  for (int k = 0; k < 7; ++k) v[k] = reinterpret_cast<double*>(w + L.vec + k * align256((size_t)N * ld * sizeof(double)));
  double *F1 = v[0], *F2 = v[1], *z = v[2], *Y = v[3], *fz = v[4], *rhs = v[5], *d = v[6];
  int32_t* info = reinterpret_cast<int32_t*>(w + L.info);
  void* nws = w + L.nws;
  const size_t nwsb = L.total - L.nws;
  pyjac_status rc = pyjac_eval_jacobian(m, n, ld, phi, p, J, stream);
  if (rc != PYJAC_OK) return rc;
  for (int i = 0; i < 3; ++i) {
    double a1, a2;
    sdirk_stage_coeffs(i, a1, a2);
    if (sdirk_stage_update(N, n, ld, phi, nullptr, z, Y, st) != hipSuccess) return fail(PYJAC_E_DEVICE, "launch failed");
    for (int it = 0; it < newton_iters; ++it) {
      rc = pyjac_eval_rates(m, n, ld, Y, p, nullptr, nullptr, nullptr, nullptr, fz, stream);
      if (rc != PYJAC_OK) return rc;
      if (sdirk_stage_rhs(N, n, ld, h, a1, F1, a2, F2, fz, z, rhs, st) != hipSuccess)
        return fail(PYJAC_E_DEVICE, "launch failed");
      // I - h gamma J(y) is the same for every solve of the step: factored once
      const int32_t nmode = mode | ((i == 0 && it == 0) ? PYJAC_NEWTON_KEEP_FACTOR : PYJAC_NEWTON_REUSE_FACTOR);
      rc = pyjac_newton_factor_solve(m, n, ld, J, h, kG, rhs, d, nmode, 4, 1e-14, info, nws, nwsb, stream);
      if (rc != PYJAC_OK) return rc;
      // the last update of the last stage writes the result (y + z_3)
      double* dst = (i == 2 && it == newton_iters - 1) ? phi_out : Y;
      if (sdirk_stage_update(N, n, ld, phi, d, z, dst, st) != hipSuccess) return fail(PYJAC_E_DEVICE, "launch failed");
    }
    if (dnorm && sdirk_max_abs(N, n, ld, d, dnorm + (int64_t)i * ld, st) != hipSuccess)
      return fail(PYJAC_E_DEVICE, "launch failed");
    if (i < 2) {
      rc = pyjac_eval_rates(m, n, ld, Y, p, nullptr, nullptr, nullptr, nullptr, i == 0 ? F1 : F2, stream);
      if (rc != PYJAC_OK) return rc;
    }
  }
  return PYJAC_OK;
}

}  // extern "C"
