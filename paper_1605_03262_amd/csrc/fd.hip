// Finite-difference Jacobian (first-order forward differences of the RHS),
// the comparison method of the paper's performance study (Sec. 5), built on
// the library's own RHS kernel.
//
// For a chunk of m states, the perturbation kernel writes m*(N+1) states in
// N+1 blocks of m columns: block 0 holds the unperturbed states and block
// 1 + j the states with Phi_j raised by its increment, state s at column
// block*m + s, so that every kernel reads and writes consecutive states with
// consecutive lanes.  The RHS kernel evaluates them all; the
// difference kernel forms J_ij = (f_i(Phi + d_j e_j) - f_i(Phi)) / d_j, where
// d_j is the increment actually represented, (Phi_j + inc_j) - Phi_j, with
// inc_j = sqrt(u) * max(|Phi_j|, floor_j) (floor 1 K for the temperature,
// 1e-10 for mass fractions).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

namespace pyjac {

namespace {

constexpr double kSqrtEps = 1.4901161193847656e-08;   // 2^-26

// grid: (ceil(m / 64), N + 1); thread = one state of the chunk, y = column
__global__ __launch_bounds__(64) void fd_perturb_kernel(int N, int64_t m, int64_t ld, const double* __restrict__ phi,
                                                        const double* __restrict__ p, int64_t s0,
                                                        double* __restrict__ phi2, double* __restrict__ p2,
                                                        int64_t ld2, double* __restrict__ inc) {
  const int64_t sl = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int c = blockIdx.y;               // 0: base, 1 + j: Phi_j perturbed
  if (sl >= m) return;
  const int64_t s = s0 + sl;
  const int64_t col = (int64_t)c * m + sl;
  for (int k = 0; k < N; ++k) {
    double v = phi[(int64_t)k * ld + s];
    if (c == k + 1) {
      const double fl = k == 0 ? 1.0 : 1e-10;
      const double vp = v + kSqrtEps * fmax(fabs(v), fl);
      inc[(int64_t)k * m + sl] = vp - v;
      v = vp;
    }
    phi2[(int64_t)k * ld2 + col] = v;
  }
  p2[col] = p[s];
}

// grid: (ceil(m / 64), N); thread = one state, y = row i; loops over columns j
__global__ __launch_bounds__(64) void fd_diff_kernel(int N, int64_t m, const double* __restrict__ f2, int64_t ld2,
                                                     const double* __restrict__ inc, int64_t s0,
                                                     double* __restrict__ jac, int64_t ld) {
  const int64_t sl = (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int i = blockIdx.y;
  if (sl >= m) return;
  const double* fr = f2 + (int64_t)i * ld2 + sl;
  const double f0 = fr[0];
  for (int j = 0; j < N; ++j)
    jac[((int64_t)i * N + j) * ld + s0 + sl] = (fr[(int64_t)(1 + j) * m] - f0) / inc[(int64_t)j * m + sl];
}

}  // namespace

// Bytes of device workspace per state of a chunk: perturbed states, their
// pressures and RHS values, and the increments.
size_t fd_bytes_per_state(int N) { return ((size_t)(N + 1) * (2 * N + 1) + (size_t)N) * sizeof(double); }

hipError_t fd_perturb(int N, int64_t m, int64_t ld, const double* phi, const double* p, int64_t s0, double* phi2,
                      double* p2, int64_t ld2, double* inc, hipStream_t st) {
  dim3 g((unsigned)((m + 63) / 64), (unsigned)(N + 1));
  hipLaunchKernelGGL(fd_perturb_kernel, g, dim3(64), 0, st, N, m, ld, phi, p, s0, phi2, p2, ld2, inc);
  return hipGetLastError();
}

hipError_t fd_diff(int N, int64_t m, const double* f2, int64_t ld2, const double* inc, int64_t s0, double* jac,
                   int64_t ld, hipStream_t st) {
  dim3 g((unsigned)((m + 63) / 64), (unsigned)N);
  hipLaunchKernelGGL(fd_diff_kernel, g, dim3(64), 0, st, N, m, f2, ld2, inc, s0, jac, ld);
  return hipGetLastError();
}

}  // namespace pyjac
