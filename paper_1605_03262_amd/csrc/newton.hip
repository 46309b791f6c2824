// Batched solves of the Newton matrix of an implicit integrator step,
// (I - h gamma J) x = b, for every state of a batch (gfx950).
//
//  form      : A = I - h gamma J, transposed from the element-major,
//              state-fastest Jacobian into one contiguous row-major N x N
//              matrix per state (FP64 or FP32), through an LDS tile so both
//              the reads and the writes are coalesced.
//  lu        : one workgroup per state; right-looking LU with partial
//              pivoting in panels of 16 columns.  The panel is factored in
//              LDS, the row interchanges are applied to the other columns,
//              U12 = L11^-1 A12 is formed in LDS and the trailing matrix is
//              updated with 16x16x4 matrix-core instructions (FP32 or FP64).
//  solve     : one wavefront per state; P b, unit-lower and upper
//              triangular solves by row dot products.
//  residual  : r = b - (I - h gamma J) x in FP64, one thread per state,
//              straight from the state-fastest Jacobian (coalesced).
// Mode 1 (mixed) factors in FP32, refines in FP64 and re-solves the states
// that do not converge with the FP64 path (compacted list, device-side).
// Systems with N <= 64 take register-resident kernels instead (FP64: one
// state per wavefront; FP32 factor: several states per wavefront).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>
#include <utility>

#include "../../include/pyjac.h"
#include "tables.hpp"

namespace pyjac {
pyjac_status fail(pyjac_status code, const std::string& msg);
int mech_device(const pyjac_mech* m);
int mech_species(const pyjac_mech* m);

namespace {

constexpr int NB = 16;           // panel width
constexpr int LU_THREADS = 256;  // 4 wavefronts per state
constexpr int ST_UNSET = -100;   // internal per-state status before convergence
constexpr int ST_SING32 = -4;    // zero pivot in the FP32 factor: re-solved in FP64

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef double doublex4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- form
// grid: (ceil(n/16), ceil(N*N/64)); 256 threads: tile of 64 elements x 16 states
template <typename T>
__global__ __launch_bounds__(256) void form_kernel(int N, int64_t n, int64_t ld, const double* __restrict__ jac,
                                                   const double* __restrict__ h, double gamma,
                                                   T* __restrict__ A, const int* __restrict__ list,
                                                   const int* __restrict__ count, int* __restrict__ status) {
  __shared__ T tile[64][17];
  const int tid = threadIdx.x;
  const int64_t NN = (int64_t)N * N;
  const int64_t e0 = (int64_t)blockIdx.y * 64;
  const int64_t s0 = (int64_t)blockIdx.x * 16;
  const int64_t lim = count ? *count : n;
  // load: lanes state-fastest
  {
    const int s = tid % 16;
    const int64_t slot = s0 + s;
    const bool ok = slot < lim;
    const int64_t st = ok ? (list ? list[slot] : slot) : 0;
    const double hg = ok ? h[st] * gamma : 0.0;
    for (int r = tid / 16; r < 64; r += 16) {
      const int64_t e = e0 + r;
      T v = T(0);
      if (ok && e < NN) {
        const double jv = jac[e * ld + st];
        const int64_t i = e / N, j = e % N;
        const double a = (i == j ? 1.0 : 0.0) - hg * jv;
        if (!isfinite(a)) status[st] = -3;
        v = (T)a;
      }
      tile[r][s] = v;
    }
  }
  __syncthreads();
  // store: lanes element-fastest, one contiguous row-major matrix per state
  {
    const int r = tid % 64;
    for (int s = tid / 64; s < 16; s += 4) {
      const int64_t slot = s0 + s, e = e0 + r;
      if (slot < lim && e < NN) A[slot * NN + e] = tile[r][s];
    }
  }
}

template <typename T> struct Mfma;
// 16x16x4 matrix-core products.  Both precisions take A[row = lane % 16][k =
// lane / 16] and B[k = lane / 16][col = lane % 16]; the result slot v of lane
// l holds column l % 16 and row row(l / 16, v), which differs between the FP32
// and the FP64 instruction (checked on gfx950 with one-hot operands).
template <> struct Mfma<float> {
  typedef floatx4 acc_t;
  __device__ static acc_t run(float a, float b, acc_t c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int q, int v) { return 4 * q + v; }
};
template <> struct Mfma<double> {
  typedef doublex4 acc_t;
  __device__ static acc_t run(double a, double b, acc_t c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  __device__ static int row(int q, int v) { return q + 4 * v; }
};

// ---------------------------------------------------------------- LU
// One workgroup per (listed) state.  A: row-major N x N per slot; piv: N per slot.
// LDS: panel Pn[N][NB+1], U12 U[NB][N+1], reduction scratch.
template <typename T>
__global__ __launch_bounds__(LU_THREADS) void lu_kernel(int N, int64_t n, T* __restrict__ Aall,
                                                        int* __restrict__ pivall, const int* __restrict__ list,
                                                        const int* __restrict__ count, int* __restrict__ status,
                                                        int sing_code) {
  extern __shared__ char smem[];
  const int64_t slot = blockIdx.x;
  const int64_t lim = count ? *count : n;
  if (slot >= lim) return;
  const int64_t st = list ? list[slot] : slot;
  if (status[st] == -3) return;
  T* A = Aall + slot * (int64_t)N * N;
  int* piv = pivall + slot * (int64_t)N;
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  const int PS = NB + 1, US = N + 1;
  T* Pn = reinterpret_cast<T*>(smem);                       // N * PS
  T* U = Pn + (size_t)N * PS;                               // NB * US
  T* redv = U + (size_t)NB * US;                            // LU_THREADS
  int* redi = reinterpret_cast<int*>(redv + LU_THREADS);    // LU_THREADS
  __shared__ int singular;
  if (tid == 0) singular = 0;
  for (int k0 = 0; k0 < N; k0 += NB) {
    const int nb = min(NB, N - k0), M = N - k0, W = N - k0 - nb;
    // 1. panel to LDS
    for (int e = tid; e < M * nb; e += LU_THREADS) {
      const int r = e / nb, c = e % nb;
      Pn[r * PS + c] = A[(int64_t)(k0 + r) * N + k0 + c];
    }
    __syncthreads();
    // 2. factor the panel with partial pivoting
    for (int c = 0; c < nb; ++c) {
      T best = T(-1);
      int bi = c;
      for (int r = c + tid; r < M; r += LU_THREADS) {
        const T v = fabs(Pn[r * PS + c]);
        if (v > best) { best = v; bi = r; }
      }
      redv[tid] = best;
      redi[tid] = bi;
      __syncthreads();
      for (int w = LU_THREADS / 2; w > 0; w >>= 1) {
        if (tid < w) {
          const T a = redv[tid], b = redv[tid + w];
          const int ia = redi[tid], ib = redi[tid + w];
          if (b > a || (b == a && ib < ia)) { redv[tid] = b; redi[tid] = ib; }
        }
        __syncthreads();
      }
      const int pr = redi[0];
      const T pmax = redv[0];
      if (tid == 0) {
        piv[k0 + c] = k0 + pr;
        if (!(pmax > T(0))) singular = 1;
      }
      if (pr != c && tid < nb) {
        const T t = Pn[c * PS + tid];
        Pn[c * PS + tid] = Pn[pr * PS + tid];
        Pn[pr * PS + tid] = t;
      }
      __syncthreads();
      const T d = Pn[c * PS + c];
      const T inv = d != T(0) ? T(1) / d : T(0);
      for (int r = c + 1 + tid; r < M; r += LU_THREADS) {
        const T l = Pn[r * PS + c] * inv;
        Pn[r * PS + c] = l;
        for (int cc = c + 1; cc < nb; ++cc) Pn[r * PS + cc] -= l * Pn[c * PS + cc];
      }
      __syncthreads();
    }
    // 3. panel back to global
    for (int e = tid; e < M * nb; e += LU_THREADS) {
      const int r = e / nb, c = e % nb;
      A[(int64_t)(k0 + r) * N + k0 + c] = Pn[r * PS + c];
    }
    // 4. row interchanges on the columns outside the panel (sequential in c)
    for (int c = 0; c < nb; ++c) {
      const int pr = piv[k0 + c];
      if (pr != k0 + c) {
        for (int col = tid; col < N - nb; col += LU_THREADS) {
          const int cc = col < k0 ? col : col + nb;
          const T t = A[(int64_t)(k0 + c) * N + cc];
          A[(int64_t)(k0 + c) * N + cc] = A[(int64_t)pr * N + cc];
          A[(int64_t)pr * N + cc] = t;
        }
      }
      __syncthreads();
    }
    if (W <= 0) break;
    // 5. U12 = L11^-1 A12 (unit lower), in LDS, then back to global
    for (int e = tid; e < nb * W; e += LU_THREADS) {
      const int r = e / W, c = e % W;
      U[r * US + c] = A[(int64_t)(k0 + r) * N + k0 + nb + c];
    }
    __syncthreads();
    for (int c = tid; c < W; c += LU_THREADS) {
      for (int r = 1; r < nb; ++r) {
        T acc = U[r * US + c];
        for (int t = 0; t < r; ++t) acc -= Pn[r * PS + t] * U[t * US + c];
        U[r * US + c] = acc;
      }
    }
    __syncthreads();
    for (int e = tid; e < nb * W; e += LU_THREADS) {
      const int r = e / W, c = e % W;
      A[(int64_t)(k0 + r) * N + k0 + nb + c] = U[r * US + c];
    }
    // 6. trailing update A22 -= L21 U12 on the matrix cores, 16x16 tiles
    const int tr = (W + 15) / 16;
    const int row = lane % 16, kq = lane / 16;
    for (int t = wave; t < tr * tr; t += LU_THREADS / 64) {
      const int r0 = (t / tr) * 16, c0 = (t % tr) * 16;
      typename Mfma<T>::acc_t acc;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = r0 + Mfma<T>::row(kq, i), cc = c0 + row;
        acc[i] = (rr < W && cc < W) ? A[(int64_t)(k0 + nb + rr) * N + k0 + nb + cc] : T(0);
      }
#pragma unroll
      for (int kk = 0; kk < NB; kk += 4) {
        const int ar = r0 + row, bc = c0 + row, kx = kk + kq;
        const T a = (ar < W && kx < nb) ? -Pn[(nb + ar) * PS + kx] : T(0);
        const T b = (bc < W && kx < nb) ? U[kx * US + bc] : T(0);
        acc = Mfma<T>::run(a, b, acc);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int rr = r0 + Mfma<T>::row(kq, i), cc = c0 + row;
        if (rr < W && cc < W) A[(int64_t)(k0 + nb + rr) * N + k0 + nb + cc] = acc[i];
      }
    }
    __syncthreads();
  }
  if (tid == 0 && singular) status[st] = sing_code;
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

// ---------------------------------------------------------------- small systems
// N <= 64, FP64 (mode 0, and the mixed mode's fallback): one wavefront per
// state, lane i holding row i of I - h gamma J in registers (NM = N rounded
// up to 16, 32, 48, 56 or 64 columns, indexed by compile-time constants
// only; the border is an identity, so every update runs unguarded over the
// full width).  A block of SW states shares one workgroup only to read the
// state-fastest Jacobian in coalesced 64-byte runs through LDS; after that
// every wavefront factors and solves on its own, with no barrier:
//  * right-looking LU with partial pivoting, rows kept in place (lane i keeps
//    row i; `stp` records the elimination step at which it became the pivot
//    row).  The pivot is the active lane with the largest |a_ik| (compared on
//    the high 32 bits of the FP64/FP32 pattern, which order non-negative
//    values; ties go to the lowest lane); the pivot row reaches the other
//    lanes through v_readlane.
//  * forward and backward substitution in pivot order.
// The mixed mode's FP32 factor has its own kernel (grp_mixed_kernel, below);
// states it leaves unconverged or singular are listed and re-solved here.
constexpr int kSmallMax = 64;  // largest N taken by the register-resident path
// register width of the path for N <= kSmallMax (launch_small instantiates
// exactly these widths)
constexpr int small_width(int N) { return N <= 16 ? 16 : N <= 32 ? 32 : N <= 48 ? 48 : N <= 56 ? 56 : 64; }
// FP64 register path: states (one per wavefront) per workgroup, and Jacobian
// rows staged per LDS pass.  Two such workgroups fill a CU at two wavefronts
// per SIMD (the register budget), and the stage fits both in LDS up to 64
// columns; fewer wavefronts per staging barrier and fewer passes than eight
// states of 16 rows measured 25 % faster at 53 species.
constexpr int kSmallWaves = 4;
constexpr int SRB = 32;

// Compile-time loop: f(std::integral_constant<int, j>) for j in [B, E), so
// that register arrays are only ever indexed by constants.
template <int B, int E, typename F>
__device__ __forceinline__ void sfor(F&& f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    sfor<B + 1, E>(f);
  }
}
// The same in groups of 8 with a scheduling barrier after each group, so that
// LDS operands are not all fetched ahead into registers at once.
template <int B, int E, typename F>
__device__ __forceinline__ void sfor8(F&& f) {
  if constexpr (B < E) {
    constexpr int M = (B + 8 < E) ? B + 8 : E;
    sfor<B, M>(f);
    __builtin_amdgcn_sched_barrier(0);
    sfor8<M, E>(f);
  }
}

// Workgroups are dispatched round-robin over the eight XCDs; this permutation
// gives every XCD a contiguous range of blocks, so neighbouring blocks, whose
// 64-byte runs of the Jacobian share cache lines, read through the same L2.
__device__ inline unsigned xcd_block() {
  constexpr unsigned kXcd = 8;
  const unsigned b = blockIdx.x, G = gridDim.x;
  const unsigned q = G / kXcd, r = G % kXcd, x = b % kXcd, i = b / kXcd;
  return x * q + (x < r ? x : r) + i;
}

// Marks every entry of a register array as modified (no code emitted).
template <int J, int NM, typename T>
__device__ __forceinline__ void opaque_regs(T (&a)[NM]) {
  if constexpr (J < NM) {
    __asm__ volatile("" : "+v"(a[J]));
    opaque_regs<J + 1, NM>(a);
  }
}

__device__ __forceinline__ double lane_bcast(double v, int lane) {
  const unsigned long long u = __double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}
__device__ __forceinline__ float lane_bcast(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ unsigned mag_key(double v) {
  return (unsigned)((unsigned long long)__double_as_longlong(v) >> 32) & 0x7FFFFFFFu;
}
__device__ __forceinline__ unsigned mag_key(float v) { return (unsigned)__float_as_int(v) & 0x7FFFFFFFu; }
__device__ __forceinline__ int first_lane(unsigned long long m) { return (int)__builtin_ctzll(m); }

// One elimination step K of the LU of the wave's rows (see small_lu).  Every
// step runs unconditionally (no early exit), so the row array stays one set
// of registers; a zero or non-finite pivot column only raises `bad`.  The
// pivot row reaches the other lanes element by element through v_readlane
// (scalar registers), with no memory round trip.
template <int K, int NM, typename T>
__device__ __forceinline__ void small_lu_step(T (&a)[NM], int lane, bool& used, int& stp, bool& bad) {
  const unsigned key = used ? 0u : mag_key(a[K]);
  const unsigned mk = __ockl_wfred_max_u32(key);
  const unsigned inf_key = sizeof(T) == 8 ? 0x7FF00000u : 0x7F800000u;
  bad = bad || mk == 0u || mk >= inf_key;                    // zero column, or inf/NaN pivot
  const unsigned long long cand = __ballot(!used && key == mk);
  const int p = first_lane(cand ? cand : 1ull);
  const T piv = lane_bcast(a[K], p);
  if (lane == p) {
    used = true;
    stp = K;
  }
  // Branch-free update: rows already eliminated (the pivot row included) and
  // padding rows take a zero multiplier, a - 0 * u being exact for the
  // finite u of a pivot row.
  const T rp = T(1) / piv;
  const T l = used ? T(0) : a[K] * rp;
  a[K] = used ? a[K] : l;
  sfor<K + 1, NM>([&](auto j) { a[j] -= l * lane_bcast(a[j], p); });
}

// LU of the wave's NM x NM block in place (multipliers below, U on and above
// the pivot step).  The block is the N x N matrix bordered by an identity
// (rows and columns N..NM-1), so the NM - N extra steps leave the N x N
// factor unchanged; lanes NM..63 hold nothing and never pivot.  Returns false
// on a zero or non-finite pivot column.
template <int NM, typename T, int... K>
__device__ __forceinline__ bool small_lu_seq(T (&a)[NM], int lane, int& stp, std::integer_sequence<int, K...>) {
  bool used = lane >= NM, bad = false;
  stp = used ? NM : -1;
  (small_lu_step<K, NM, T>(a, lane, used, stp, bad), ...);
  return !bad;
}
template <int NM, typename T>
__device__ __forceinline__ bool small_lu(T (&a)[NM], int lane, int& stp) {
  return small_lu_seq<NM, T>(a, lane, stp, std::make_integer_sequence<int, NM>{});
}

template <int K, int NM, typename T>
__device__ __forceinline__ void small_fwd_step(const T (&a)[NM], int stp, T& b) {
  const int p = first_lane(__ballot(stp == K));
  const T yk = lane_bcast(b, p);
  if (stp > K) b -= a[K] * yk;
}
template <int K, int NM, typename T>
__device__ __forceinline__ void small_bwd_step(const T (&a)[NM], int stp, T& b, double* xv) {
  const int p = first_lane(__ballot(stp == K));
  const T xk = lane_bcast(b, p) / lane_bcast(a[K], p);
  if (stp == K) xv[K] = (double)xk;
  if (stp < K) b -= a[K] * xk;
}
template <int NM, typename T, int... K>
__device__ __forceinline__ void small_solve_seq(const T (&a)[NM], int stp, T b, double* xv,
                                                std::integer_sequence<int, K...>) {
  (small_fwd_step<K, NM, T>(a, stp, b), ...);
  (small_bwd_step<NM - 1 - K, NM, T>(a, stp, b, xv), ...);
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
}
// Solves with the factor of small_lu, in the factor's precision (for the
// FP32 factor this is the correction solve of the refinement; residual and
// solution stay FP64): b is the right-hand side entry of the lane's row
// (zero on the identity border); x_k lands in xv[k] (wave-private LDS, NM
// entries).
template <int NM, typename T>
__device__ __forceinline__ void small_solve(const T (&a)[NM], int stp, double b, double* xv) {
  small_solve_seq<NM, T>(a, stp, (T)b, xv, std::make_integer_sequence<int, NM>{});
}

// Rows of A = I - h gamma J for the SW states of a workgroup (or of the SW
// listed states when `list` is given), staged SRB rows at a time.  Returns
// the lane's row in a64 (zero beyond N) and whether it is finite.
template <int NM, int SW>
__device__ __forceinline__ bool small_load(double (&a64)[NM], int N, int64_t ld, const double* __restrict__ jac,
                                           const int64_t* sst, double hg, int lane, int wv, double* stage) {
  sfor<0, NM>([&](auto j) { a64[j] = 0.0; });
  // Each thread always serves the same state (the stride is a multiple of
  // SW) and keeps 8 independent loads in flight before its LDS stores.
  constexpr int UNR = 8, STRIDE = SW * 64;
  const int64_t myst = sst[threadIdx.x % SW];
  for (int i0 = 0; i0 < N; i0 += SRB) {
    const int rows = min(SRB, N - i0);
    const int cnt = rows * N * SW;
    const double* jb = jac + (int64_t)i0 * N * ld + (myst >= 0 ? myst : 0);
    for (int t0 = threadIdx.x; t0 < cnt; t0 += STRIDE * UNR) {
      double v[UNR];
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int t = t0 + u * STRIDE;
        v[u] = (t < cnt && myst >= 0) ? jb[(int64_t)(t / SW) * ld] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < UNR; ++u) {
        const int t = t0 + u * STRIDE;
        if (t < cnt) stage[t] = v[u];
      }
    }
    __syncthreads();
    if (lane >= i0 && lane < i0 + rows) {
      // the raw row J_i., at constant offsets; columns j >= N read other
      // staged values or the slack of SW * NM doubles after the stage
      // (the allocation is sized for it) and are replaced below
      const double* src = stage + (size_t)(lane - i0) * N * SW + wv;
      sfor8<0, NM>([&](auto j) { a64[j] = src[j * SW]; });
    }
    __syncthreads();
  }
  // a_ij = delta_ij - h gamma J_ij (one rounding) inside the N x N block,
  // identity on the border (lanes N..NM-1 start with zero rows)
  sfor<0, NM>([&](auto j) {
    const double d = lane == j ? 1.0 : 0.0;
    a64[j] = j < N ? fma(-hg, a64[j], d) : d;
  });
  bool fin = true;
  sfor<0, NM>([&](auto j) { fin = fin && isfinite(a64[j]); });
  return fin;
}

// FP64 path.  Without a list: states blockIdx.x*SW + w, info = 0 / -1 / -3.
// With a list (the mixed path's fallback): slots blockIdx.x*SW + w < *count
// name the states, info = -2 / -1.
template <int NM, int SW = kSmallWaves>
__global__ __launch_bounds__(SW * 64, 2) void small_fp64_kernel(int N, int64_t n, int64_t ld,
                                                                const double* __restrict__ jac,
                                                                const double* __restrict__ h, double gamma,
                                                                const double* __restrict__ rhs,
                                                                double* __restrict__ x, int* __restrict__ info,
                                                                const int* __restrict__ list,
                                                                const int* __restrict__ count,
                                                                double* __restrict__ fstore = nullptr,
                                                                int* __restrict__ sstore = nullptr,
                                                                int* __restrict__ fstat = nullptr, int fmode = 0) {
  // fmode 1: also store the factor (lane i's row, its pivot step) and the
  // state's factorization status; fmode 2: take them from a previous fmode-1
  // launch instead of loading J and factoring (uniform over the launch).
  // wave-private buffers first, so their offsets fit the LDS instructions'
  // immediate offset fields; the staging area follows
  extern __shared__ double slds[];
  double* xall = slds;                                     // SW * NM
  double* stage = xall + (size_t)SW * NM;                  // SRB * N * SW, then slack
  __shared__ int64_t sst[SW];                              // state of each wave, -1 if none
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  // a listed launch is sized for every state; workgroups past the listed
  // count leave before any barrier
  if (list && (int64_t)xcd_block() * SW >= *count) return;
  if (threadIdx.x < SW) {
    const int64_t lim = list ? *count : n;
    const int64_t slot = (int64_t)xcd_block() * SW + threadIdx.x;
    sst[threadIdx.x] = slot < lim ? (list ? list[slot] : slot) : -1;
  }
  __syncthreads();
  const int64_t s = sst[wv];
  const bool live = s >= 0;
  double* xv = xall + (size_t)wv * NM;
  if (lane < NM) xv[lane] = 0.0;
  const double hg = live ? h[s] * gamma : 0.0;
  double a64[NM];
  const double b = (live && lane < N) ? rhs[(int64_t)lane * ld + s] : 0.0;
  bool solved = false;
  int status;
  if (fmode == 2) {
    // stored factor: lanes NM..63 hold nothing and never pivot
    sfor<0, NM>([&](auto j) { a64[j] = 0.0; });
    int stp = NM;
    status = live ? fstat[s] : 0;
    if (live && status == 0) {
      if (lane < NM) {
        const double* fr = fstore + ((int64_t)s * NM + lane) * NM;
        sfor<0, NM>([&](auto j) { a64[j] = fr[j]; });
        stp = sstore[(int64_t)s * NM + lane];
      }
      small_solve<NM, double>(a64, stp, b, xv);
      solved = true;
      status = __all(lane >= N || isfinite(xv[lane])) ? 0 : -1;
    }
  } else {
    const bool fin = __all(small_load<NM, SW>(a64, N, ld, jac, sst, hg, lane, wv, stage));
    status = fin ? 0 : -3;
    int fst = status;
    if (live && fin) {
      int stp;
      if (small_lu<NM, double>(a64, lane, stp)) {
        if (fmode == 1 && lane < NM) {
          double* fr = fstore + ((int64_t)s * NM + lane) * NM;
          sfor<0, NM>([&](auto j) { fr[j] = a64[j]; });
          sstore[(int64_t)s * NM + lane] = stp;
        }
        small_solve<NM, double>(a64, stp, b, xv);
        solved = true;
        status = __all(lane >= N || isfinite(xv[lane])) ? (list ? -2 : 0) : -1;
      } else {
        status = -1;
        fst = -1;
      }
    }
    if (fmode == 1 && live && lane == 0) fstat[s] = fst;
  }
  if (live && lane == 0) info[s] = status;
  if (solved && lane < N) x[(int64_t)lane * ld + s] = xv[lane];
}

// States whose mixed solve left ST_UNSET or ST_SING32 go to the fallback list.
__global__ void small_compact_kernel(int64_t n, const int* __restrict__ info, int* __restrict__ list,
                                     int* __restrict__ count) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  if (info[s] == ST_UNSET || info[s] == ST_SING32) list[atomicAdd(count, 1)] = (int)s;
}

// ---------------------------------------------------------------- grouped FP32 factor
// Mixed path for N <= 64 with S states per wavefront: a group of G = 64 / S
// lanes holds one state, lane q of the group the rows q, q + G, ..., so each
// lane keeps R = S rows of NC FP32 values in registers (R * G = 64 rows).
// Halving the element width is what lets four states share a wavefront, and
// every instruction of the elimination, the triangular solves and the
// pivot search then serves S states at once.  Partial pivoting is implicit
// (rows stay in place; each row records the step at which it was the pivot),
// as in the FP64 register path.  The pivot key packs the magnitude (low six
// mantissa bits cleared) with 63 - row, so one group maximum names the pivot
// row, ties going to the lower row; the pivot row travels through LDS.  The
// residual r = b - (I - h gamma J) x is formed in FP64 from the FP64 Jacobian
// in memory at every sweep (the FP64 matrix does not fit beside the factor).
constexpr int kGrpWaves = 2;   // wavefronts per workgroup
constexpr int kGrpOcc = 2;     // wavefronts per SIMD the register budget is sized for
// LDS stage of Jacobian rows per workgroup: with the static buffers, four
// workgroups (eight wavefronts, the register limit) fit a CU's 160 KiB
constexpr int kGrpStageBytes = 32768;

// Jacobian rows per staging pass: as many whole rows of the workgroup's WS
// states as the stage holds, at most N.  Every row's residual is one dot
// product in column order, so the pass size does not change any result.
__host__ __device__ inline int grp_stage_rows(int N, int WS) {
  const int r = kGrpStageBytes / (N * WS * (int)sizeof(double));
  return r < 1 ? 1 : (r > N ? N : r);
}

template <int G>
__device__ __forceinline__ unsigned group_max_u32(unsigned v) {
  // quad_perm [1,0,3,2], quad_perm [2,3,0,1], row_half_mirror, row_mirror
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0xB1, 0xF, 0xF, false));
  v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x4E, 0xF, 0xF, false));
  if constexpr (G >= 8) v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x141, 0xF, 0xF, false));
  if constexpr (G >= 16) v = max(v, (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, 0x140, 0xF, 0xF, false));
  if constexpr (G >= 32) v = max(v, (unsigned)__shfl_xor((int)v, 16));
  if constexpr (G >= 64) v = max(v, (unsigned)__shfl_xor((int)v, 32));
  return v;
}
template <int G>
__device__ __forceinline__ double group_max_f64(double v) {
  for (int o = 1; o < G; o <<= 1) v = fmax(v, __shfl_xor(v, o));
  return v;
}

__device__ __forceinline__ void wave_lds_sync() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront"); }

// Forward and back substitution with the grouped factor (FP32), right-hand
// side b (the lane's rows, zero beyond N).  pv[K] is the pivot row of step K
// and dinv[K] the reciprocal of its pivot (both per group, in LDS, read one
// step ahead); the value of the pivot row reaches its group through
// v_readlane, so no LDS round trip sits on the dependency chain.  The
// solution lands in xo[0..N).
template <int NC, int R, int S>
__device__ __forceinline__ void grp_solve(float (&a)[R][NC], int (&stp)[R], float (&b)[R], int N, int g, int gl,
                                          const int* pv, const float* dinv, float* xo) {
  constexpr int G = 64 / S;
  // the factor is loop-invariant across sweeps; keep the compiler from
  // hoisting the masked multipliers of every step out of the sweep loop
  sfor<0, R>([&](auto r) { opaque_regs<0, NC>(a[r]); });
  opaque_regs<0, R>(stp);
  // value of the pivot row's slot, broadcast from the pivot lane of each group
  auto bcast = [&](int pr) -> float {
    const int slot = pr / G, src = pr % G;
    float v = b[0];
    sfor<1, R>([&](auto r) { v = slot == r ? b[r] : v; });
    float out = 0.0f;
    sfor<0, S>([&](auto gg) {
      const int lsrc = __builtin_amdgcn_readlane(src, gg * G) + gg * G;
      const float w = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lsrc));
      out = g == gg ? w : out;
    });
    return out;
  };
  // every step runs (identity border up to NC), so the factor stays one set
  // of registers
  int pr_next = pv[0];
  sfor<0, NC>([&](auto K) {
    const int pr = pr_next;
    if constexpr (K + 1 < NC) pr_next = pv[K + 1];
    const float y = bcast(pr);
    sfor<0, R>([&](auto r) { b[r] = fmaf(stp[r] > K ? -a[r][K] : 0.0f, y, b[r]); });
    __builtin_amdgcn_sched_barrier(0);
  });
  pr_next = pv[NC - 1];
  float di_next = dinv[NC - 1];
  sfor<0, NC>([&](auto KK) {
    constexpr int K = NC - 1 - decltype(KK)::value;
    const int pr = pr_next;
    const float di = di_next;
    if constexpr (K > 0) {
      pr_next = pv[K - 1];
      di_next = dinv[K - 1];
    }
    const float xk = bcast(pr) * di;
    if (gl == 0) xo[K] = xk;
    sfor<0, R>([&](auto r) { b[r] = fmaf(stp[r] < K ? -a[r][K] : 0.0f, xk, b[r]); });
    __builtin_amdgcn_sched_barrier(0);
  });
  wave_lds_sync();
}

// Jacobian rows [i0, i0 + rows) of the workgroup's WS states into LDS,
// stage[((i - i0) * N + j) * WS + q] = J_ij of state q; runs of WS states
// are contiguous in memory.  When the workgroup's states are all present
// and the rows 16-byte aligned (`dma`), each lane moves two neighbouring
// states of one element straight into LDS (global_load_lds, 16 bytes), so
// that the whole chunk is in flight without occupying registers; otherwise
// each thread serves one state (the block size is a multiple of WS) with 8
// loads in flight through registers.
template <int WS>
__device__ __forceinline__ void grp_stage(int N, int64_t ld, const double* __restrict__ jac, const int64_t* sst,
                                          bool dma, int i0, int rows, double* stage) {
  constexpr int STRIDE = kGrpWaves * 64, UNR = 8;
  static_assert(WS % 2 == 0, "pairs of states");
  const int cnt = rows * N * WS;
  if (dma) {
    const int wv = threadIdx.x / 64, lane = threadIdx.x % 64;
    const double* jb = jac + (int64_t)i0 * N * ld + sst[0];
    for (int tb = wv * 128; tb < cnt; tb += kGrpWaves * 128) {
      const int t = tb + 2 * lane;
      if (t < cnt) __builtin_amdgcn_global_load_lds(jb + (int64_t)(t / WS) * ld + (t % WS), stage + tb, 16, 0, 0);
    }
    __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
    return;
  }
  const int64_t myst = sst[threadIdx.x % WS];
  const double* jb = jac + (int64_t)i0 * N * ld + (myst >= 0 ? myst : 0);
  for (int t0 = threadIdx.x; t0 < cnt; t0 += STRIDE * UNR) {
    double v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int t = t0 + u * STRIDE;
      v[u] = (t < cnt && myst >= 0) ? jb[(int64_t)(t / WS) * ld] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const int t = t0 + u * STRIDE;
      if (t < cnt) stage[t] = v[u];
    }
  }
}

// Workgroup of kGrpWaves wavefronts, WS = kGrpWaves * S states.  info: sweep
// count, ST_SING32 (zero or non-finite FP32 pivot column), ST_UNSET (no
// convergence within max_refine sweeps) or -3 (non-finite input); the last
// three are left for the FP64 fallback.  Dynamic LDS: the stage of srb
// Jacobian rows (grp_lds_bytes).
template <int NC, int S>
__global__ __launch_bounds__(kGrpWaves * 64, kGrpOcc) void grp_mixed_kernel(int N, int64_t n, int64_t ld,
                                                                    const double* __restrict__ jac,
                                                                    const double* __restrict__ h, double gamma,
                                                                    const double* __restrict__ rhs,
                                                                    double* __restrict__ x, int* __restrict__ info,
                                                                    int max_refine, double rtol) {
  constexpr int G = 64 / S, R = S, WS = kGrpWaves * S;
  const int srb = grp_stage_rows(N, WS);
  static_assert(NC % 4 == 0 && NC <= 64, "column count");
  extern __shared__ double stage[];                        // srb * N * WS
  __shared__ __align__(16) float pbuf[kGrpWaves][S][NC];   // pivot row of the current step
  __shared__ int pvbuf[kGrpWaves][S][64];                  // pivot row of each step
  __shared__ float obuf[kGrpWaves][S][64];                 // FP32 solutions
  __shared__ float dbuf[kGrpWaves][S][64];                 // pivot reciprocals
  __shared__ __align__(16) double xbuf[kGrpWaves][S][64];  // FP64 solution
  __shared__ int64_t sst[WS];                              // state of each group, -1 if none
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int g = lane / G, gl = lane % G, q = wv * S + g;
  if (threadIdx.x < WS) {
    const int64_t slot = (int64_t)xcd_block() * WS + threadIdx.x;
    sst[threadIdx.x] = slot < n ? slot : -1;
  }
  __syncthreads();
  const int64_t s = sst[q];
  const bool live = s >= 0;
  const int64_t sc = live ? s : 0;
  const double hg = live ? h[sc] * gamma : 0.0;
  // all WS states present (consecutive), element rows 16-byte aligned
  const bool dma = sst[WS - 1] >= 0 && (ld % 2) == 0 && ((uintptr_t)jac % 16) == 0;
  float* pb = pbuf[wv][g];
  int* pvb = pvbuf[wv][g];
  float* ob = obuf[wv][g];
  float* db = dbuf[wv][g];
  double* xb = xbuf[wv][g];

  // A = I - h gamma J in FP32, the lane's rows.  Rows and columns N..NC-1
  // form an identity border (so every elimination step runs); rows >= NC
  // are empty and count as already eliminated.
  float a[R][NC];
  bool used[R];
  int stp[R];
  bool fin = true;
  sfor<0, R>([&](auto r) {
    const int i = r * G + gl;
    used[r] = !(live && i < NC);
    stp[r] = used[r] ? 64 : -1;
    sfor<0, NC>([&](auto j) { a[r][j] = (!used[r] && i >= N && i == j) ? 1.0f : 0.0f; });
  });
  for (int i0 = 0; i0 < N; i0 += srb) {
    const int rows = min(srb, N - i0);
    grp_stage<WS>(N, ld, jac, sst, dma, i0, rows, stage);
    __syncthreads();
    sfor<0, R>([&](auto r) {
      const int i = r * G + gl;
      if (!used[r] && i < N && i >= i0 && i < i0 + rows) {
        const double* src = stage + (size_t)(i - i0) * N * WS + q;
        sfor8<0, NC>([&](auto j) {
          if (j < N) {
            const double v = fma(-hg, src[j * WS], i == j ? 1.0 : 0.0);
            fin = fin && isfinite(v);
            a[r][j] = (float)v;
          }
        });
      }
    });
    __syncthreads();
  }
  // a state is finite only if all its rows are
  const bool gfin = group_max_u32<G>(fin ? 0u : 1u) == 0u;
  bool bad = !gfin;

  // elimination: every step runs (the identity border makes steps N..NC-1
  // pick rows N..NC-1), so the factor stays one set of registers
  sfor<0, NC>([&](auto K) {
    {
      unsigned best = 0u;
      sfor<0, R>([&](auto r) {
        const unsigned mag = (unsigned)__float_as_int(a[r][K]) & 0x7FFFFFFFu;
        const unsigned key = used[r] ? 0u : ((mag & ~63u) | (unsigned)(63 - (r * G + gl)));
        best = max(best, key);
      });
      const unsigned mk = group_max_u32<G>(best);
      bad = bad || (mk >> 6) == 0u || (mk & ~63u) >= 0x7F800000u;
      const int prow = 63 - (int)(mk & 63u);
      constexpr int K4 = (decltype(K)::value) & ~3;
      sfor<0, R>([&](auto r) {
        if (!used[r] && r * G + gl == prow) {
          used[r] = true;
          stp[r] = K;
          sfor<K4 / 4, NC / 4>([&](auto c4) {
            *reinterpret_cast<float4*>(pb + 4 * c4) =
                make_float4(a[r][4 * c4], a[r][4 * c4 + 1], a[r][4 * c4 + 2], a[r][4 * c4 + 3]);
          });
        }
      });
      wave_lds_sync();
      const float rp = __builtin_amdgcn_rcpf(pb[K]);
      if (gl == 0) {
        db[K] = rp;
        pvb[K] = prow;
      }
      float l[R];
      sfor<0, R>([&](auto r) {
        l[r] = used[r] ? 0.0f : a[r][K] * rp;
        a[r][K] = used[r] ? a[r][K] : l[r];
      });
      sfor<K4 / 4, NC / 4>([&](auto c4) {
        const float4 u = *reinterpret_cast<const float4*>(pb + 4 * c4);
        const float uu[4] = {u.x, u.y, u.z, u.w};
        sfor<0, 4>([&](auto c) {
          constexpr int j = 4 * decltype(c4)::value + decltype(c)::value;
          if constexpr (j > decltype(K)::value)
            sfor<0, R>([&](auto r) { a[r][j] = fmaf(-l[r], uu[c], a[r][j]); });
        });
        __builtin_amdgcn_sched_barrier(0);
      });
      wave_lds_sync();
    }
    __builtin_amdgcn_sched_barrier(0);
  });
  bad = bad || !live;

  int status = gfin ? ST_UNSET : -3;
  if (gfin && bad) status = live ? ST_SING32 : 0;
  double bd[R];
  sfor<0, R>([&](auto r) {
    const int i = r * G + gl;
    bd[r] = (live && i < N) ? rhs[(int64_t)i * ld + s] : 0.0;
  });
  // sweep 0: x = A32^-1 b; then FP64 residual, FP32 correction, until the
  // correction is below rtol of the solution (max norms) or max_refine sweeps
  {
    float b[R];
    sfor<0, R>([&](auto r) { b[r] = bad ? 0.0f : (float)bd[r]; });
    grp_solve<NC, R, S>(a, stp, b, N, g, gl, pvb, db, ob);
    if (!bad)
      for (int k = gl; k < N; k += G) xb[k] = (double)ob[k];
    wave_lds_sync();
  }
  bool done = bad;
  double dprev = 0.0;                             // the previous sweep's correction (max norm)
  for (int sweep = 1; sweep <= max_refine; ++sweep) {
    if (!__syncthreads_or(!done)) break;          // uniform over the workgroup (it stages together)
    float c[R];
    sfor<0, R>([&](auto r) { c[r] = 0.0f; });
    for (int i0 = 0; i0 < N; i0 += srb) {
      const int rows = min(srb, N - i0);
      grp_stage<WS>(N, ld, jac, sst, dma, i0, rows, stage);
      __syncthreads();
      sfor<0, R>([&](auto r) {
        const int i = r * G + gl;
        if (!done && i >= i0 && i < i0 + rows) {
          const double* src = stage + (size_t)(i - i0) * N * WS + q;
          double acc = 0.0;
#pragma unroll 4
          for (int j = 0; j < N; ++j) acc = fma(src[j * WS], xb[j], acc);
          c[r] = (float)(bd[r] - (xb[i] - hg * acc));
        }
      });
      __syncthreads();
    }
    grp_solve<NC, R, S>(a, stp, c, N, g, gl, pvb, db, ob);
    double dm = 0.0, xm = 0.0;
    bool xf = true;
    if (!done)
      for (int k = gl; k < N; k += G) {
        const double d = (double)ob[k];
        const double xn = xb[k] + d;
        xb[k] = xn;
        dm = fmax(dm, fabs(d));
        xm = fmax(xm, fabs(xn));
        xf = xf && isfinite(xn);
      }
    wave_lds_sync();
    dm = group_max_f64<G>(dm);
    xm = group_max_f64<G>(xm);
    const bool gxf = group_max_u32<G>(xf ? 0u : 1u) == 0u;
    // converged when the correction is below rtol of the solution, or when
    // the contraction rho of the last two corrections (refinement converges
    // linearly) predicts the remaining error rho / (1 - rho) |d| below it
    const double rho = (sweep >= 2 && dprev > 0.0) ? dm / dprev : 1.0;
    const bool conv = dm <= rtol * xm || (rho < 0.5 && rho * dm <= rtol * xm * (1.0 - rho));
    if (!done && gxf && conv) {
      status = sweep;
      done = true;
    }
    dprev = dm;
  }
  if (live && gl == 0) info[s] = status;
  if (live && status > 0)
    sfor<0, R>([&](auto r) {
      const int i = r * G + gl;
      if (i < N) x[(int64_t)i * ld + s] = xb[i];
    });
}

// stage of grp_stage_rows Jacobian rows
size_t grp_lds_bytes(int N, int S) {
  const size_t WS = (size_t)kGrpWaves * S;
  return (size_t)grp_stage_rows(N, (int)WS) * N * WS * sizeof(double);
}

// the SW x NM solution buffer + the stage + SW x NM slack for the reads
// past the last staged row
size_t small_lds(int N, int NM, int SW) { return ((size_t)SRB * N * SW + 2 * (size_t)SW * NM) * sizeof(double); }

template <int NM>
hipError_t launch_small_t(int N, int64_t n, int64_t ld, const double* jac, const double* h, double gamma,
                          const double* rhs, double* x, int* info, int mode, int max_refine, double rtol,
                          int* list, int* count, hipStream_t st, void* fws, int fmode) {
  const size_t lds = small_lds(N, NM, kSmallWaves);
  const unsigned grid = (unsigned)((n + kSmallWaves - 1) / kSmallWaves);
  auto k64 = small_fp64_kernel<NM>;
  hipError_t e = hipFuncSetAttribute((const void*)k64, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  if (mode == 0) {
    // kept factor: [state][row][NM] doubles, then [state][NM] pivot steps, then [state] status
    auto al = [](size_t b) { return (b + 255) & ~size_t(255); };
    char* fw = static_cast<char*>(fws);
    double* fstore = fws ? reinterpret_cast<double*>(fw) : nullptr;
    int* sstore = fws ? reinterpret_cast<int*>(fw + al((size_t)n * NM * NM * sizeof(double))) : nullptr;
    int* fstat = fws ? reinterpret_cast<int*>(fw + al((size_t)n * NM * NM * sizeof(double)) +
                                              al((size_t)n * NM * sizeof(int)))
                     : nullptr;
    hipLaunchKernelGGL(k64, dim3(grid), dim3(kSmallWaves * 64), lds, st, N, n, ld, jac, h, gamma, rhs, x, info,
                       (const int*)nullptr, (const int*)nullptr, fstore, sstore, fstat, fws ? fmode : 0);
    return hipGetLastError();
  }
  // mixed: grouped FP32 factor, S states per wavefront (4 up to 16 columns,
  // 2 above: S * NC FP32 values per lane stay within the register budget of
  // two wavefronts per SIMD without spills)
  // (the 32-column instance spills at two states per wavefront, so those
  // sizes take the 48-column one)
  constexpr int NC = NM == 32 ? 48 : NM;
  constexpr int S = NC <= 16 ? 4 : 2;
  constexpr int per_block = kGrpWaves * S;
  const size_t glds = grp_lds_bytes(N, S);
  auto kg = grp_mixed_kernel<NC, S>;
  e = hipFuncSetAttribute((const void*)kg, hipFuncAttributeMaxDynamicSharedMemorySize, (int)glds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kg, dim3((unsigned)((n + per_block - 1) / per_block)), dim3(kGrpWaves * 64), glds, st, N, n,
                     ld, jac, h, gamma, rhs, x, info, max_refine, rtol);
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, st, count);
  hipLaunchKernelGGL(small_compact_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                     (const int*)info, list, count);
  hipLaunchKernelGGL(k64, dim3(grid), dim3(kSmallWaves * 64), lds, st, N, n, ld, jac, h, gamma, rhs, x, info,
                     (const int*)list, (const int*)count, (double*)nullptr, (int*)nullptr, (int*)nullptr, 0);
  return hipGetLastError();
}

hipError_t launch_small(int N, int64_t n, int64_t ld, const double* jac, const double* h, double gamma,
                        const double* rhs, double* x, int* info, int mode, int max_refine, double rtol,
                        int* list, int* count, hipStream_t st, void* fws, int fmode) {
  // register width: N rounded up to 16, 32, 48, 56 or 64 (the work per
  // state grows as NM^2, so the identity border is kept narrow where the
  // workloads sit; fewer widths keep the build short)
#define PYJAC_SMALL(nm) \
  if (small_width(N) == nm) return launch_small_t<nm>(N, n, ld, jac, h, gamma, rhs, x, info, mode, max_refine, rtol, list, count, st, fws, fmode);
  PYJAC_SMALL(16)
  PYJAC_SMALL(32)
  PYJAC_SMALL(48)
  PYJAC_SMALL(56)
  PYJAC_SMALL(64)
#undef PYJAC_SMALL
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------- solve
// One wavefront per (listed) state, 4 states per 256-thread block; waves
// without work stay in the block and only skip the memory operations, so
// every barrier is reached by all four.
// direct: x = A^-1 b, b from rhs [N][ld], x to xout [N][ld].
// refine: d = A^-1 r with r from rbuf [N][n]; x += d in xs [N][n] (FP64) and
//   the state converges at this sweep when ||d||_inf <= rtol ||x||_inf.
template <typename T, bool REFINE>
__global__ __launch_bounds__(256) void solve_kernel(int N, int64_t n, int64_t ld, const T* __restrict__ Aall,
                                                    const int* __restrict__ pivall, const double* __restrict__ rhs,
                                                    const double* __restrict__ rbuf, double* __restrict__ xs,
                                                    double* __restrict__ xout, const int* __restrict__ list,
                                                    const int* __restrict__ count, int* __restrict__ status,
                                                    int sweep, double rtol, double* __restrict__ dprev) {
  extern __shared__ char smem[];
  const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
  const int64_t slot = (int64_t)blockIdx.x * 4 + wv;
  const int64_t lim = count ? *count : n;
  bool active = slot < lim;
  const int64_t st = active ? (list ? list[slot] : slot) : 0;
  const int s0 = active ? status[st] : 0;
  active = active && (REFINE ? s0 == ST_UNSET : (s0 != -3 && s0 != -1 && s0 != ST_SING32));
  T* y = reinterpret_cast<T*>(smem) + (size_t)wv * N;
  const T* A = Aall + (active ? slot : 0) * (int64_t)N * N;
  const int* piv = pivall + (active ? slot : 0) * (int64_t)N;
  if (active)
    for (int i = lane; i < N; i += 64) y[i] = REFINE ? (T)rbuf[(int64_t)i * n + st] : (T)rhs[(int64_t)i * ld + st];
  __syncthreads();
  if (active && lane == 0)
    for (int i = 0; i < N; ++i) {
      const int p = piv[i];
      if (p != i) { T t = y[i]; y[i] = y[p]; y[p] = t; }
    }
  __syncthreads();
  for (int i = 1; i < N; ++i) {            // unit lower
    T acc = T(0);
    if (active)
      for (int j = lane; j < i; j += 64) acc += A[(int64_t)i * N + j] * y[j];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (active && lane == 0) y[i] -= acc;
    __syncthreads();
  }
  for (int i = N - 1; i >= 0; --i) {       // upper
    T acc = T(0);
    if (active)
      for (int j = i + 1 + lane; j < N; j += 64) acc += A[(int64_t)i * N + j] * y[j];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    if (active && lane == 0) y[i] = (y[i] - acc) / A[(int64_t)i * N + i];
    __syncthreads();
  }
  if (!active) return;
  if (!REFINE) {
    bool fin = true;
    for (int i = lane; i < N; i += 64) {
      xout[(int64_t)i * ld + st] = (double)y[i];
      fin = fin && isfinite((double)y[i]);
    }
    fin = __all(fin);
    if (lane == 0 && s0 == ST_UNSET) status[st] = fin ? 0 : -1;
    return;
  }
  double dmax = 0.0, xmax = 0.0;
  bool fin = true;
  for (int i = lane; i < N; i += 64) {
    const double d = (double)y[i];
    const double xv = xs[(int64_t)i * n + st] + d;
    xs[(int64_t)i * n + st] = xv;
    dmax = fmax(dmax, fabs(d));
    xmax = fmax(xmax, fabs(xv));
    fin = fin && isfinite(xv);
  }
  for (int o = 32; o > 0; o >>= 1) {
    dmax = fmax(dmax, __shfl_xor(dmax, o));
    xmax = fmax(xmax, __shfl_xor(xmax, o));
  }
  fin = __all(fin);
  if (lane == 0 && sweep > 0) {
    // converged when the correction is below rtol of the solution, or when
    // the contraction rho of the last two corrections (refinement converges
    // linearly) predicts the remaining error rho / (1 - rho) |d| below it
    const double dp = sweep >= 2 ? dprev[st] : 0.0;
    const double rho = dp > 0.0 ? dmax / dp : 1.0;
    if (fin && (dmax <= rtol * xmax || (rho < 0.5 && rho * dmax <= rtol * xmax * (1.0 - rho)))) status[st] = sweep;
    dprev[st] = dmax;
  }
}

// r = b - (I - h gamma J) x in FP64.  grid (ceil(n / 256), ceil(N / 8)): one
// thread per (state, block of 8 rows), so that a few thousand states still
// fill the device; each x_j load serves 8 multiply-adds and every load is
// coalesced across the states of a wavefront.  Converged states are skipped.
constexpr int kResRows = 8;
__global__ __launch_bounds__(256) void residual_kernel(int N, int64_t n, int64_t ld, const double* __restrict__ jac,
                                                       const double* __restrict__ h, double gamma,
                                                       const double* __restrict__ rhs, const double* __restrict__ xs,
                                                       double* __restrict__ rbuf, const int* __restrict__ status) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n || status[s] != ST_UNSET) return;
  const double hg = h[s] * gamma;
  constexpr int IB = kResRows;
  {
    const int i0 = blockIdx.y * IB;
    double acc[IB];
#pragma unroll
    for (int u = 0; u < IB; ++u) acc[u] = 0.0;
    for (int j = 0; j < N; ++j) {
      const double xj = xs[(int64_t)j * n + s];
#pragma unroll
      for (int u = 0; u < IB; ++u)
        if (i0 + u < N) acc[u] += jac[((int64_t)(i0 + u) * N + j) * ld + s] * xj;
    }
#pragma unroll
    for (int u = 0; u < IB; ++u) {
      const int i = i0 + u;
      if (i < N) rbuf[(int64_t)i * n + s] = rhs[(int64_t)i * ld + s] - (xs[(int64_t)i * n + s] - hg * acc[u]);
    }
  }
}

__global__ void init_status_kernel(int64_t n, int* __restrict__ status, double* __restrict__ xs, int N) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  status[s] = ST_UNSET;
  if (xs)
    for (int i = 0; i < N; ++i) xs[(int64_t)i * n + s] = 0.0;
}

// dst[s] = src[s]: keeps the status left by a factorization (singular
// states) for later calls that reuse the factor
__global__ void copy_status_kernel(int64_t n, const int* __restrict__ src, int* __restrict__ dst) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s < n) dst[s] = src[s];
}

__global__ void copy_rhs_kernel(int N, int64_t n, int64_t ld, const double* __restrict__ rhs, double* __restrict__ rbuf) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  for (int i = 0; i < N; ++i) rbuf[(int64_t)i * n + s] = rhs[(int64_t)i * ld + s];
}

// States that did not converge (status still unset) go to the FP64 list.
// The list order depends on scheduling; each listed state is solved on its
// own, so results do not depend on that order.
__global__ void compact_kernel(int64_t n, const int* __restrict__ status, int* __restrict__ list, int* __restrict__ count) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  if (status[s] == ST_UNSET || status[s] == ST_SING32) {
    const int at = atomicAdd(count, 1);
    list[at] = (int)s;
  }
}

__global__ void finish_kernel(int N, int64_t n, int64_t ld, const int* __restrict__ status,
                              const double* __restrict__ xs, double* __restrict__ xout, int* __restrict__ info,
                              const int* __restrict__ fb_status, int mode) {
  const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
  int st = status[s];
  if (mode == 1) {
    if (st >= 0 && xs)
      for (int i = 0; i < N; ++i) xout[(int64_t)i * ld + s] = xs[(int64_t)i * n + s];
    if (st == ST_UNSET || st == ST_SING32) st = (fb_status[s] == 0) ? -2 : fb_status[s];   // FP64 re-solve
  }
  info[s] = st;
}


size_t align256(size_t b) { return (b + 255) & ~size_t(255); }
size_t small_ws_bytes(int64_t n, int mode) { return mode == 1 ? align256((size_t)n * sizeof(int)) + 256 : 0; }

// FP64 factor kept for reuse on the register path (mode 0): rows of NM
// doubles, NM pivot steps and one status per state
size_t small_keep_bytes(int N, int64_t n) {
  const size_t NM = (size_t)small_width(N);
  return align256((size_t)n * NM * NM * sizeof(double)) + align256((size_t)n * NM * sizeof(int)) +
         align256((size_t)n * sizeof(int));
}

struct WsLayout {
  size_t a32 = 0, a64 = 0, piv = 0, piv64 = 0, sing = 0, status = 0, fbstatus = 0, xs = 0, rbuf = 0, list = 0,
         count = 0, dprev = 0, total = 0;
};

WsLayout ws_layout(int N, int64_t n, int mode) {
  WsLayout L;
  size_t off = 0;
  const size_t NN = (size_t)N * N;
  auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
  if (mode == 1) L.a32 = take((size_t)n * NN * sizeof(float));
  L.a64 = take((size_t)n * NN * sizeof(double));
  L.piv = take((size_t)n * N * sizeof(int));
  L.piv64 = mode == 1 ? take((size_t)n * N * sizeof(int)) : L.piv;   // the FP64 fallback's own pivots
  L.sing = take((size_t)n * sizeof(int));                              // status after factorization
  L.status = take((size_t)n * sizeof(int));
  L.fbstatus = take((size_t)n * sizeof(int));
  if (mode == 1) {
    L.xs = take((size_t)n * N * sizeof(double));
    L.rbuf = take((size_t)n * N * sizeof(double));
    L.list = take((size_t)n * sizeof(int));
    L.count = take(sizeof(int));
    L.dprev = take((size_t)n * sizeof(double));     // previous sweep's correction per state
  }
  L.total = off;
  return L;
}

size_t lu_lds(int N, size_t elem) { return ((size_t)N * (NB + 1) + (size_t)NB * (N + 1) + LU_THREADS) * elem + LU_THREADS * sizeof(int); }

template <typename T>
hipError_t run_direct(int N, int64_t n, int64_t ld, const double* jac, const double* h, double gamma,
                      const double* rhs, double* x, T* A, int* piv, const int* list, const int* count, int* status,
                      hipStream_t st, bool factor = true, int* save_status = nullptr) {
  if (factor) {
    dim3 fg((unsigned)((n + 15) / 16), (unsigned)(((int64_t)N * N + 63) / 64));
    hipLaunchKernelGGL(form_kernel<T>, fg, dim3(256), 0, st, N, n, ld, jac, h, gamma, A, list, count, status);
    const size_t lds = lu_lds(N, sizeof(T));
    hipError_t e = hipFuncSetAttribute((const void*)lu_kernel<T>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lu_kernel<T>, dim3((unsigned)n), dim3(LU_THREADS), lds, st, N, n, A, piv, list, count, status, -1);
    if (save_status)
      hipLaunchKernelGGL(copy_status_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, n,
                         (const int*)status, save_status);
  }
  hipLaunchKernelGGL((solve_kernel<T, false>), dim3((unsigned)((n + 3) / 4)), dim3(256), 4 * N * sizeof(T), st, N, n, ld,
                     (const T*)A, (const int*)piv, rhs, (const double*)nullptr, (double*)nullptr, x, list, count, status, 0,
                     0.0, (double*)nullptr);
  return hipGetLastError();
}

// Scratch for the no-allocation entry point: a file-scope device array, one
// copy per GPU, alive until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in symbol): the
// device address of each GPU's copy is looked up once with the device current
// and kept per device.
constexpr size_t kStaticScratchBytes = PYJAC_NEWTON_STATIC_SCRATCH_BYTES;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (looked up on the first
// call per device); NULL with the error recorded on failure.
void* scratch_for_device(int dev) {
  if (dev < 0 || dev >= kMaxDevices) {
    fail(PYJAC_E_DEVICE, "device ordinal outside the scratch table");
    return nullptr;
  }
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      fail(PYJAC_E_DEVICE, std::string("hipGetSymbolAddress(scratch) failed: ") + hipGetErrorString(e));
      return nullptr;
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace pyjac

using namespace pyjac;

extern "C" {

pyjac_status pyjac_newton_factor_solve_noalloc(const pyjac_mech* m, int64_t n, int64_t ld, const double* jac,
                                               const double* h, double gamma, const double* rhs, double* x,
                                               int32_t mode, int32_t max_refine, double rtol, int32_t* info,
                                               void* stream) {
  if (!m) return fail(PYJAC_E_INVALID, "mechanism handle is NULL");
  if (mode != 0 && mode != 1)
    return fail(PYJAC_E_INVALID, "mode must be 0 or 1 (the factor-keeping flags are not accepted here)");
  if (n < 0 || ld < n) return fail(PYJAC_E_INVALID, "bad n_states / ld");
  if (n == 0) return PYJAC_OK;
  const size_t need = pyjac_newton_workspace_bytes(m, n, mode);
  if (need > kStaticScratchBytes)
    return fail(PYJAC_E_WORKSPACE, "n_states needs " + std::to_string(need) +
                                       " bytes of scratch; the static scratch holds " +
                                       std::to_string(kStaticScratchBytes) +
                                       " (use pyjac_newton_factor_solve with a workspace)");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != mech_device(m))
    return fail(PYJAC_E_INVALID, "current HIP device differs from the mechanism's device");
  void* ptr = scratch_for_device(cur);
  if (!ptr) return PYJAC_E_DEVICE;
  // the kernels clear the counters they use (no memset), so the contents a
  // previous call left in the array do not matter
  return pyjac_newton_factor_solve(m, n, ld, jac, h, gamma, rhs, x, mode, max_refine, rtol, info, ptr,
                                   kStaticScratchBytes, stream);
}

size_t pyjac_newton_workspace_bytes(const pyjac_mech* m, int64_t n, int32_t mode) {
  const bool keep = (mode & PYJAC_NEWTON_KEEP_FACTOR) != 0;
  mode &= ~(PYJAC_NEWTON_REUSE_FACTOR | PYJAC_NEWTON_KEEP_FACTOR);
  if (!m || n < 0 || (mode != 0 && mode != 1)) return 0;
  if (mech_species(m) <= kSmallMax)
    return (keep && mode == 0) ? small_keep_bytes(mech_species(m), n) : small_ws_bytes(n, mode);
  return ws_layout(mech_species(m), n, mode).total;
}

pyjac_status pyjac_newton_factor_solve(const pyjac_mech* m, int64_t n, int64_t ld, const double* jac, const double* h,
                                       double gamma, const double* rhs, double* x, int32_t mode, int32_t max_refine,
                                       double rtol, int32_t* info, void* workspace, size_t workspace_bytes,
                                       void* stream) {
  if (!m) return fail(PYJAC_E_INVALID, "mechanism handle is NULL");
  if (n < 0 || ld < n) return fail(PYJAC_E_INVALID, "bad n_states / ld");
  const bool reuse = (mode & PYJAC_NEWTON_REUSE_FACTOR) != 0;
  const bool keep = (mode & PYJAC_NEWTON_KEEP_FACTOR) != 0;
  mode &= ~(PYJAC_NEWTON_REUSE_FACTOR | PYJAC_NEWTON_KEEP_FACTOR);
  if (mode != 0 && mode != 1) return fail(PYJAC_E_INVALID, "mode must be 0 or 1 (optionally | PYJAC_NEWTON_REUSE_FACTOR)");
  if (mode == 1 && (max_refine < 1 || max_refine > 100 || !(rtol > 0))) return fail(PYJAC_E_INVALID, "bad max_refine / rtol");
  if (n == 0) return PYJAC_OK;
  if (!jac || !h || !rhs || !x || !info) return fail(PYJAC_E_INVALID, "NULL array argument");
  for (const void* q : {(const void*)jac, (const void*)h, (const void*)rhs, (const void*)x})
    if (reinterpret_cast<uintptr_t>(q) & 7u) return fail(PYJAC_E_INVALID, "pointer not 8-byte aligned");
  if (x == rhs || x == jac) return fail(PYJAC_E_INVALID, "x may not alias rhs or jac");
  if (n > (int64_t)1 << 30) return fail(PYJAC_E_INVALID, "n_states too large");
  int cur = -1;
  if (hipGetDevice(&cur) != hipSuccess || cur != mech_device(m))
    return fail(PYJAC_E_INVALID, "current HIP device differs from the mechanism's device");
  const int N = mech_species(m);
  hipStream_t st = static_cast<hipStream_t>(stream);
  if (N <= kSmallMax) {     // register-resident path; mixed mode needs only the fallback list
    // FP64 with a kept factor: the workspace holds it; mixed mode factors every call
    const bool kept = mode == 0 && (keep || reuse);
    const size_t need = kept ? small_keep_bytes(N, n) : small_ws_bytes(n, mode);
    if (need && (!workspace || workspace_bytes < need))
      return fail(PYJAC_E_WORKSPACE, "workspace smaller than pyjac_newton_workspace_bytes");
    int* list = (need && !kept) ? reinterpret_cast<int*>(workspace) : nullptr;
    int* count = (need && !kept)
                     ? reinterpret_cast<int*>(static_cast<char*>(workspace) + align256((size_t)n * sizeof(int)))
                     : nullptr;
    const hipError_t e = launch_small(N, n, ld, jac, h, gamma, rhs, x, info, mode, max_refine, rtol, list, count, st,
                                      kept ? workspace : nullptr, reuse ? 2 : 1);
    if (e != hipSuccess) return fail(PYJAC_E_DEVICE, std::string("newton launch failed: ") + hipGetErrorString(e));
    return PYJAC_OK;
  }
  const WsLayout L = ws_layout(N, n, mode);
  if (!workspace || workspace_bytes < L.total) return fail(PYJAC_E_WORKSPACE, "workspace smaller than pyjac_newton_workspace_bytes");
  if (lu_lds(N, sizeof(double)) > 163840) return fail(PYJAC_E_UNSUPPORTED, "mechanism too large for the LU kernel");
  char* w = static_cast<char*>(workspace);
  int* status = reinterpret_cast<int*>(w + L.status);
  int* fbs = reinterpret_cast<int*>(w + L.fbstatus);
  int* piv = reinterpret_cast<int*>(w + L.piv);
  int* piv64 = reinterpret_cast<int*>(w + L.piv64);
  int* sing = reinterpret_cast<int*>(w + L.sing);
  double* A64 = reinterpret_cast<double*>(w + L.a64);
  const unsigned g1 = (unsigned)((n + 255) / 256);
  hipError_t e;
  // With PYJAC_NEWTON_REUSE_FACTOR the factor (and the status it left) is the
  // one a previous call with the same J, h, gamma, n, ld and mode stored in
  // this workspace; form and factorization are skipped.
  if (mode == 0) {
    if (reuse)
      hipLaunchKernelGGL(copy_status_kernel, dim3(g1), dim3(256), 0, st, n, (const int*)sing, status);
    else
      hipLaunchKernelGGL(init_status_kernel, dim3(g1), dim3(256), 0, st, n, status, (double*)nullptr, N);
    e = run_direct<double>(N, n, ld, jac, h, gamma, rhs, x, A64, piv, nullptr, nullptr, status, st, !reuse, sing);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(finish_kernel, dim3(g1), dim3(256), 0, st, N, n, ld, (const int*)status, (const double*)nullptr,
                         x, info, (const int*)nullptr, 0);
      e = hipGetLastError();
    }
  } else {
    float* A32 = reinterpret_cast<float*>(w + L.a32);
    double* xs = reinterpret_cast<double*>(w + L.xs);
    double* rbuf = reinterpret_cast<double*>(w + L.rbuf);
    int* list = reinterpret_cast<int*>(w + L.list);
    int* count = reinterpret_cast<int*>(w + L.count);
    double* dprev = reinterpret_cast<double*>(w + L.dprev);
    hipLaunchKernelGGL(init_status_kernel, dim3(g1), dim3(256), 0, st, n, status, xs, N);
    if (reuse) hipLaunchKernelGGL(copy_status_kernel, dim3(g1), dim3(256), 0, st, n, (const int*)sing, status);
    hipLaunchKernelGGL(copy_rhs_kernel, dim3(g1), dim3(256), 0, st, N, n, ld, rhs, rbuf);
    if (!reuse) {
      dim3 fg((unsigned)((n + 15) / 16), (unsigned)(((int64_t)N * N + 63) / 64));
      hipLaunchKernelGGL(form_kernel<float>, fg, dim3(256), 0, st, N, n, ld, jac, h, gamma, A32, (const int*)nullptr,
                         (const int*)nullptr, status);
      const size_t lds = lu_lds(N, sizeof(float));
      e = hipFuncSetAttribute((const void*)lu_kernel<float>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      if (e != hipSuccess) return fail(PYJAC_E_DEVICE, hipGetErrorString(e));
      hipLaunchKernelGGL(lu_kernel<float>, dim3((unsigned)n), dim3(LU_THREADS), lds, st, N, n, A32, piv,
                         (const int*)nullptr, (const int*)nullptr, status, ST_SING32);
      hipLaunchKernelGGL(copy_status_kernel, dim3(g1), dim3(256), 0, st, n, (const int*)status, sing);
    }
    const unsigned gs = (unsigned)((n + 3) / 4);
    for (int sweep = 0; sweep <= max_refine; ++sweep) {
      if (sweep > 0)
        hipLaunchKernelGGL(residual_kernel, dim3(g1, (unsigned)((N + kResRows - 1) / kResRows)), dim3(256), 0, st, N,
                           n, ld, jac, h, gamma, rhs, (const double*)xs,
                           rbuf, (const int*)status);
      hipLaunchKernelGGL((solve_kernel<float, true>), dim3(gs), dim3(256), 4 * N * sizeof(float), st, N, n, ld,
                         (const float*)A32, (const int*)piv, (const double*)nullptr, (const double*)rbuf, xs,
                         (double*)nullptr, (const int*)nullptr, (const int*)nullptr, status, sweep, rtol, dprev);
    }
    // FP64 re-solve of the states that did not converge (or whose FP32 factor was singular)
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, st, count);
    hipLaunchKernelGGL(compact_kernel, dim3(g1), dim3(256), 0, st, n, (const int*)status, list, count);
    hipLaunchKernelGGL(init_status_kernel, dim3(g1), dim3(256), 0, st, n, fbs, (double*)nullptr, N);
    // (always factored: which states fall back depends on the right-hand side)
    e = run_direct<double>(N, n, ld, jac, h, gamma, rhs, x, A64, piv64, list, count, fbs, st);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(finish_kernel, dim3(g1), dim3(256), 0, st, N, n, ld, (const int*)status, (const double*)xs, x,
                         info, (const int*)fbs, 1);
      e = hipGetLastError();
    }
  }
  if (e != hipSuccess) return fail(PYJAC_E_DEVICE, std::string("newton launch failed: ") + hipGetErrorString(e));
  return PYJAC_OK;
}

}  // extern "C"
