// Complex-step Jacobian of the constant-pressure RHS on the GPU: column j of
// J for state s is Im f(Phi + i h e_j) / h, with f the RHS of Sec. 2.1
// (Eqs. ode, dTdt) and the rate laws of Sec. 2.3 evaluated in complex
// arithmetic.  It is an accuracy reference of the kind the paper's validation
// discusses (Sec. 5.1): exact to rounding for any step h, since no difference
// of nearby values is taken.
//
// One thread per (state, column) pair, the state index fastest, so phi reads
// and Jacobian writes are coalesced and neighbouring lanes walk the same
// reaction records.  Per-thread arrays (concentrations, B_k, production rates)
// live in private memory; this is a comparison method, not the product path.
// Branch decisions (NASA range, PLOG bracket, sign of P_r) use real parts.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <string>

#include "tables.hpp"

namespace pyjac {
namespace {

constexpr double kRg = kGasConstant;
constexpr double kLn10c = 2.302585092994045684;

struct cd {
  double re, im;
};
__device__ inline cd mk(double r, double i = 0.0) { return cd{r, i}; }
__device__ inline cd operator+(cd a, cd b) { return cd{a.re + b.re, a.im + b.im}; }
__device__ inline cd operator-(cd a, cd b) { return cd{a.re - b.re, a.im - b.im}; }
__device__ inline cd operator-(cd a) { return cd{-a.re, -a.im}; }
__device__ inline cd operator*(cd a, cd b) { return cd{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cd operator*(double s, cd a) { return cd{s * a.re, s * a.im}; }
__device__ inline cd operator+(double s, cd a) { return cd{s + a.re, a.im}; }
__device__ inline cd inv(cd a) {
  const double d = a.re * a.re + a.im * a.im;
  return cd{a.re / d, -a.im / d};
}
__device__ inline cd operator/(cd a, cd b) { return a * inv(b); }
// exp(a + ib) = e^a (cos b + i sin b)
__device__ inline cd cexp_(cd a) {
  const double e = exp(a.re);
  return cd{e * cos(a.im), e * sin(a.im)};
}
// principal logarithm: ln|a| + i arg(a)
__device__ inline cd clog_(cd a) { return cd{0.5 * log(a.re * a.re + a.im * a.im), atan2(a.im, a.re)}; }

// NASA-7: C_p/R, H/(RT), and B_k of Sec. 2.3.1 (the species' share of ln K_c)
__device__ inline void thermo_c(const MechDev& md, int k, cd T, cd lT, cd iT, cd* cpR, cd* hRT, cd* B) {
  const double* a = md.nasa + (size_t)k * 14 + (T.re <= md.tmid[k] ? 0 : 7);
  *cpR = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + a[4] * T)));
  *hRT = a[0] + T * (0.5 * a[1] + T * ((1.0 / 3.0) * a[2] + T * (0.25 * a[3] + (0.2 * a[4]) * T))) + a[5] * iT;
  *B = (a[6] - a[0]) + (a[0] - 1.0) * lT +
       T * (0.5 * a[1] + T * ((1.0 / 6.0) * a[2] + T * ((1.0 / 12.0) * a[3] + (0.05 * a[4]) * T))) - a[5] * iT;
}

template <int NMAX>
__global__ void cs_jacobian_kernel(MechDev md, int64_t n, int64_t ld, const double* __restrict__ phi,
                                   const double* __restrict__ pin, double step, double* __restrict__ jac) {
  const int N = md.N, NR = md.NR;
  const int64_t total = n * N;
  for (int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; idx < total;
       idx += (int64_t)gridDim.x * blockDim.x) {
    const int64_t s = idx % n;
    const int col = (int)(idx / n);
    cd X[NMAX + 1], Bk[NMAX], wd[NMAX];
    // ---- state with the imaginary perturbation on variable col (Sec. 2.1)
    const cd T = mk(phi[s], col == 0 ? step : 0.0);
    const double p = pin[s];
    double sre = 0.0, cre = 0.0, sim = 0.0;        // Neumaier on the real parts
    for (int k = 0; k < N - 1; ++k) {
      const double y = phi[(int64_t)(k + 1) * ld + s];
      X[k] = mk(y, col == k + 1 ? step : 0.0);
      const double t = sre + y;
      cre += (fabs(sre) >= fabs(y)) ? (sre - t) + y : (y - t) + sre;
      sre = t;
      sim += X[k].im;
    }
    X[N - 1] = mk(1.0 - (sre + cre), -sim);       // Y_N, Eq. (y_nsp)
    cd sYW = mk(0.0);
    for (int k = 0; k < N; ++k) sYW = sYW + md.invW[k] * X[k];
    const cd W = inv(sYW);
    const cd lT = clog_(T), iT = inv(T);
    const cd rho = (p / kRg) * W * iT;
    const cd M = (p / kRg) * iT;
    cd cp = mk(0.0);
    for (int k = 0; k < N; ++k) {
      cd cpR, hRT;
      thermo_c(md, k, T, lT, iT, &cpR, &hRT, &Bk[k]);
      cp = cp + (kRg * md.invW[k]) * (X[k] * cpR);  // X holds Y here
      X[k] = (md.invW[k]) * (rho * X[k]);           // [X_k] = rho Y_k / W_k
      wd[k] = mk(0.0);
    }
    X[N] = mk(1.0);
    // real parts of the concentrations for the sign of P_r, from the real
    // parts of rho and Y: the real part of the complex product carries an
    // O(step^2) term that would misplace the test at an exactly zero
    // concentration
    const double YNre = 1.0 - (sre + cre);
    auto xre = [&](int k) {
      const double y = k < N - 1 ? phi[(int64_t)(k + 1) * ld + s] : YNre;
      return rho.re * y * md.invW[k];
    };
    const double lp = log(p), l10p = lp / kLn10c;
    // ---- reactions (Sec. 2.3)
    for (int i = 0; i < NR; ++i) {
      const RxnRec& R = md.rx[i];
      const int info = R.info;
      const int kind = info & 0xF, blend = (info >> 4) & 0xF, rev = (info >> 8) & 0xF, coll = (info >> 12) & 0xF;
      const double* ar = R.arr;
      cd kf;
      if (kind <= K_CHEMACT) {
        kf = ar[0] * cexp_(ar[1] * lT - ar[2] * iT);
      } else if (kind == K_PLOG) {
        const double* pl = md.plog;
        const int p0 = R.aux0, p1 = R.aux1;
        int lo = p0;
        double frac = 0.0;
        if (p1 - p0 > 1 && lp > pl[4 * p0]) {
          if (lp >= pl[4 * (p1 - 1)]) lo = p1 - 1;
          else {
            for (int q = p0; q < p1 - 1; ++q) if (pl[4 * q] <= lp) lo = q;
            frac = (lp - pl[4 * lo]) / (pl[4 * (lo + 1)] - pl[4 * lo]);
          }
        }
        cd lk = pl[4 * lo + 1] + (pl[4 * lo + 2] * lT - pl[4 * lo + 3] * iT);
        if (frac != 0.0) {
          const int hi = lo + 1;
          const cd lk2 = pl[4 * hi + 1] + (pl[4 * hi + 2] * lT - pl[4 * hi + 3] * iT);
          lk = lk + frac * (lk2 - lk);
        }
        kf = cexp_(lk);
      } else {
        const double* cb = md.cheb + R.aux0;
        const int nT = (int)cb[0], nP = (int)cb[1];
        const cd xT = cb[3] + cb[2] * iT;
        const double xP = cb[4] * l10p + cb[5];
        const double* eta = cb + 6;
        cd val = mk(0.0), Tm1 = mk(0.0), Tc = mk(1.0);
        for (int a = 0; a < nT; ++a) {
          double e = 0.0, Pm1 = 0.0, Pc = 1.0;
          for (int b = 0; b < nP; ++b) {
            e += eta[a * nP + b] * Pc;
            const double Pn = (b == 0) ? xP : 2.0 * xP * Pc - Pm1;
            Pm1 = Pc;
            Pc = Pn;
          }
          val = val + e * Tc;
          const cd Tn = (a == 0) ? xT : 2.0 * (xT * Tc) - Tm1;
          Tm1 = Tc;
          Tc = Tn;
        }
        kf = cexp_(kLn10c * val);
      }
      cd kr = mk(0.0);
      if (rev == R_KC) {
        cd sB = mk(R.dnu_lnpr);
        for (int q = 0; q < kMaxNet; ++q) {
          const int v = R.net[q];
          if (v == -1) break;
          sB = sB + (double)(v >> 16) * Bk[v & 0xFFFF];
        }
        kr = kf * cexp_(-sB);                          // k_r = k_f / K_c
      } else if (rev == R_EXPLICIT) {
        const double* arg = R.arr;
        kr = arg[6] * cexp_(arg[7] * lT - arg[8] * iT);
      }
      const int* mo = R.mol;
      const cd Rf = kf * (X[mo[0]] * X[mo[1]] * X[mo[2]]);
      const cd Rr = kr * (X[mo[3]] * X[mo[4]] * X[mo[5]]);
      cd c = mk(1.0);
      if (coll != C_NONE) {
        cd E;
        double Ere;
        if (coll == C_SPECIES) {
          E = X[R.coll_m];
          Ere = xre(R.coll_m);
        } else {
          E = M;
          Ere = M.re;
          if (coll == C_EFF)
            for (int e = R.aux0; e < R.aux1; ++e) {
              E = E + md.eff_am1[e] * X[md.eff_sp[e]];
              Ere += md.eff_am1[e] * xre(md.eff_sp[e]);
            }
        }
        if (kind == K_THD) c = E;
        else {
          const cd ratio = ar[3] * cexp_(ar[4] * lT - ar[5] * iT);
          const cd Pr = ratio * E;
          const bool pos = ratio.re * Ere > 0.0;        // P_r <= 0: the P_r -> 0+ limit
          cd F = mk(1.0);
          const double* fp = R.fpar;
          if (blend == B_TROE) {
            cd Fc = (1.0 - fp[0]) * cexp_(-R.frcp[0] * T) + fp[0] * cexp_(-R.frcp[1] * T);
            if (info & F_TROE_T2) Fc = Fc + cexp_(-fp[3] * iT);
            const cd lnFc = clog_(Fc);
            if (pos) {
              const cd lFc = (1.0 / kLn10c) * lnFc, lPr = (1.0 / kLn10c) * clog_(Pr);
              const cd At = lPr - 0.67 * lFc - mk(0.4);
              const cd Bt = 0.806 + (-1.1762 * lFc - 0.14 * lPr);
              const cd r = At / Bt;
              F = cexp_(lnFc / (1.0 + r * r));
            } else {
              F = cexp_((1.0 / (1.0 + 1.0 / (0.14 * 0.14))) * lnFc);
            }
          } else if (blend == B_SRI) {
            const cd base = fp[0] * cexp_(-fp[1] * iT) + cexp_(-R.frcp[0] * T);
            cd Xs = mk(0.0);
            if (pos) {
              const cd lPr = (1.0 / kLn10c) * clog_(Pr);
              Xs = inv(1.0 + lPr * lPr);
            }
            F = fp[3] * cexp_(fp[4] * lT + Xs * clog_(base));
          }
          c = (kind == K_FALLOFF) ? (Pr / (1.0 + Pr)) * F : F / (1.0 + Pr);
        }
      }
      const cd q = c * (Rf - Rr);
      for (int u = 0; u < kMaxNet; ++u) {
        const int v = R.net[u];
        if (v == -1) break;
        const int k = v & 0xFFFF;
        wd[k] = wd[k] + (double)(v >> 16) * q;
      }
    }
    // ---- RHS (Eqs. ode, dTdt) and the column of the Jacobian
    cd hsum = mk(0.0);
    for (int k = 0; k < N; ++k) {
      cd cpR, hRT, B;
      thermo_c(md, k, T, lT, iT, &cpR, &hRT, &B);
      hsum = hsum + (kRg * T) * (hRT * wd[k]);        // h_k W_k wdot_k
    }
    const cd irho = inv(rho);
    const cd f0 = -(hsum * irho) / cp;
    jac[(int64_t)col * ld + s] = f0.im / step;
    for (int k = 0; k < N - 1; ++k) {
      const cd fk = md.W[k] * (wd[k] * irho);
      jac[((int64_t)(k + 1) * N + col) * ld + s] = fk.im / step;
    }
  }
}

}  // namespace

hipError_t launch_cs_jacobian(const MechDev& md, int64_t n, int64_t ld, const double* phi, const double* p,
                              double step, double* jac, hipStream_t st) {
  const int64_t total = n * md.N;
  const unsigned grid = (unsigned)std::min<int64_t>((total + 127) / 128, 1 << 20);
#define PYJAC_CS(nm)                                                                                         \
  if (md.N <= nm) {                                                                                          \
    hipLaunchKernelGGL(cs_jacobian_kernel<nm>, dim3(grid), dim3(128), 0, st, md, n, ld, phi, p, step, jac); \
    return hipGetLastError();                                                                                \
  }
  PYJAC_CS(16)
  PYJAC_CS(64)
  PYJAC_CS(128)
  PYJAC_CS(384)
#undef PYJAC_CS
  return hipErrorInvalidValue;
}

}  // namespace pyjac
