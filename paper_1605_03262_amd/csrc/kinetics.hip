// HIP kernels (gfx950) for reaction rates, production rates, the
// constant-pressure RHS and its dense analytical Jacobian.
//
// Mapping: one workgroup owns a tile of TS consecutive states and NT threads;
// thread t works on state s = t % TS of the tile and index group g = t / TS,
// so every LDS array is laid out [index][TS] and every HBM access of a
// per-state array touches TS consecutive doubles (element-major, state-fastest
// layout).  All per-state temporaries of the tile stay in LDS:
//   persistent : X[N+1] (concentrations, X[N] = 1), KF[NR] = c k_f,
//                KR[NR] = c k_r, G[NG] = (dc/dE) R, per-state scalars
//   alias      : phase A  Bk[N], dBk[N], per-species c_p terms [2][N]
//                phase B  Bk[N], dBk[N], chunk[2][4][G] of per-reaction results
//                         (two buffers used in turn)
//                phase C+ WA[N], WB[N], JT[N], H[N], per-species sum terms [2][N]
// Every per-state sum over species is formed by one thread in species order
// and no atomics are used, so a state's results depend neither on its
// neighbours nor on the launch shape (TS, NT).
//
// Jacobian algebra (derived from the element formulas of Sec. 3.1, evaluated
// in a reuse order of our own rather than Algorithm 2's dense per-reaction
// update): for species rows k = 1..N (row N is the placeholder of Sec. 3.2)
// and species columns j,
//   J[k][j] = W_k (A_k v_j + B_k) / rho + sum_t coef_t P[src_t] X[x1_t] X[x2_t]
// with v_j = 1/W_j - 1/W_N (from d rho/dY_j and d[X]/dY_j), A_k collecting
// every term proportional to v_j, B_k the j-independent terms of the last
// species, and the table terms the j-specific mass-action and third-body
// efficiency derivatives.  The temperature row follows Sec. 3.2 (Eq. jac_dt)
// and is accumulated while the species rows of a column are stored.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>

#include "tables.hpp"

namespace pyjac {

constexpr double kR = kGasConstant;
constexpr double kLn10 = 2.302585092994045684;
constexpr double kInvLn10 = 0.4342944819032518277;
constexpr int NSC = 16;
enum { SC_T = 0, SC_IT, SC_LT, SC_P, SC_LP, SC_L10P, SC_RHO, SC_W, SC_M, SC_CP, SC_DCP, SC_SHW, SC_J00, SC_HA, SC_HB,
       SC_IRHO };
// per-state scalars of the concentration-based form, in the same rows
enum { SC_IM = SC_RHO, SC_DEN = SC_CP, SC_SUW = SC_DCP, SC_SUU = SC_SHW };

// Register budget of the tile kernels, as wavefronts per SIMD: 4 (128
// registers) for 512- and 1024-thread workgroups; 3 (168 registers, no
// spills at 53 species) for 256-thread ones, whose LDS lets three
// workgroups share a CU.
constexpr int tile_waves_per_eu(int nt) { return nt == 256 ? 3 : (nt <= 512 ? 4 : 1); }

// Phase B keeps its per-reaction results in two buffers used in turn (one
// barrier per reaction chunk instead of two) when the second buffer costs no
// workgroup per CU: the workgroups a CU holds are the fewer of what its
// register budget (4 SIMDs) and its 160 KiB of LDS allow.
__host__ __device__ inline bool two_chunk_buffers(int rows1, int rows2, int TS, int NT) {
  const int waves = NT / 64;
  const int by_regs = (4 * (NT == 256 ? 3 : 4)) / waves;
  const int lds1 = (160 * 1024) / (rows1 * TS * 8), lds2 = (160 * 1024) / (rows2 * TS * 8);
  const int wg1 = by_regs < lds1 ? by_regs : lds1, wg2 = by_regs < lds2 ? by_regs : lds2;
  return wg2 >= wg1;
}

// LDS layout in doubles; each entry counts rows of TS doubles.
struct TileLayout {
  int X, KF, KR, G, SC, alias;
  int Bk, dBk, chunk, redA;      // phases A/B (alias)
  int WA, WB, JT, H, redC;       // phases C/D (alias)
  int rows;                      // total rows
  int nbuf;                      // phase-B chunk buffers (1 or 2)
  __host__ __device__ TileLayout(int N, int NR, int NG, int TS, int NT, bool jac) {
    const int Gr = NT / TS;
    X = 0;
    KF = X + N + 1;                         // must directly follow X: column streams index both from X
    KR = KF + (jac ? NR : 0);
    G = KR + (jac ? NR : 0);
    SC = G + (jac ? NG : 0);
    alias = SC + NSC;
    Bk = alias;
    dBk = Bk + N;
    redA = dBk + (jac ? N : 0);             // per-species terms summed in species order
    chunk = redA;                           // phase B reuses the phase-A reduction rows
    int endA = redA + (jac ? 2 : 1) * N;
    WA = alias;                             // WA and WB interleaved: [k][s][2], k = 0..N (row N: slack)
    WB = WA;
    JT = WA + (jac ? 2 * (N + 1) : 0);
    H = JT + (jac ? N : 0);                 // k = 0..N (row N: slack)
    redC = H + (jac ? N + 1 : 0);
    int endC = redC + (jac ? 2 : 1) * N;
    auto total = [&](int nb) {
      const int endB = chunk + nb * (jac ? 4 : 1) * Gr;
      const int e = endB > endA ? endB : endA;
      return e > endC ? e : endC;
    };
    nbuf = two_chunk_buffers(total(1), total(2), TS, NT) ? 2 : 1;
    rows = total(nbuf);
  }
};

struct RxnResult {
  double q, thT, a, b, KF, KR, G, Rf, Rr, c;
};

// NASA-7 coefficient pointer for species k at temperature T.
__device__ inline const double* nasa_coeffs(const MechDev& md, int k, double T) {
  return md.nasa + (size_t)k * 14 + (T <= md.tmid[k] ? 0 : 7);
}

// Per-reaction evaluation for one state.  Xs points at X[0][s] (stride TS);
// R is the reaction's packed record, fetched by the caller before any branch.
// CV selects the concentration-based, constant-volume form: temperature
// derivatives at constant concentrations (P_r moves with T only through
// k_0/k_inf, a third-body concentration not at all), the pressure
// p = R T sum [X] enters PLOG and Chebyshev rates, and the dense part of
// d q_i / d[X_j] (the all-species collider baseline and the pressure
// dependence) is returned in o.a; iM = 1 / sum [X] is then used.
template <int TS, bool JAC, bool CV = false>
__device__ inline void eval_reaction(const MechDev& md, const RxnRec& R, const RxnRec* __restrict__ Rg,
                                     const double* Xs,
                                     const double* Bks, const double* dBks, double T, double iT,
                                     double lT, double lp, double l10p, double rho, double irho,
                                     double W, double M, RxnResult& o, double iM = 0.0) {
  const int info = R.info;
  const int kind = info & 0xF, blend = (info >> 4) & 0xF, rev = (info >> 8) & 0xF,
            coll = (info >> 12) & 0xF;
  const double* ar = R.arr;          // primary Arrhenius (hot part of the record)
  const double* arg = Rg->arr;       // secondary / reverse parameters, read where needed
  // ---- forward rate coefficient and D_f = T dln k_f/dT (Sec. 2.3, 2.3.4; Sec. 3.1)
  double kf, Df, Dp = 0.0;            // Dp = d ln k_f / d ln p (CV form only)
  if (kind <= K_CHEMACT) {
    kf = ar[0] * exp(ar[1] * lT - ar[2] * iT);
    Df = ar[1] + ar[2] * iT;
  } else if (kind == K_PLOG) {
    const int p0 = R.aux0, p1 = R.aux1;
    const double* pl = md.plog;
    int lo = p0;
    double frac = 0.0;
    bool inside = false;
    if (p1 - p0 > 1 && lp > pl[4 * p0]) {
      if (lp >= pl[4 * (p1 - 1)]) lo = p1 - 1;
      else {
        for (int q = p0; q < p1 - 1; ++q) if (pl[4 * q] <= lp) lo = q;
        frac = (lp - pl[4 * lo]) / (pl[4 * (lo + 1)] - pl[4 * lo]);
        inside = true;
      }
    }
    double lk1 = pl[4 * lo + 1] + pl[4 * lo + 2] * lT - pl[4 * lo + 3] * iT;
    double D1 = pl[4 * lo + 2] + pl[4 * lo + 3] * iT;
    // inside the grid ln k is linear in ln p over the bracket; on a grid point
    // the derivative is the slope of the bracket that starts there
    if (CV ? inside : frac != 0.0) {
      int hi = lo + 1;
      double lk2 = pl[4 * hi + 1] + pl[4 * hi + 2] * lT - pl[4 * hi + 3] * iT;
      double D2 = pl[4 * hi + 2] + pl[4 * hi + 3] * iT;
      if (CV) Dp = (lk2 - lk1) / (pl[4 * hi] - pl[4 * lo]);
      lk1 = lk1 + (lk2 - lk1) * frac;
      D1 = D1 + (D2 - D1) * frac;
    }
    kf = exp(lk1);
    Df = D1;
  } else {   // Chebyshev
    const double* cb = md.cheb + R.aux0;
    const int nT = (int)cb[0], nP = (int)cb[1];
    const double xT = cb[2] * iT + cb[3];
    const double xP = cb[4] * l10p + cb[5];
    const double* eta = cb + 6;
    double val = 0.0, dval = 0.0, pval = 0.0;
    double Tm1 = 0.0, Tc = 1.0;        // T_{a-1}, T_a of the temperature variable
    double Um2 = 0.0, Um1 = 0.0;       // U_{a-2}, U_{a-1}
    for (int a = 0; a < nT; ++a) {
      double e = 0.0, ep = 0.0, Pm1 = 0.0, Pc = 1.0;
      double Qm2 = 0.0, Qm1 = 0.0;     // U_{b-2}, U_{b-1} of the pressure variable
      for (int b = 0; b < nP; ++b) {
        e += eta[a * nP + b] * Pc;
        if (CV) {
          if (b > 0) ep += eta[a * nP + b] * b * Qm1;      // dT_b/dx = b U_{b-1}
          const double Qn = (b == 0) ? 1.0 : ((b == 1) ? 2.0 * xP : 2.0 * xP * Qm1 - Qm2);
          Qm2 = Qm1;
          Qm1 = Qn;
        }
        double Pn = (b == 0) ? xP : 2.0 * xP * Pc - Pm1;
        Pm1 = Pc;
        Pc = Pn;
      }
      val += e * Tc;
      if (CV) pval += ep * Tc;
      if (a > 0) dval += e * a * Um1;
      double Tn = (a == 0) ? xT : 2.0 * xT * Tc - Tm1;
      Tm1 = Tc;
      Tc = Tn;
      double Un = (a == 0) ? 1.0 : ((a == 1) ? 2.0 * xT : 2.0 * xT * Um1 - Um2);
      Um2 = Um1;
      Um1 = Un;
    }
    kf = exp(kLn10 * val);
    Df = -kLn10 * dval * cb[2] * iT;
    if (CV) Dp = pval * cb[4];         // d log10 k / d log10 p
  }
  // ---- reverse rate coefficient (Sec. 2.3.1)
  double kr = 0.0, Dr = 0.0;
  if (rev == R_KC) {
    double sB = 0.0, sdB = 0.0;
#pragma unroll
    for (int q = 0; q < kMaxNet; ++q) {
      int v = R.net[q];
      if (v == -1) break;
      int k = v & 0xFFFF, nu = v >> 16;
      sB += nu * Bks[k * TS];
      if (JAC) sdB += nu * dBks[k * TS];
    }
    kr = kf * exp(-sB - R.dnu_lnpr);
    Dr = Df - T * sdB;                 // K_c depends on T only: d ln k_r / d ln p = Dp
  } else if (rev == R_EXPLICIT) {
    kr = arg[6] * exp(arg[7] * lT - arg[8] * iT);
    Dr = arg[7] + arg[8] * iT;
  }
  // ---- mass-action products over the molecule lists (absent molecules read X[N] = 1)
  const int* mo = R.mol;
  const double pf = Xs[mo[0] * TS] * Xs[mo[1] * TS] * Xs[mo[2] * TS];
  const double pr = Xs[mo[3] * TS] * Xs[mo[4] * TS] * Xs[mo[5] * TS];
  const double Rf = kf * pf, Rr = kr * pr, Rn = Rf - Rr;
  // ---- pressure modification (Sec. 2.3.2, 2.3.3) and its derivatives
  double c = 1.0, psi = 0.0, dcdT = 0.0, E = 0.0;
  if (coll != C_NONE) {
    if (coll == C_SPECIES) E = Xs[R.coll_m * TS];
    else {
      E = M;
      if (coll == C_EFF)
        // four entries per step, loads issued together (the lists carry slack)
        for (int e0 = R.aux0; e0 < R.aux1; e0 += 4) {
          int sp[4];
          double am[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            sp[u] = md.eff_sp[e0 + u];
            am[u] = md.eff_am1[e0 + u];
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (e0 + u < R.aux1) E += am[u] * Xs[sp[u] * TS];
        }
    }
    if (kind == K_THD) {
      c = E;
      psi = 1.0;
      dcdT = CV ? 0.0 : -E * iT;       // constant p: [X] ~ 1/T; constant volume: fixed
    } else {
      const double ratio = arg[3] * exp(arg[4] * lT - arg[5] * iT);   // k0 / kinf
      const double Pr = ratio * E;
      double F = 1.0, Lam = 0.0, dlnFdT = 0.0;
      const double* fp = Rg->fpar;
      if (blend == B_TROE) {
        const double a = fp[0], r3 = Rg->frcp[0], r1 = Rg->frcp[1];
        const double e3 = exp(-T * r3), e1 = exp(-T * r1);
        double Fc = (1.0 - a) * e3 + a * e1;
        double dFc = -(1.0 - a) * r3 * e3 - a * r1 * e1;
        if (info & F_TROE_T2) {
          double e2 = exp(-fp[3] * iT);
          Fc += e2;
          dFc += fp[3] * iT * iT * e2;
        }
        const double lnFc = log(Fc);
        if (Pr > 0.0) {
          const double lFc = lnFc * kInvLn10, lPr = log(Pr) * kInvLn10;
          const double At = lPr - 0.67 * lFc - 0.4;
          const double Bt = 0.806 - 1.1762 * lFc - 0.14 * lPr;
          const double iBt = 1.0 / Bt, iFc = 1.0 / Fc;
          const double r = At * iBt, den = 1.0 + r * r, iden = 1.0 / den;
          F = exp(lnFc * iden);
          const double iden2B3 = iden * iden * iBt * iBt * iBt;          // 1 / (den^2 B^3)
          Lam = -lnFc * 2.0 * At * (Bt + 0.14 * At) * kInvLn10 * iden2B3;
          const double dAB = (-0.67 * Bt + 1.1762 * At) * kInvLn10 * iFc;   // (dA/dFc B - A dB/dFc)
          const double dlnF_dFc = iFc * iden - lnFc * 2.0 * At * dAB * iden2B3;
          dlnFdT = dlnF_dFc * dFc;
        } else {
          // no collider present: the limit P_r -> 0+, where A/B -> -1/0.14
          // and the P_r-derivative term of ln F vanishes
          constexpr double den0 = 1.0 + 1.0 / (0.14 * 0.14);
          F = exp(lnFc / den0);
          dlnFdT = dFc / (Fc * den0);
        }
      } else if (blend == B_SRI) {
        const double rc = Rg->frcp[0];
        const double ea = exp(-fp[1] * iT), ec = exp(-T * rc);
        const double base = fp[0] * ea + ec;
        const double dbase = fp[0] * fp[1] * iT * iT * ea - ec * rc;
        // P_r <= 0 (no collider present) takes the limit P_r -> 0+: X -> 0
        const double lPr = Pr > 0.0 ? log(Pr) * kInvLn10 : 0.0;
        const double Xs_ = Pr > 0.0 ? 1.0 / (1.0 + lPr * lPr) : 0.0;
        const double lnb = log(base);
        F = fp[3] * exp(fp[4] * lT + Xs_ * lnb);
        Lam = -lnb * Xs_ * Xs_ * 2.0 * lPr * kInvLn10;
        dlnFdT = fp[4] * iT + Xs_ * dbase / base;
      }
      // (1/Pr) dPr/dT: through k_0/k_inf, and at constant p through [X]_i ~ 1/T
      const double dlnPr = (arg[4] + arg[5] * iT - (CV ? 0.0 : 1.0)) * iT;
      double Phi;
      const double i1p = 1.0 / (1.0 + Pr);
      if (kind == K_FALLOFF) {
        c = Pr * i1p * F;
        Phi = i1p + Lam;
        psi = ratio * F * Phi * i1p;
      } else {
        c = F * i1p;
        Phi = -Pr * i1p + Lam;
        // dc/dE = c (-ratio/(1+P_r) + dlnF/dP_r ratio); the second term is
        // Lam/E, zero in the P_r -> 0+ limit taken when no collider is present
        psi = -c * ratio * i1p + (Pr > 0.0 ? c * Lam / E : 0.0);
      }
      dcdT = c * (Phi * dlnPr + dlnFdT);
    }
  }
  o.Rf = Rf;
  o.Rr = Rr;
  o.c = c;
  o.q = c * Rn;
  if (JAC && CV) {
    // d ln k / dT at constant concentrations: (D + Dp) / T, since d ln p / dT = 1/T
    const double Dpr = rev == R_KC ? Dp : 0.0;
    o.thT = dcdT * Rn + c * (Rf * (Df + Dp) - Rr * (Dr + Dpr)) * iT;
    const double Gv = psi * Rn;
    // dense part of dq/d[X_j]: the collider baseline alpha = 1 of an
    // all-species third body, and the pressure through d ln p / d[X_j] = 1/sum[X]
    o.a = ((coll == C_EFF || coll == C_UNITY) ? Gv : 0.0) + c * (Rf * Dp - Rr * Dpr) * iM;
    o.b = 0.0;
    o.KF = c * kf;
    o.KR = c * kr;
    o.G = Gv;
  } else if (JAC) {
    const int sf = R.sum_f, sr = R.sum_r;
    const double dRdT = (Rf * (Df - sf) - Rr * (Dr - sr)) * iT;
    o.thT = (dcdT * Rn + c * (dRdT + Rn * iT)) * irho;
    const double Gv = psi * Rn;
    double kappa = 0.0, beta = 0.0;
    if (coll == C_EFF) {
      kappa = rho - E * W;
      beta = -rho * R.alphaN_m1 * md.invW[md.N - 1];
    } else if (coll == C_SPECIES) {
      kappa = -E * W;
      if (R.coll_m == md.N - 1) beta = -rho * md.invW[md.N - 1];
    }
    o.a = -W * c * (Rf * sf - Rr * sr) + Gv * kappa;
    double b = Gv * beta;
    if (info & F_LAST_SPECIES) {
      // c (k_f S'_N - k_r S''_N) with S'_N = d(prod [X]^nu')/d[X_N]: by the
      // product rule over the molecule list, the sum over the molecules equal
      // to N of the product of the other two
      const int L = md.N - 1;
      double SfN = 0.0, SrN = 0.0;
#pragma unroll
      for (int q = 0; q < kMaxSide; ++q) {
        const int u = (q + 1) % kMaxSide, v = (q + 2) % kMaxSide;
        if (mo[q] == L) SfN += Xs[mo[u] * TS] * Xs[mo[v] * TS];
        if (mo[kMaxSide + q] == L) SrN += Xs[mo[kMaxSide + u] * TS] * Xs[mo[kMaxSide + v] * TS];
      }
      b += -c * rho * md.invW[L] * (kf * SfN - kr * SrN);
    }
    o.b = b;
    o.KF = c * kf;
    o.KR = c * kr;
    o.G = Gv;
  }
}

// Workgroups are dispatched round-robin over the eight XCDs (each with its
// own L2).  This permutation hands every XCD a contiguous range of tiles, so
// neighbouring tiles, whose short per-element runs of the Jacobian share
// cache lines, are written through the same L2.
__device__ inline unsigned xcd_tile() {
  constexpr unsigned kXcd = 8;
  const unsigned b = blockIdx.x, G = gridDim.x;
  const unsigned q = G / kXcd, r = G % kXcd, x = b % kXcd, i = b / kXcd;
  return x * q + (x < r ? x : r) + i;
}

// SPLIT selects the form of the Jacobian column streams: every row streamed
// (false) or only the rows with terms, the others written by a dense pass (true).
// The body of one tile (states tile*TS .. tile*TS + TS - 1 of the batch).
template <int TS, int NT, int KPT, bool JAC, bool SPLIT>
__device__ __forceinline__ void tile_body(const MechDev& md, unsigned tile, int64_t n, int64_t ld,
                                          const double* __restrict__ phi, const double* __restrict__ pin,
                                          double* __restrict__ rop_f, double* __restrict__ rop_r,
                                          double* __restrict__ pmod, double* __restrict__ wdot_out,
                                          double* __restrict__ dphi_out, double* __restrict__ jac) {
  constexpr int Gr = NT / TS;
  static_assert(Gr >= 3, "the per-state sums of phase C use three index groups");
  extern __shared__ double lds[];
  const int N = md.N, NR = md.NR, NG = md.NG;
  const int tid = threadIdx.x, s = tid % TS, g = tid / TS;
  const int64_t sg = (int64_t)tile * TS + s;
  const bool live = sg < n;
  const int64_t sl = live ? sg : n - 1;
  const TileLayout L(N, NR, NG, TS, NT, JAC);
  double* X = lds + (size_t)L.X * TS + s;
  double* SC = lds + (size_t)L.SC * TS + s;
  double* Bk = lds + (size_t)L.Bk * TS + s;
  double* dBk = lds + (size_t)L.dBk * TS + s;
  double* red = lds + (size_t)L.redA * TS + s;

  // ---- phase A1: mass fractions, Y_N, mean molecular weight, density (Sec. 2.1)
  for (int k = g; k < N - 1; k += Gr) X[k * TS] = phi[(int64_t)(k + 1) * ld + sl];
  __syncthreads();
  if (g == 0) {
    // Y_N = 1 - sum Y_k with Neumaier compensation: the difference can be
    // tiny when the last species is scarce, so the sum is kept to ~1 ulp.
    double sY = 0.0, cY = 0.0, sYW = 0.0;
    for (int k = 0; k < N - 1; ++k) {
      const double y = X[k * TS];
      const double t = sY + y;
      cY += (fabs(sY) >= fabs(y)) ? (sY - t) + y : (y - t) + sY;
      sY = t;
      sYW += y * md.invW[k];
    }
    const double YN = 1.0 - (sY + cY);
    X[(N - 1) * TS] = YN;
    X[N * TS] = 1.0;
    sYW += YN * md.invW[N - 1];
    const double T = phi[sl], p = pin[sl];
    const double W = 1.0 / sYW;
    SC[SC_T * TS] = T;
    SC[SC_IT * TS] = 1.0 / T;
    SC[SC_LT * TS] = log(T);
    SC[SC_P * TS] = p;
    const double lp = log(p);
    SC[SC_LP * TS] = lp;
    SC[SC_L10P * TS] = lp * kInvLn10;
    SC[SC_W * TS] = W;
    SC[SC_RHO * TS] = p * W / (kR * T);
    SC[SC_IRHO * TS] = kR * T / (p * W);
    SC[SC_M * TS] = p / (kR * T);
  }
  __syncthreads();

  // ---- phase A2: concentrations and NASA-7 thermo (Sec. 2.2), B_k of Sec. 2.3.1
  // (the per-state scalars are read from LDS where they are used, here and in
  // every reaction chunk, rather than held in registers across phase B)
  for (int k = g; k < N; k += Gr) {
    const double T = SC[SC_T * TS], iT = SC[SC_IT * TS], lT = SC[SC_LT * TS];
    const double rho = SC[SC_RHO * TS];
    const double y = X[k * TS];
    X[k * TS] = rho * y * md.invW[k];
    const double* a = nasa_coeffs(md, k, T);
    const double cpR = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + a[4] * T)));
    const double rW = kR * md.invW[k];
    red[k * TS] = y * cpR * rW;
    if (JAC) red[(N + k) * TS] = y * rW * (a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + 4.0 * a[4] * T)));
    Bk[k * TS] = a[6] - a[0] + (a[0] - 1.0) * lT +
                 T * (a[1] * 0.5 + T * (a[2] * (1.0 / 6.0) + T * (a[3] * (1.0 / 12.0) + a[4] * 0.05 * T))) -
                 a[5] * iT;
    if (JAC)
      dBk[k * TS] = (a[0] - 1.0 + a[5] * iT) * iT + a[1] * 0.5 +
                    T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + a[4] * 0.2 * T));
  }
  __syncthreads();
  if (g == 0) {
    // four interleaved partial sums in a fixed order (independent of the
    // launch shape), so the dependent-add chain is a quarter as long
    double c0[4] = {0.0, 0.0, 0.0, 0.0}, c1[4] = {0.0, 0.0, 0.0, 0.0};
    int k = 0;
    for (; k + 4 <= N; k += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        c0[u] += red[(k + u) * TS];
        if (JAC) c1[u] += red[(N + k + u) * TS];
      }
    }
    for (int u = 0; k < N; ++k, ++u) {
      c0[u] += red[k * TS];
      if (JAC) c1[u] += red[(N + k) * TS];
    }
    SC[SC_CP * TS] = (c0[0] + c0[1]) + (c0[2] + c0[3]);
    SC[SC_DCP * TS] = (c1[0] + c1[1]) + (c1[2] + c1[3]);
  }
  __syncthreads();

  // ---- phase B: reactions in chunks of Gr, gathered per species (no atomics)
  double* const chunk0 = lds + (size_t)L.chunk * TS + s;
  double* KF = lds + (size_t)L.KF * TS + s;
  double* KR = lds + (size_t)L.KR * TS + s;
  double* Gs = lds + (size_t)L.G * TS + s;
  double acc[KPT][4];
#pragma unroll
  for (int q = 0; q < KPT; ++q) acc[q][0] = acc[q][1] = acc[q][2] = acc[q][3] = 0.0;
  // With two result buffers the chunks alternate between them and one
  // barrier per chunk suffices: the barrier after chunk c's evaluation also
  // orders every gather of chunk c - 1 before chunk c + 1 overwrites that
  // buffer.  With one, a second barrier follows the gathers.
  const bool two = L.nbuf == 2;
  for (int c0 = 0, ch = 0; c0 < NR; c0 += Gr, ++ch) {
    const int i = c0 + g;
    double* const chunk = chunk0 + (two ? (ch & 1) : 0) * (JAC ? 4 : 1) * Gr * TS;
    // this chunk's gather bounds and first list entries, fetched before the
    // reaction evaluation so that their latency overlaps it
    const int* bnd = md.spg_chunk + (size_t)ch * N;
    int gb0[KPT], gb1[KPT];
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int k = min(g + q * Gr, N - 1);
      gb0[q] = bnd[k];
      gb1[q] = bnd[N + k];
    }
    if (i < NR) {
      RxnRec Rr;
      {   // hot half of the record: 8 independent 16-byte loads
        const int4* src = reinterpret_cast<const int4*>(md.rx + i);
        int4* dst = reinterpret_cast<int4*>(&Rr);
#pragma unroll
        for (int u = 0; u < 8; ++u) dst[u] = src[u];
      }
      RxnResult o;
      eval_reaction<TS, JAC>(md, Rr, md.rx + i, X, Bk, dBk, SC[SC_T * TS], SC[SC_IT * TS], SC[SC_LT * TS],
                             SC[SC_LP * TS], SC[SC_L10P * TS], SC[SC_RHO * TS], SC[SC_IRHO * TS],
                             SC[SC_W * TS], SC[SC_M * TS], o);
      chunk[g * TS] = o.q;
      if (JAC) {
        chunk[(Gr + g) * TS] = o.thT;
        chunk[(2 * Gr + g) * TS] = o.a;
        chunk[(3 * Gr + g) * TS] = o.b;
        KF[i * TS] = o.KF;
        KR[i * TS] = o.KR;
        if (Rr.gslot >= 0) Gs[Rr.gslot * TS] = o.G;
      } else if (live) {
        const int64_t io = Rr.orig;
        if (rop_f) rop_f[io * ld + sg] = o.Rf;
        if (rop_r) rop_r[io * ld + sg] = o.Rr;
        if (pmod) pmod[io * ld + sg] = o.c;
      }
    }
    __syncthreads();
    // species gathers over this chunk: list entries [bnd[ch][k], bnd[ch+1][k]),
    // fetched four at a time so their loads overlap
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int k = g + q * Gr;
      if (k < N) {
        const int e1 = gb1[q];
        for (int e = gb0[q]; e < e1; e += 4) {
          int ent[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) ent[u] = md.spg_ent[e + u];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (e + u < e1) {
              const int r = (ent[u] & 0xFFFF) - c0;
              const double nu = (double)(ent[u] >> 16);
              acc[q][0] += nu * chunk[r * TS];
              if (JAC) {
                acc[q][1] += nu * chunk[(Gr + r) * TS];
                acc[q][2] += nu * chunk[(2 * Gr + r) * TS];
                acc[q][3] += nu * chunk[(3 * Gr + r) * TS];
              }
            }
          }
        }
      }
    }
    if (!two) __syncthreads();
  }
  if (two) __syncthreads();     // the last gathers, before phase C reuses the rows

  // ---- phase C: species terms, RHS (Eqs. ode, dTdt), J[0][0] sums
  double2* WAB = reinterpret_cast<double2*>(lds + (size_t)L.WA * TS) + s;
  double* JT = lds + (size_t)L.JT * TS + s;
  double* H = lds + (size_t)L.H * TS + s;
  double* redc = lds + (size_t)L.redC * TS + s;
  const double T = SC[SC_T * TS], iT = SC[SC_IT * TS];
  const double rho = SC[SC_RHO * TS], irho = SC[SC_IRHO * TS], W = SC[SC_W * TS];
  const double cp = SC[SC_CP * TS], dcpdT = SC[SC_DCP * TS];
  const double icp = 1.0 / cp;
#pragma unroll
  for (int q = 0; q < KPT; ++q) {
    const int k = g + q * Gr;
    if (k < N) {
      const double wd = acc[q][0];
      const double Wk = md.W[k];
      const double* a = nasa_coeffs(md, k, T);
      const double hRT = a[0] + T * (a[1] * 0.5 + T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + a[4] * 0.2 * T))) +
                         a[5] * iT;
      const double hk = hRT * kR * T * md.invW[k];       // mass-specific enthalpy
      redc[k * TS] = hk * Wk * wd;
      if (JAC) {
        const double cpk = (a[0] + T * (a[1] + T * (a[2] + T * (a[3] + a[4] * T)))) * kR * md.invW[k];
        const double JTk = Wk * acc[q][1];
        WAB[k * TS] = make_double2(Wk * (wd * W + acc[q][2]) * irho, Wk * acc[q][3] * irho);
        JT[k * TS] = JTk;
        H[k * TS] = hk;
        redc[(N + k) * TS] = (cpk - hk * icp * dcpdT) * Wk * wd * irho + hk * JTk;
      } else if (live) {
        if (wdot_out) wdot_out[(int64_t)k * ld + sg] = wd;
        if (dphi_out && k < N - 1) dphi_out[(int64_t)(k + 1) * ld + sg] = Wk * wd * irho;
      }
    }
  }
  __syncthreads();
  // per-state sums over species, each formed by one thread in species order;
  // with split column streams two more threads form the sums of h_k times the
  // two dense coefficients, which give the dense part's share of every
  // temperature-row entry in closed form
  if (g == 0) {
    double p0[4] = {0.0, 0.0, 0.0, 0.0}, p1[4] = {0.0, 0.0, 0.0, 0.0};
    int k = 0;
    for (; k + 4 <= N; k += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        p0[u] += redc[(k + u) * TS];
        if (JAC) p1[u] += redc[(N + k + u) * TS];
      }
    }
    for (int u = 0; k < N; ++k, ++u) {
      p0[u] += redc[k * TS];
      if (JAC) p1[u] += redc[(N + k) * TS];
    }
    const double a0 = (p0[0] + p0[1]) + (p0[2] + p0[3]), a1 = (p1[0] + p1[1]) + (p1[2] + p1[3]);
    SC[SC_SHW * TS] = a0;
    if (!JAC && live && dphi_out) dphi_out[sg] = -a0 / (rho * cp);
    if (JAC && live) jac[sg] = -a1 / cp;
  } else if (SPLIT && g < 3) {
    double a = 0.0;
    for (int k = 0; k < N; ++k) a += H[k * TS] * (g == 1 ? WAB[k * TS].x : WAB[k * TS].y);
    SC[(g == 1 ? SC_HA : SC_HB) * TS] = a;
  }
  if (!JAC) return;
  __syncthreads();

  // ---- phase D: temperature column, species columns with the temperature row
  const double Shw = SC[SC_SHW * TS];
  const double HA = SPLIT ? SC[SC_HA * TS] : 0.0, HB = SPLIT ? SC[SC_HB * TS] : 0.0;
  if (live)
    for (int k = g; k < N - 1; k += Gr) jac[(int64_t)((k + 1) * N) * ld + sg] = JT[k * TS];
  const double* aN = nasa_coeffs(md, N - 1, T);
  const double cpN = (aN[0] + T * (aN[1] + T * (aN[2] + T * (aN[3] + aN[4] * T)))) * kR * md.invW[N - 1];
  const double* Xb = lds + (size_t)L.X * TS + s;
  // temperature-row element of column j from TR = sum_k h_k J[k][j] (Sec. 3.2)
  auto finish = [&](int j, double TR) {
    const double* aj = nasa_coeffs(md, j, T);
    const double cpj = (aj[0] + T * (aj[1] + T * (aj[2] + T * (aj[3] + aj[4] * T)))) * kR * md.invW[j];
    if (live) jac[(int64_t)(j + 1) * ld + sg] = -(-(cpj - cpN) * irho * icp * Shw + TR) * icp;
  };
  if constexpr (!SPLIT) {
    // Column segments, longest first, dealt to the groups in snake order
    // (forward on even passes, backward on odd ones) so that a group with a
    // long segment gets a short one next.  A column cut into several segments
    // leaves one partial temperature-row sum per segment in the rows of the
    // phase-C sums (free by now); after a barrier they are added in row order.
    const int nit = md.n_col_item;
    for (int m = 0; m * Gr < nit; ++m) {
      const int it = m * Gr + ((m & 1) ? Gr - 1 - g : g);
      if (it >= nit) continue;
      const ColItem I = md.col_item[it];
      const int j = I.j;
      const double vj = md.vcol[j];
      // Column j, every row streamed: each row's terms, the last one marked
      // (a row without terms is a marker alone), read kColBatch records at a
      // time with independent loads; every record is evaluated without
      // branching (markers and padding have coef = 0) and a marked record
      // finishes the current row after its own term and starts the next.
      // A lane past the end of the batch computes the last state's values
      // (it read that state's inputs) and stores them to that state's
      // elements, the same values the live lane stores, so no store needs a
      // condition.
      const ColRec* rec = md.colrec + I.rec;
      const int cnt = I.cnt;
      double* outp = jac + (int64_t)((I.k0 + 1) * N + j + 1) * ld + sl;   // element (k0+1, j+1)
      const int64_t rstride = (int64_t)N * ld;
      double TR = 0.0;
      // row k's (A_k, B_k) and h_k; the arrays hold a slack row N, so the
      // look-ahead of row k + 1 needs no clamp (its value is then never used)
      const double2* wab = WAB + I.k0 * TS;
      const double* hp = H + I.k0 * TS;
      double val = wab[0].x * vj + wab[0].y;
      double hk = hp[0];
      double2 abn = wab[TS];
      // one batch: the products first, with no branch between them, so that
      // all their LDS reads are in flight together; then the row bookkeeping
      auto batch = [&](const ColRec (&r)[kColBatch]) {
        double t[kColBatch];
#pragma unroll
        for (int u = 0; u < kColBatch; ++u) {
          const int x = r[u].x;
          t[u] = r[u].coef * Xb[r[u].src * TS] * Xb[(x & 0x7FFF) * TS] * Xb[((x >> 15) & 0x7FFF) * TS];
        }
#pragma unroll
        for (int u = 0; u < kColBatch; ++u) {
          val += t[u];
          if (r[u].x & kColMark) {     // ends row k < N - 1 and opens row k + 1
            *outp = val;
            TR += hk * val;
            outp += rstride;
            val = abn.x * vj + abn.y;
            wab += TS;
            hp += TS;
            hk = *hp;
            abn = wab[TS];
          }
        }
      };
      // Two record buffers in turn, each batch's loads issued one batch of
      // work ahead, then a last single batch when the count is odd.  Every
      // load stays inside the table: a segment is followed by another
      // segment or by the table's batch of slack.
      ColRec ra[kColBatch], rb[kColBatch];
#pragma unroll
      for (int u = 0; u < kColBatch; ++u) ra[u] = rec[u];
      int b = 0;
      for (; b + 2 * kColBatch <= cnt; b += 2 * kColBatch) {
#pragma unroll
        for (int u = 0; u < kColBatch; ++u) rb[u] = rec[b + kColBatch + u];
        batch(ra);
#pragma unroll
        for (int u = 0; u < kColBatch; ++u) ra[u] = rec[b + 2 * kColBatch + u];
        batch(rb);
      }
      if (b < cnt) batch(ra);
      // the placeholder row N - 1 (not stored) ends the column's last segment;
      // after an earlier segment the open row belongs to the next one
      if (I.last) TR += hk * val;
      if (I.slot < 0)
        finish(j, TR);
      else
        redc[I.slot * TS] = TR;
    }
    if (md.n_col_join > 0) {
      __syncthreads();
      for (int c = g; c < md.n_col_join; c += Gr) {
        const ColJoin Jn = md.col_join[c];
        double TR = redc[Jn.slot0 * TS];
        for (int q = 1; q < Jn.nslot; ++q) TR += redc[(Jn.slot0 + q) * TS];
        finish(Jn.j, TR);
      }
    }
  } else {
    // columns, longest first, dealt to the groups in snake order
    for (int m = 0; m * Gr < N - 1; ++m) {
      const int jc = m * Gr + ((m & 1) ? Gr - 1 - g : g);
      if (jc >= N - 1) continue;
      const int j = md.col_order[jc];
      const double vj = md.vcol[j];
      double TR;
      double* colp = jac + (int64_t)(N + j + 1) * ld + sg;       // element (1, j+1): row k = 0
      const int64_t rstride = (int64_t)N * ld;
      const int FW = colFlagWords(N);
      // temperature row: sum_k h_k J[k][j], the dense part in closed form here,
      // the terms of the present rows added by the stream below
      TR = vj * HA + HB;
      // Rows without column-stream terms hold the dense part W_k (A_k v_j + B_k)/rho
      // alone.  This pass visits the rows of every 32-row block that has rows
      // not flagged present, in the same order in all lanes, and stores those
      // rows; the present rows are left to the stream.
      const uint32_t* fl = md.col_flags + (size_t)j * FW;
      for (int k0 = 0; k0 < N; k0 += 32) {
        const uint32_t f = fl[k0 >> 5];
        const int kn = min(32, N - k0);
        // rows to store: not present, below the placeholder row N - 1, in range
        uint32_t st = ~f & (kn == 32 ? 0xFFFFFFFFu : (1u << kn) - 1u);
        if (st == 0u) continue;
        if (k0 + kn > N - 1) st &= ~(1u << (N - 1 - k0));
        if (!live) st = 0u;
        for (int kk = 0; kk < kn; kk += 4) {
          // four rows read before any store, so the reads overlap (the empty
          // asm keeps the compiler from moving each read into its store branch)
          double2 ab[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) ab[u] = WAB[min(k0 + kk + u, N - 1) * TS];
#pragma unroll
          for (int u = 0; u < 4; ++u) asm volatile("" : "+v"(ab[u].x), "+v"(ab[u].y));
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if ((st >> (kk + u)) & 1u) colp[(k0 + kk + u) * rstride] = ab[u].x * vj + ab[u].y;
        }
      }
      // Present rows: the column stream, kColBatch records at a time with
      // independent loads.  Every record's product is formed without branching
      // (markers and padding have coef = 0); a marker ends the open row, storing
      // its terms plus the dense part and adding h_k times its terms to the
      // temperature row, and opens the row it names.  No row is open at the
      // start (k = N: nothing is stored and hk = 0).
      const ColRec* rec = md.colrec + md.col_start[j];
      const int cnt = md.col_start[j + 1] - md.col_start[j];
      double val = 0.0, hk = 0.0;
      double2 ab = make_double2(0.0, 0.0);
      int k = N;
      // one batch: the products first, with no branch between them, so that all
      // their LDS reads are in flight together; then the row bookkeeping
      auto batch = [&](const ColRec (&r)[kColBatch]) {
        double t[kColBatch];
#pragma unroll
        for (int u = 0; u < kColBatch; ++u) {
          const int x = r[u].x;
          t[u] = r[u].coef * Xb[r[u].src * TS] * Xb[(x & 0x7FFF) * TS] * Xb[((x >> 15) & 0x7FFF) * TS];
        }
#pragma unroll
        for (int u = 0; u < kColBatch; ++u) {
          val += t[u];
          if (r[u].x & kColMark) {
            if (k < N - 1 && live) colp[k * rstride] = val + (ab.x * vj + ab.y);
            TR += hk * val;
            k = r[u].src;
            val = 0.0;
            // k = N after the last present row: only zero terms follow, so the
            // clamped reads are never used
            const int kc = min(k, N - 1);
            ab = WAB[kc * TS];
            hk = H[kc * TS];
          }
        }
      };
      // Two record buffers in turn: each batch's loads are issued one batch of
      // work ahead.  Streams are padded to a multiple of two batches, and one
      // batch of slack follows the last, so every load stays inside the table.
      ColRec ra[kColBatch], rb[kColBatch];
#pragma unroll
      for (int u = 0; u < kColBatch; ++u) ra[u] = rec[u];
      for (int b = 0; b < cnt; b += 2 * kColBatch) {
#pragma unroll
        for (int u = 0; u < kColBatch; ++u) rb[u] = rec[b + kColBatch + u];
        batch(ra);
#pragma unroll
        for (int u = 0; u < kColBatch; ++u) ra[u] = rec[b + 2 * kColBatch + u];
        batch(rb);
      }
      finish(j, TR);
    }
  }
}

template <int TS, int NT, int KPT, bool JAC, bool SPLIT>
__global__ __launch_bounds__(NT, tile_waves_per_eu(NT)) void tile_kernel(MechDev md, int64_t n, int64_t ld,
                                                  const double* __restrict__ phi,
                                                  const double* __restrict__ pin,
                                                  double* __restrict__ rop_f, double* __restrict__ rop_r,
                                                  double* __restrict__ pmod, double* __restrict__ wdot_out,
                                                  double* __restrict__ dphi_out, double* __restrict__ jac) {
  tile_body<TS, NT, KPT, JAC, SPLIT>(md, xcd_tile(), n, ld, phi, pin, rop_f, rop_r, pmod, wdot_out, dphi_out, jac);
}

// ------------------------------------------------ multi-mechanism work list
// One launch over the Jacobians of several batches, each with its own
// mechanism tables, arrays and size: item i owns the tiles [tile0_i,
// tile0_{i+1}) of the grid (every item shares the launch shape, the stream
// form and an upper bound KPT of species per thread; the dynamic LDS is the
// largest item's).  Per state the results are those of tile_kernel.
template <int TS, int NT, int KPT, bool SPLIT>
__global__ __launch_bounds__(NT, tile_waves_per_eu(NT)) void tile_multi_kernel(WorkList wl) {
  const unsigned t = xcd_tile();
  int i = 0;
  while (i + 1 < wl.n_items && (int64_t)t >= wl.item[i + 1].tile0) ++i;
  const WorkItem& it = wl.item[i];
  tile_body<TS, NT, KPT, true, SPLIT>(it.md, (unsigned)(t - it.tile0), it.n, it.ld, it.phi, it.p, nullptr, nullptr,
                                      nullptr, nullptr, nullptr, it.jac);
}

// ---------------------------------------------- concentration-based Jacobian
// State {T, [X_1..X_N]} of a constant-volume reactor (Sec. 3.3's sparse
// formulation): d[X_k]/dt = wdot_k, dT/dt = -sum U_k wdot_k / sum [X_k] C_v,k
// with U_k = H_k - R T, C_v,k = C_p,k - R (molar).  Output per state, element
// e at out[e*ld + s]:
//   e = 0            J_00 = d(dT/dt)/dT
//   e = 1 .. N       J_k0 = d wdot_k / dT
//   e = N+1 .. 2N    J_0j = d(dT/dt)/d[X_j]
//   e = 2N+1 .. 3N   u_k, the dense part of row k: J_kj = u_k + S_kj
//   e = 3N+1 + q     value q of the sparse part S in compressed-column order
// The tile mapping and the reaction phase are those of tile_kernel; phase D
// streams only the rows with terms and stores each once.
struct CvLayout {
  int X, KF, KR, G, SC, alias, Bk, dBk, chunk, H, red, rows, nbuf;
  __host__ __device__ CvLayout(int N, int NR, int NG, int TS, int NT) {
    const int Gr = NT / TS;
    X = 0;
    KF = X + N + 1;
    KR = KF + NR;
    G = KR + NR;
    SC = G + NG;
    alias = SC + NSC;
    Bk = alias;                         // phases A, B
    dBk = Bk + N;
    chunk = dBk + N;
    H = alias;                          // phases C, D: U_k (row N: slack)
    red = H + N + 1;                    // five per-species sum terms [5][N]
    const int endC = red + 5 * N;
    auto total = [&](int nb) {
      const int endB = chunk + nb * 4 * Gr;
      return endB > endC ? endB : endC;
    };
    nbuf = two_chunk_buffers(total(1), total(2), TS, NT) ? 2 : 1;   // as TileLayout
    rows = total(nbuf);
  }
};

template <int TS, int NT, int KPT>
__global__ __launch_bounds__(NT, tile_waves_per_eu(NT)) void conc_tile_kernel(MechDev md, int64_t n, int64_t ld,
                                                                           const double* __restrict__ phi,
                                                                           double* __restrict__ out) {
  constexpr int Gr = NT / TS;
  extern __shared__ double lds[];
  const int N = md.N, NR = md.NR, NG = md.NG;
  const int tid = threadIdx.x, s = tid % TS, g = tid / TS;
  const int64_t sg = (int64_t)xcd_tile() * TS + s;
  const bool live = sg < n;
  const int64_t sl = live ? sg : n - 1;
  const CvLayout L(N, NR, NG, TS, NT);
  double* X = lds + (size_t)L.X * TS + s;
  double* SC = lds + (size_t)L.SC * TS + s;
  double* Bk = lds + (size_t)L.Bk * TS + s;
  double* dBk = lds + (size_t)L.dBk * TS + s;

  // ---- phase A: concentrations are the state; p = R T sum [X] (Eq. state)
  for (int k = g; k < N; k += Gr) X[k * TS] = phi[(int64_t)(k + 1) * ld + sl];
  __syncthreads();
  if (g == 0) {
    double c4[4] = {0.0, 0.0, 0.0, 0.0};
    int k = 0;
    for (; k + 4 <= N; k += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) c4[u] += X[(k + u) * TS];
    }
    for (int u = 0; k < N; ++k, ++u) c4[u] += X[k * TS];
    const double M = (c4[0] + c4[1]) + (c4[2] + c4[3]);
    const double T = phi[sl];
    const double p = kR * T * M;
    X[N * TS] = 1.0;
    SC[SC_T * TS] = T;
    SC[SC_IT * TS] = 1.0 / T;
    SC[SC_LT * TS] = log(T);
    SC[SC_P * TS] = p;
    const double lp = log(p);
    SC[SC_LP * TS] = lp;
    SC[SC_L10P * TS] = lp * kInvLn10;
    SC[SC_M * TS] = M;
    SC[SC_IM * TS] = 1.0 / M;
  }
  __syncthreads();
  for (int k = g; k < N; k += Gr) {
    const double T = SC[SC_T * TS], iT = SC[SC_IT * TS], lT = SC[SC_LT * TS];
    const double* a = nasa_coeffs(md, k, T);
    Bk[k * TS] = a[6] - a[0] + (a[0] - 1.0) * lT +
                 T * (a[1] * 0.5 + T * (a[2] * (1.0 / 6.0) + T * (a[3] * (1.0 / 12.0) + a[4] * 0.05 * T))) -
                 a[5] * iT;
    dBk[k * TS] = (a[0] - 1.0 + a[5] * iT) * iT + a[1] * 0.5 +
                  T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + a[4] * 0.2 * T));
  }
  __syncthreads();

  // ---- phase B: reactions in chunks, gathered per species (no atomics):
  // acc 0 wdot_k, 1 d wdot_k/dT, 2 u_k
  double* const chunk0 = lds + (size_t)L.chunk * TS + s;
  double* KF = lds + (size_t)L.KF * TS + s;
  double* KR = lds + (size_t)L.KR * TS + s;
  double* Gs = lds + (size_t)L.G * TS + s;
  double acc[KPT][3];
#pragma unroll
  for (int q = 0; q < KPT; ++q) acc[q][0] = acc[q][1] = acc[q][2] = 0.0;
  // one or two result buffers, as in tile_body
  const bool two = L.nbuf == 2;
  for (int c0 = 0, ch = 0; c0 < NR; c0 += Gr, ++ch) {
    const int i = c0 + g;
    double* const chunk = chunk0 + (two ? (ch & 1) : 0) * 4 * Gr * TS;
    const int* bnd = md.spg_chunk + (size_t)ch * N;
    int gb0[KPT], gb1[KPT];
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int k = min(g + q * Gr, N - 1);
      gb0[q] = bnd[k];
      gb1[q] = bnd[N + k];
    }
    if (i < NR) {
      RxnRec Rr;
      {
        const int4* src = reinterpret_cast<const int4*>(md.rx + i);
        int4* dst = reinterpret_cast<int4*>(&Rr);
#pragma unroll
        for (int u = 0; u < 8; ++u) dst[u] = src[u];
      }
      RxnResult o;
      eval_reaction<TS, true, true>(md, Rr, md.rx + i, X, Bk, dBk, SC[SC_T * TS], SC[SC_IT * TS],
                                    SC[SC_LT * TS], SC[SC_LP * TS], SC[SC_L10P * TS], 0.0, 0.0, 0.0,
                                    SC[SC_M * TS], o, SC[SC_IM * TS]);
      chunk[g * TS] = o.q;
      chunk[(Gr + g) * TS] = o.thT;
      chunk[(2 * Gr + g) * TS] = o.a;
      KF[i * TS] = o.KF;
      KR[i * TS] = o.KR;
      if (Rr.gslot >= 0) Gs[Rr.gslot * TS] = o.G;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int k = g + q * Gr;
      if (k < N) {
        const int e1 = gb1[q];
        for (int e = gb0[q]; e < e1; e += 4) {
          int ent[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) ent[u] = md.spg_ent[e + u];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            if (e + u < e1) {
              const int r = (ent[u] & 0xFFFF) - c0;
              const double nu = (double)(ent[u] >> 16);
              acc[q][0] += nu * chunk[r * TS];
              acc[q][1] += nu * chunk[(Gr + r) * TS];
              acc[q][2] += nu * chunk[(2 * Gr + r) * TS];
            }
          }
        }
      }
    }
    if (!two) __syncthreads();
  }
  if (two) __syncthreads();     // the last gathers, before phase C reuses the rows

  // ---- phase C: temperature column, dense row parts, temperature-row sums
  double* H = lds + (size_t)L.H * TS + s;
  double* red = lds + (size_t)L.red * TS + s;
  {
    const double T = SC[SC_T * TS];
#pragma unroll
    for (int q = 0; q < KPT; ++q) {
      const int k = g + q * Gr;
      if (k < N) {
        const double* a = nasa_coeffs(md, k, T);
        const double cpR = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + a[4] * T)));
        const double hRT = a[0] + T * (a[1] * 0.5 + T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + a[4] * 0.2 * T))) +
                           a[5] / T;
        const double U = kR * T * (hRT - 1.0);                  // molar internal energy
        const double Cv = kR * (cpR - 1.0);                      // molar C_v
        const double dCv = kR * (a[1] + T * (2.0 * a[2] + T * (3.0 * a[3] + 4.0 * a[4] * T)));
        const double Ck = X[k * TS];
        H[k * TS] = U;
        red[k * TS] = U * acc[q][0];
        red[(N + k) * TS] = Ck * Cv;
        red[(2 * N + k) * TS] = Cv * acc[q][0] + U * acc[q][1];
        red[(3 * N + k) * TS] = Ck * dCv;
        red[(4 * N + k) * TS] = U * acc[q][2];
        if (live) {
          out[(int64_t)(1 + k) * ld + sg] = acc[q][1];
          out[(int64_t)(2 * N + 1 + k) * ld + sg] = acc[q][2];
        }
      }
    }
  }
  __syncthreads();
  if (g < 5) {
    // five per-state sums over species, each by one thread group in a fixed
    // order (four interleaved partial sums)
    double p4[4] = {0.0, 0.0, 0.0, 0.0};
    const double* r = red + (size_t)g * N * TS;
    int k = 0;
    for (; k + 4 <= N; k += 4) {
#pragma unroll
      for (int u = 0; u < 4; ++u) p4[u] += r[(k + u) * TS];
    }
    for (int u = 0; k < N; ++k, ++u) p4[u] += r[k * TS];
    const double v = (p4[0] + p4[1]) + (p4[2] + p4[3]);
    // sums: 0 sum U wdot, 1 D = sum [X] C_v, 2 sum (C_v wdot + U dwdot/dT),
    // 3 sum [X] dC_v/dT, 4 sum U u
    SC[(g == 0 ? SC_SUW : g == 1 ? SC_DEN : g == 4 ? SC_SUU : (g == 2 ? SC_J00 : SC_HA)) * TS] = v;
  }
  __syncthreads();
  const double D = SC[SC_DEN * TS], SUw = SC[SC_SUW * TS], SUu = SC[SC_SUU * TS];
  const double iD = 1.0 / D;
  if (g == 0 && live) out[sg] = (-SC[SC_J00 * TS] + SUw * SC[SC_HA * TS] * iD) * iD;

  // ---- phase D: sparse part, one column stream per group (present rows)
  const double T = SC[SC_T * TS];
  const double* Xb = lds + (size_t)L.X * TS + s;
  for (int jc = g; jc < N; jc += Gr) {
    const int j = md.cv_col_order[jc];
    const ColRec* rec = md.cv_colrec + md.cv_col_start[j];
    const int cnt = md.cv_col_start[j + 1] - md.cv_col_start[j];
    // lanes past the batch end store the last state's (identical) values
    double* outp = out + (int64_t)(3 * N + 1 + md.cv_colptr[j]) * ld + sl;
    double val = 0.0, hk = 0.0, TR = 0.0;
    int k = N;                          // no row open before the first marker
    auto batch = [&](const ColRec (&r)[kColBatch]) {
      double t[kColBatch];
#pragma unroll
      for (int u = 0; u < kColBatch; ++u) {
        const int x = r[u].x;
        t[u] = r[u].coef * Xb[r[u].src * TS] * Xb[(x & 0x7FFF) * TS] * Xb[((x >> 15) & 0x7FFF) * TS];
      }
#pragma unroll
      for (int u = 0; u < kColBatch; ++u) {
        val += t[u];
        if (r[u].x & kColMark) {       // ends the open row (if any), opens row src
          if (k < N) {
            *outp = val;
            outp += ld;
            TR += hk * val;
          }
          k = r[u].src;
          val = 0.0;
          hk = H[k * TS];              // row N: slack, never used
        }
      }
    };
    ColRec ra[kColBatch], rb[kColBatch];
#pragma unroll
    for (int u = 0; u < kColBatch; ++u) ra[u] = rec[u];
    for (int b = 0; b < cnt; b += 2 * kColBatch) {
#pragma unroll
      for (int u = 0; u < kColBatch; ++u) rb[u] = rec[b + kColBatch + u];
      batch(ra);
#pragma unroll
      for (int u = 0; u < kColBatch; ++u) ra[u] = rec[b + 2 * kColBatch + u];
      batch(rb);
    }
    // temperature row: sum_k U_k J_kj = sum_k U_k S_kj + sum_k U_k u_k
    const double* aj = nasa_coeffs(md, j, T);
    const double Cvj = kR * (aj[0] + T * (aj[1] + T * (aj[2] + T * (aj[3] + aj[4] * T))) - 1.0);
    if (live) out[(int64_t)(N + 1 + j) * ld + sg] = (-(TR + SUu) + SUw * Cvj * iD) * iD;
  }
}

// ------------------------------------------------- PaSR mixing fractional step
// Pairwise mixing of a partially stirred reactor's particles (App. C): each
// particle s with a partner q relaxes towards it in mixture enthalpy and mass
// fractions, phi_s <- phi_s - w (phi_s - phi_q) with w = (1 - exp(-2 dt/tau))/2,
// and its temperature is recovered from the mixed enthalpy by Newton's method
// on h(T) = sum_k Y_k h_k(T) (Sec. 2.2 polynomials).  Out of place: every
// particle reads the old state of both members of its pair.
__device__ inline double mix_enthalpy(const MechDev& md, double T, const double* Y, double* cp) {
  double h = 0.0, c = 0.0;
  for (int k = 0; k < md.N; ++k) {
    const double* a = nasa_coeffs(md, k, T);
    const double cpR = a[0] + T * (a[1] + T * (a[2] + T * (a[3] + a[4] * T)));
    const double hR = T * (a[0] + T * (a[1] * 0.5 + T * (a[2] * (1.0 / 3.0) + T * (a[3] * 0.25 + a[4] * 0.2 * T)))) +
                      a[5];
    h += Y[k] * hR * kR * md.invW[k];
    c += Y[k] * cpR * kR * md.invW[k];
  }
  *cp = c;
  return h;
}

template <int NMAX>
__global__ void mix_pairs_kernel(MechDev md, int64_t n, int64_t ld, const double* __restrict__ phi,
                                 const int* __restrict__ partner, double w, double* __restrict__ out) {
  const int N = md.N;
  for (int64_t s = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; s < n; s += (int64_t)gridDim.x * blockDim.x) {
    const int q = partner[s];
    if (q < 0 || q >= n) {
      for (int e = 0; e < N; ++e) out[(int64_t)e * ld + s] = phi[(int64_t)e * ld + s];
      continue;
    }
    double Ys[NMAX], Yq[NMAX], Ym[NMAX];
    double ss = 0.0, sq = 0.0;
    for (int k = 0; k < N - 1; ++k) {
      Ys[k] = phi[(int64_t)(k + 1) * ld + s];
      Yq[k] = phi[(int64_t)(k + 1) * ld + q];
      ss += Ys[k];
      sq += Yq[k];
    }
    Ys[N - 1] = 1.0 - ss;
    Yq[N - 1] = 1.0 - sq;
    const double Ts = phi[s], Tq = phi[q];
    double cp;
    const double hs = mix_enthalpy(md, Ts, Ys, &cp), hq = mix_enthalpy(md, Tq, Yq, &cp);
    for (int k = 0; k < N; ++k) Ym[k] = Ys[k] - w * (Ys[k] - Yq[k]);
    const double hm = hs - w * (hs - hq);
    double T = Ts - w * (Ts - Tq);
    for (int it = 0; it < 50; ++it) {
      const double h = mix_enthalpy(md, T, Ym, &cp);
      const double dT = (hm - h) / cp;
      T += dT;
      if (fabs(dT) <= 1e-13 * T) break;
    }
    out[s] = T;
    for (int k = 0; k < N - 1; ++k) out[(int64_t)(k + 1) * ld + s] = Ym[k];
  }
}

hipError_t launch_mix_pairs(const MechDev& md, int64_t n, int64_t ld, const double* phi, const int* partner, double w,
                            double* out, hipStream_t st) {
  const unsigned grid = (unsigned)std::min<int64_t>((n + 255) / 256, 65536);
#define PYJAC_MIX(nm) \
  if (md.N <= nm) { hipLaunchKernelGGL(mix_pairs_kernel<nm>, dim3(grid), dim3(256), 0, st, md, n, ld, phi, partner, w, out); return hipGetLastError(); }
  PYJAC_MIX(64)
  PYJAC_MIX(128)
  PYJAC_MIX(384)
  PYJAC_MIX(1024)
#undef PYJAC_MIX
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------------ launchers
size_t tile_lds_bytes(int N, int NR, int NG, int TS, int NT, bool jac) {
  TileLayout L(N, NR, NG, TS, NT, jac);
  return (size_t)L.rows * TS * sizeof(double);
}

template <int TS, int NT, int KPT, bool JAC, bool SPLIT>
static hipError_t launch_t(const MechDev& md, int64_t n, int64_t ld, const double* phi, const double* p,
                           double* a, double* b, double* c, double* d, double* e, double* jac,
                           size_t lds, hipStream_t st) {
  auto kern = tile_kernel<TS, NT, KPT, JAC, SPLIT>;
  hipError_t err = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  const int64_t tiles = (n + TS - 1) / TS;
  hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(NT), lds, st, md, n, ld, phi, p, a, b, c, d, e, jac);
  return hipGetLastError();
}

template <int TS, int NT, bool JAC, bool SPLIT>
static hipError_t launch_k(int kpt, const MechDev& md, int64_t n, int64_t ld, const double* phi,
                           const double* p, double* a, double* b, double* c, double* d, double* e,
                           double* jac, size_t lds, hipStream_t st) {
  if (kpt <= 1) return launch_t<TS, NT, 1, JAC, SPLIT>(md, n, ld, phi, p, a, b, c, d, e, jac, lds, st);
  if (kpt <= 2) return launch_t<TS, NT, 2, JAC, SPLIT>(md, n, ld, phi, p, a, b, c, d, e, jac, lds, st);
  if (kpt <= 4) return launch_t<TS, NT, 4, JAC, SPLIT>(md, n, ld, phi, p, a, b, c, d, e, jac, lds, st);
  if (kpt <= 8) return launch_t<TS, NT, 8, JAC, SPLIT>(md, n, ld, phi, p, a, b, c, d, e, jac, lds, st);
  return hipErrorInvalidValue;
}

size_t conc_lds_bytes(int N, int NR, int NG, int TS, int NT) {
  CvLayout L(N, NR, NG, TS, NT);
  return (size_t)L.rows * TS * sizeof(double);
}

template <int TS, int NT, int KPT>
static hipError_t launch_conc_t(const MechDev& md, int64_t n, int64_t ld, const double* phi, double* out,
                                size_t lds, hipStream_t st) {
  auto kern = conc_tile_kernel<TS, NT, KPT>;
  hipError_t err = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  const int64_t tiles = (n + TS - 1) / TS;
  hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(NT), lds, st, md, n, ld, phi, out);
  return hipGetLastError();
}

template <int TS, int NT, int KPT, bool SPLIT>
static hipError_t launch_multi_t(const WorkList& wl, int64_t tiles, size_t lds, hipStream_t st) {
  auto kern = tile_multi_kernel<TS, NT, KPT, SPLIT>;
  hipError_t err = hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (err != hipSuccess) return err;
  hipLaunchKernelGGL(kern, dim3((unsigned)tiles), dim3(NT), lds, st, wl);
  return hipGetLastError();
}

// Work-list Jacobian launch (see tile_multi_kernel); tiles = the grid size.
hipError_t launch_tile_multi(int TS, int NT, int kpt, bool split, const WorkList& wl, int64_t tiles, size_t lds,
                             hipStream_t st) {
#define PYJAC_MULTI_K(ts, nt, k)                                                            \
  if (kpt <= k) return split ? launch_multi_t<ts, nt, k, true>(wl, tiles, lds, st)          \
                             : launch_multi_t<ts, nt, k, false>(wl, tiles, lds, st);
#define PYJAC_MULTI(ts, nt)      \
  if (TS == ts && NT == nt) {    \
    PYJAC_MULTI_K(ts, nt, 1)     \
    PYJAC_MULTI_K(ts, nt, 2)     \
    PYJAC_MULTI_K(ts, nt, 4)     \
    PYJAC_MULTI_K(ts, nt, 8)     \
    return hipErrorInvalidValue; \
  }
  PYJAC_MULTI(16, 1024)
  PYJAC_MULTI(8, 256)
  PYJAC_MULTI(4, 256)
  PYJAC_MULTI(8, 512)
  PYJAC_MULTI(8, 1024)
  PYJAC_MULTI(4, 512)
  PYJAC_MULTI(4, 1024)
  PYJAC_MULTI(2, 512)
  PYJAC_MULTI(2, 1024)
#undef PYJAC_MULTI
#undef PYJAC_MULTI_K
  return hipErrorInvalidValue;
}

// Concentration-form Jacobian launch; shapes (TS, NT) as listed in the body.
hipError_t launch_conc(int TS, int NT, const MechDev& md, int64_t n, int64_t ld, const double* phi, double* out,
                       size_t lds, hipStream_t st) {
  const int kpt = (md.N + NT / TS - 1) / (NT / TS);
#define PYJAC_CONC(ts, nt)                                                             \
  if (TS == ts && NT == nt) {                                                          \
    if (kpt <= 1) return launch_conc_t<ts, nt, 1>(md, n, ld, phi, out, lds, st);       \
    if (kpt <= 2) return launch_conc_t<ts, nt, 2>(md, n, ld, phi, out, lds, st);       \
    if (kpt <= 4) return launch_conc_t<ts, nt, 4>(md, n, ld, phi, out, lds, st);       \
    if (kpt <= 8) return launch_conc_t<ts, nt, 8>(md, n, ld, phi, out, lds, st);       \
    return hipErrorInvalidValue;                                                       \
  }
  PYJAC_CONC(16, 1024)
  PYJAC_CONC(8, 256)
  PYJAC_CONC(4, 256)
  PYJAC_CONC(8, 512)
  PYJAC_CONC(8, 1024)
  PYJAC_CONC(4, 512)
  PYJAC_CONC(4, 1024)
  PYJAC_CONC(2, 512)
#undef PYJAC_CONC
  return hipErrorInvalidValue;
}

// Supported (TS, NT) variants; species per thread kpt = ceil(N / (NT/TS)) <= 8.
hipError_t launch_tile(bool jac_mode, int TS, int NT, const MechDev& md, int64_t n, int64_t ld,
                       const double* phi, const double* p, double* rop_f, double* rop_r, double* pmod,
                       double* wdot, double* dphi, double* jac, size_t lds, hipStream_t st) {
  const int kpt = (md.N + NT / TS - 1) / (NT / TS);
#define PYJAC_VARIANT(ts, nt)                                                                          \
  if (TS == ts && NT == nt)                                                                            \
    return !jac_mode ? launch_k<ts, nt, false, false>(kpt, md, n, ld, phi, p, rop_f, rop_r, pmod, wdot, dphi, jac, lds, st) \
         : md.col_split ? launch_k<ts, nt, true, true>(kpt, md, n, ld, phi, p, rop_f, rop_r, pmod, wdot, dphi, jac, lds, st) \
                        : launch_k<ts, nt, true, false>(kpt, md, n, ld, phi, p, rop_f, rop_r, pmod, wdot, dphi, jac, lds, st);
  PYJAC_VARIANT(16, 1024)
  PYJAC_VARIANT(16, 512)
  PYJAC_VARIANT(8, 256)
  PYJAC_VARIANT(4, 256)
  PYJAC_VARIANT(32, 1024)
  PYJAC_VARIANT(64, 1024)
  PYJAC_VARIANT(8, 512)
  PYJAC_VARIANT(8, 1024)
  PYJAC_VARIANT(4, 512)
  PYJAC_VARIANT(4, 1024)
  PYJAC_VARIANT(2, 512)
  PYJAC_VARIANT(2, 1024)
#undef PYJAC_VARIANT
  return hipErrorInvalidValue;
}

}  // namespace pyjac
