// CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
//
// A plain, slow FP64 evaluation of the constant-pressure ideal-gas chemical
// source terms and of their exact Jacobian, written directly from the
// formulas of Niemeyer, Curtis & Sung, "pyJac: analytical Jacobian generator
// for chemical kinetics" (arXiv:1605.03262).  Only the tests, the smoke check
// and the benchmark's CPU-baseline leg may load this library; the GPU library
// never links or calls it, and the two share no source, header, table or
// constant.
//
// What is computed, and where it is defined in the paper:
//   state, mean molecular weight, density, concentrations   Sec. 2.1, Eqs. (vars),(y_nsp),(state)
//   RHS f = {dT/dt, dY_k/dt}                                  Sec. 2.1, Eqs. (ode),(dTdt)
//   NASA-7 thermo                                            Sec. 2.2, Eqs. (cpk),(hk),(sk)
//   rates of progress, pressure modification c_i             Sec. 2.3, Eq. (rxn_pressure)
//   Arrhenius k_f in its plain form                          Sec. 2.3, Eq. (arrhenius)
//   k_r = k_f / K_c with K_c from Delta S - Delta H          Sec. 2.3.1, Eq. (kri) and K_p
//   third-body concentration                                 Sec. 2.3.2
//   falloff: P_r, Lindemann / Troe / SRI blending            Sec. 2.3.3
//   PLOG and Chebyshev rate expressions                      Sec. 2.3.4
//   Jacobian elements, all partial derivatives               Sec. 3.1
//   evaluation order: species rows (with the last-species
//   placeholder row) first, then the temperature row         Sec. 3.2, Eqs. (jac_dydt),(jac_dydy),(jac_dt)
//   constant-volume, concentration-based RHS and Jacobian   Sec. 3.3 (the sparse formulation), Sec. 6
//
// The Jacobian is assembled element by element in the naive order of
// Algorithm 1 (species rows, reactions innermost), NOT in the restructured
// order of Algorithm 2 / Sec. 4, so its rounding path differs from any
// reuse-based evaluation.  The per-reaction derivative vectors dc_i/dY_j and
// dR_i/dY_j are formed literally from the printed product-rule expressions
// (Kronecker deltas included, [X]^(nu-1) formed directly, no division by [X]).
//
// Readings where the paper is silent or inconsistent:
//   * temperature row: the second statement (Sec. 3.2, Eq. jac_dt and the
//     J_{1,1} expression before it) is used; it follows from differentiating
//     Eq. (dTdt).  The first statement in Sec. 3.1 misplaces 1/c_p.
//   * chemically activated reactions use k_f = k_0 (low-pressure Arrhenius),
//     falloff reactions k_f = k_inf; P_r = k_0 [X]_i / k_inf in both.
//   * PLOG outside its pressure grid is clamped to the end-point rate; inside,
//     the bracket is the last grid point p_n <= p.
//   * Chebyshev polynomials are evaluated by the three-term recurrences for
//     T_n (first kind) and U_n (second kind), without clamping.
//   * NASA range: T <= T_mid uses the low-temperature coefficients.
//   * P_r <= 0 (no collider present): the Troe and SRI blending functions take
//     their limits as P_r -> 0+ (log10 P_r -> -inf), and the derivatives of c
//     are written so that nothing divides by P_r (Sec. 2.3.3, Sec. 3.1).
//   * SI-kmol units: R = 8314.462618 J/(kmol K), p_atm = 101325 Pa.
//
// The RHS is a template over the scalar type so the same code runs in
// double, long double and std::complex<double> (complex-step Jacobian).

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <fstream>
#include <map>
#include <sstream>
#include <stdexcept>
#include <string>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr double kR = 8314.462618;      // J / (kmol K)
constexpr double kPatm = 101325.0;      // Pa
const double kLn10 = std::log(10.0);

thread_local std::string g_err;

enum Kind { ELEM = 0, THD = 1, FALLOFF = 2, CHEMACT = 3, PLOG = 4, CHEB = 5 };
enum Rev { KC = 0, EXPLICIT = 1, IRREV = 2 };
enum Blend { LIND = 0, TROE = 1, SRI = 2 };

struct Arr { double A = 0, b = 0, Ta = 0; };

struct Rxn {
  Kind kind = ELEM;
  Rev rev = KC;
  Blend blend = LIND;
  std::vector<std::pair<int, int>> reac, prod;   // (species, nu)
  Arr arr, low, high, revarr;
  std::vector<double> troe;       // a, T***, T*, [T**]
  std::vector<double> sri;        // a, b, c, [d, e]
  bool has_collider = false;
  bool collider_species = false;  // [X]_i = [X_m]
  int m = -1;
  std::vector<double> alpha;      // third-body efficiency of every species
  std::vector<std::array<double, 4>> plog;   // p, A, b, Ta (sorted by p)
  int nT = 0, nP = 0;
  double Tmin = 0, Tmax = 0, Pmin = 0, Pmax = 0;
  std::vector<double> eta;        // nT x nP, row-major over T index
};

struct Mech {
  int N = 0, NR = 0;
  std::vector<std::string> names;
  std::vector<double> W, tmid;
  std::vector<std::array<double, 7>> lo, hi;
  std::vector<Rxn> rxn;
  std::vector<int> nu_f, nu_r;    // dense N x NR, [k * NR + i]
  // index lists that only skip zero stoichiometric terms of the sums below
  std::vector<std::vector<int>> rxn_species;   // species with nu' or nu'' != 0, ascending
  std::vector<std::vector<int>> species_rxns;  // reactions with nu_ki != 0, ascending
  int nuf(int k, int i) const { return nu_f[(size_t)k * NR + i]; }
  int nur(int k, int i) const { return nu_r[(size_t)k * NR + i]; }
  int nu(int k, int i) const { return nur(k, i) - nuf(k, i); }
};

// ------------------------------------------------------------------ parser
struct Tok {
  std::vector<std::string> t;
  size_t i = 0;
  explicit Tok(const std::string& text) {
    std::istringstream lines(text);
    std::string line;
    while (std::getline(lines, line)) {
      auto h = line.find('#');
      if (h != std::string::npos) line = line.substr(0, h);
      std::istringstream ws(line);
      std::string w;
      while (ws >> w) t.push_back(w);
    }
  }
  bool done() const { return i >= t.size(); }
  const std::string& peek() const {
    if (done()) throw std::runtime_error("unexpected end of mechanism text");
    return t[i];
  }
  std::string next() { std::string s = peek(); ++i; return s; }
  double num() {
    std::string s = next();
    char* end = nullptr;
    double v = std::strtod(s.c_str(), &end);
    if (end == s.c_str() || *end) throw std::runtime_error("expected a number, got '" + s + "'");
    return v;
  }
  long integer() {
    std::string s = next();
    char* end = nullptr;
    long v = std::strtol(s.c_str(), &end, 10);
    if (end == s.c_str() || *end) throw std::runtime_error("expected an integer, got '" + s + "'");
    return v;
  }
  void expect(const char* w) {
    std::string s = next();
    if (s != w) throw std::runtime_error(std::string("expected '") + w + "', got '" + s + "'");
  }
};

Arr read_arr(Tok& tk) { Arr a; a.A = tk.num(); a.b = tk.num(); a.Ta = tk.num(); return a; }

Mech parse(const std::string& text) {
  Tok tk(text);
  Mech m;
  tk.expect("pyjac-mech");
  if (tk.integer() != 1) throw std::runtime_error("unsupported mechanism format version");
  tk.expect("elements");
  long ne = tk.integer();
  for (long e = 0; e < ne; ++e) { tk.next(); tk.num(); }
  tk.expect("species");
  m.N = (int)tk.integer();
  if (m.N < 2) throw std::runtime_error("need at least two species");
  std::map<std::string, int> idx;
  for (int k = 0; k < m.N; ++k) {
    std::string name = tk.next();
    if (idx.count(name)) throw std::runtime_error("duplicate species " + name);
    idx[name] = k;
    m.names.push_back(name);
    m.W.push_back(tk.num());
    m.tmid.push_back(tk.num());
    long nc = tk.integer();
    for (long c = 0; c < nc; ++c) { tk.next(); tk.integer(); }
    std::array<double, 7> lo{}, hi{};
    for (auto& a : lo) a = tk.num();
    for (auto& a : hi) a = tk.num();
    m.lo.push_back(lo);
    m.hi.push_back(hi);
  }
  auto sp = [&](const std::string& s) {
    auto it = idx.find(s);
    if (it == idx.end()) throw std::runtime_error("unknown species " + s);
    return it->second;
  };
  tk.expect("reactions");
  m.NR = (int)tk.integer();
  m.nu_f.assign((size_t)m.N * m.NR, 0);
  m.nu_r.assign((size_t)m.N * m.NR, 0);
  for (int i = 0; i < m.NR; ++i) {
    tk.expect("reaction");
    Rxn r;
    std::string kind = tk.next(), rev = tk.next();
    if (kind == "elementary") r.kind = ELEM;
    else if (kind == "thirdbody") r.kind = THD;
    else if (kind == "falloff") r.kind = FALLOFF;
    else if (kind == "chemact") r.kind = CHEMACT;
    else if (kind == "plog") r.kind = PLOG;
    else if (kind == "cheb") r.kind = CHEB;
    else throw std::runtime_error("unknown reaction type " + kind);
    if (rev == "kc") r.rev = KC;
    else if (rev == "explicit") r.rev = EXPLICIT;
    else if (rev == "irrev") r.rev = IRREV;
    else throw std::runtime_error("unknown reversibility " + rev);
    r.alpha.assign(m.N, 1.0);
    while (!tk.done() && tk.peek() != "reaction" && tk.peek() != "end") {
      std::string key = tk.next();
      if (key == "reactants" || key == "products") {
        long n = tk.integer();
        for (long c = 0; c < n; ++c) {
          int k = sp(tk.next());
          long nu = tk.integer();
          (key == "reactants" ? r.reac : r.prod).push_back({k, (int)nu});
        }
      } else if (key == "arrhenius") r.arr = read_arr(tk);
      else if (key == "low") r.low = read_arr(tk);
      else if (key == "high") r.high = read_arr(tk);
      else if (key == "reverse") r.revarr = read_arr(tk);
      else if (key == "lindemann") r.blend = LIND;
      else if (key == "troe") {
        r.blend = TROE;
        long n = tk.integer();
        for (long c = 0; c < n; ++c) r.troe.push_back(tk.num());
      } else if (key == "sri") {
        r.blend = SRI;
        long n = tk.integer();
        for (long c = 0; c < n; ++c) r.sri.push_back(tk.num());
      } else if (key == "collider") {
        r.has_collider = true;
        std::string how = tk.next();
        if (how == "mix") {
          long n = tk.integer();
          for (long c = 0; c < n; ++c) { int k = sp(tk.next()); r.alpha[k] = tk.num(); }
        } else if (how == "species") {
          r.collider_species = true;
          r.m = sp(tk.next());
        } else throw std::runtime_error("unknown collider " + how);
      } else if (key == "plog") {
        long n = tk.integer();
        for (long c = 0; c < n; ++c) {
          std::array<double, 4> pt{};
          for (auto& v : pt) v = tk.num();
          r.plog.push_back(pt);
        }
        std::sort(r.plog.begin(), r.plog.end(),
                  [](const std::array<double, 4>& a, const std::array<double, 4>& b) { return a[0] < b[0]; });
      } else if (key == "cheb") {
        r.nT = (int)tk.integer(); r.nP = (int)tk.integer();
        r.Tmin = tk.num(); r.Tmax = tk.num(); r.Pmin = tk.num(); r.Pmax = tk.num();
        for (int c = 0; c < r.nT * r.nP; ++c) r.eta.push_back(tk.num());
      } else throw std::runtime_error("unknown reaction keyword " + key);
    }
    for (auto& [k, n] : r.reac) m.nu_f[(size_t)k * m.NR + i] += n;
    for (auto& [k, n] : r.prod) m.nu_r[(size_t)k * m.NR + i] += n;
    if ((r.kind == THD || r.kind == FALLOFF || r.kind == CHEMACT) && !r.has_collider)
      throw std::runtime_error("pressure-dependent reaction without collider");
    if (r.kind == PLOG && r.plog.empty()) throw std::runtime_error("PLOG without points");
    if (r.kind == CHEB && (r.nT < 1 || r.nP < 1)) throw std::runtime_error("bad Chebyshev shape");
    m.rxn.push_back(r);
  }
  tk.expect("end");
  m.rxn_species.assign(m.NR, {});
  m.species_rxns.assign(m.N, {});
  for (int i = 0; i < m.NR; ++i)
    for (int k = 0; k < m.N; ++k) {
      if (m.nuf(k, i) || m.nur(k, i)) m.rxn_species[i].push_back(k);
      if (m.nu(k, i)) m.species_rxns[k].push_back(i);
    }
  return m;
}

// ------------------------------------------------------- scalar helpers
inline double re(double x) { return x; }
inline long double re(long double x) { return x; }
inline double re(const std::complex<double>& x) { return x.real(); }

template <class S> S ipow(S x, int n) { S r = S(1); for (int c = 0; c < n; ++c) r *= x; return r; }
template <class S> S log10s(const S& x) { using std::log; return log(x) / S(kLn10); }

// Neumaier compensated sum of Y_1..Y_{N-1} (branching on real parts only).
template <class S> S compensated_sum(const S* y, int n) {
  S s = S(0), c = S(0);
  for (int k = 0; k < n; ++k) {
    S t = s + y[k];
    using std::abs;
    if (abs(re(s)) >= abs(re(y[k]))) c += (s - t) + y[k];
    else c += (y[k] - t) + s;
    s = t;
  }
  return s + c;
}

// Arrhenius expression in its plain form, Sec. 2.3 Eq. (arrhenius).
template <class S> S arrhenius(const Arr& a, const S& T) {
  using std::exp; using std::pow;
  return S(a.A) * pow(T, S(a.b)) * exp(-S(a.Ta) / T);
}

// ---------------------------------------------------- state & thermo (Sec. 2.1, 2.2)
template <class S> struct State {
  int N;
  S T, W, rho, cp;
  std::vector<S> Y, X, cpR, hRT, sR;   // all N species
  // real parts of the concentrations, formed from the real parts of rho and
  // Y, for branch decisions only: in a complex-step evaluation the real part
  // of rho * Y carries an O(h^2) term that would misplace the sign test of an
  // exactly zero concentration
  std::vector<double> Xre;
};

template <class S> void thermo(const Mech& m, const S& T, S* cpR, S* hRT, S* sR) {
  using std::log;
  for (int k = 0; k < m.N; ++k) {
    const auto& a = (re(T) <= m.tmid[k]) ? m.lo[k] : m.hi[k];
    // Eqs. (cpk), (hk), (sk): C_p/R, H/R (divided by T), S/R
    cpR[k] = S(a[0]) + T * (S(a[1]) + T * (S(a[2]) + T * (S(a[3]) + S(a[4]) * T)));
    hRT[k] = (T * (S(a[0]) + T * (S(a[1] / 2) + T * (S(a[2] / 3) + T * (S(a[3] / 4) + S(a[4] / 5) * T))))
              + S(a[5])) / T;
    sR[k] = S(a[0]) * log(T) + T * (S(a[1]) + T * (S(a[2] / 2) + T * (S(a[3] / 3) + S(a[4] / 4) * T)))
            + S(a[6]);
  }
}

template <class S> void make_state(const Mech& m, const S& T, double p, const S* yfirst, State<S>& st) {
  const int N = m.N;
  st.N = N;
  st.T = T;
  st.Y.assign(N, S(0));
  for (int k = 0; k < N - 1; ++k) st.Y[k] = yfirst[k];
  st.Y[N - 1] = S(1) - compensated_sum(yfirst, N - 1);           // Eq. (y_nsp)
  S inv = S(0);
  for (int k = 0; k < N; ++k) inv += st.Y[k] / S(m.W[k]);
  st.W = S(1) / inv;                                              // mean molecular weight
  st.rho = S(p) * st.W / (S(kR) * T);                             // Eq. (state)
  st.X.resize(N);
  for (int k = 0; k < N; ++k) st.X[k] = st.rho * st.Y[k] / S(m.W[k]);   // [X_k]
  st.Xre.resize(N);
  for (int k = 0; k < N; ++k) st.Xre[k] = double(re(st.rho)) * double(re(st.Y[k])) / m.W[k];
  st.cpR.resize(N); st.hRT.resize(N); st.sR.resize(N);
  thermo(m, T, st.cpR.data(), st.hRT.data(), st.sR.data());
  st.cp = S(0);
  for (int k = 0; k < N; ++k) st.cp += st.Y[k] * st.cpR[k] * S(kR) / S(m.W[k]);
}

// ---------------------------------------------------- per-reaction rate terms (Sec. 2.3)
template <class S> struct RxnVals {
  S kf, kr, c, Rf, Rr, Kc;
  // falloff intermediates
  S k0, kinf, E, Pr, F, Fcent, At, Bt, Xs, sri_base;
};

// The pressure is of the scalar type: in the constant-volume form it is a
// function of the state (p = R T sum [X_k]).  Bracket decisions use its real part.
template <class S> S plog_kf(const Rxn& r, const S& T, const S& p, int* lo_out, double* frac_out) {
  using std::log; using std::exp;
  const auto& pts = r.plog;
  int n = (int)pts.size();
  auto lnk = [&](int q) { return log(S(pts[q][1])) + S(pts[q][2]) * log(T) - S(pts[q][3]) / T; };
  if (n == 1 || re(p) <= pts[0][0]) { *lo_out = 0; *frac_out = -1; return exp(lnk(0)); }
  if (re(p) >= pts[n - 1][0]) { *lo_out = n - 1; *frac_out = -1; return exp(lnk(n - 1)); }
  int lo = 0;
  for (int q = 0; q < n - 1; ++q) if (pts[q][0] <= re(p)) lo = q;
  S frac = (log(p) - S(std::log(pts[lo][0]))) / S(std::log(pts[lo + 1][0]) - std::log(pts[lo][0]));
  *lo_out = lo; *frac_out = double(re(frac));
  S l1 = lnk(lo), l2 = lnk(lo + 1);
  return exp(l1 + (l2 - l1) * frac);                           // Eq. (plog)
}

template <class S> void cheb_polys(int n, const S& x, S* Tn, S* Un) {
  // first kind T_0..T_{n-1}, second kind U_0..U_{n-1}, by recurrence
  if (n > 0) { Tn[0] = S(1); Un[0] = S(1); }
  if (n > 1) { Tn[1] = x; Un[1] = S(2) * x; }
  for (int q = 2; q < n; ++q) {
    Tn[q] = S(2) * x * Tn[q - 1] - Tn[q - 2];
    Un[q] = S(2) * x * Un[q - 1] - Un[q - 2];
  }
}

template <class S> S cheb_kf(const Rxn& r, const S& T, const S& p) {
  using std::pow;
  S Tr = (S(2) / T - S(1.0 / r.Tmin) - S(1.0 / r.Tmax)) / S(1.0 / r.Tmax - 1.0 / r.Tmin);
  S pr = (S(2) * log10s(p) - S(std::log10(r.Pmin) + std::log10(r.Pmax))) /
         S(std::log10(r.Pmax) - std::log10(r.Pmin));
  std::vector<S> tT(r.nT), uT(r.nT), tP(r.nP), uP(r.nP);
  cheb_polys(r.nT, Tr, tT.data(), uT.data());
  cheb_polys(r.nP, pr, tP.data(), uP.data());
  S lg = S(0);
  for (int i = 0; i < r.nT; ++i)
    for (int j = 0; j < r.nP; ++j) lg += S(r.eta[i * r.nP + j]) * tT[i] * tP[j];   // Eq. (cheb)
  return pow(S(10), lg);
}

template <class S> void reaction_values(const Mech& m, int i, const State<S>& st, const S& p, RxnVals<S>& v) {
  using std::exp; using std::log; using std::pow;
  const Rxn& r = m.rxn[i];
  const S& T = st.T;
  v.c = S(1);
  v.k0 = v.kinf = v.E = v.Pr = v.F = v.Fcent = v.At = v.Bt = v.Xs = v.sri_base = S(0);
  int lo; double frac;
  switch (r.kind) {
    case ELEM: case THD: v.kf = arrhenius(r.arr, T); break;
    case FALLOFF: v.k0 = arrhenius(r.low, T); v.kinf = arrhenius(r.high, T); v.kf = v.kinf; break;
    case CHEMACT: v.k0 = arrhenius(r.low, T); v.kinf = arrhenius(r.high, T); v.kf = v.k0; break;
    case PLOG: v.kf = plog_kf(r, T, p, &lo, &frac); break;
    case CHEB: v.kf = cheb_kf(r, T, p); break;
  }
  if (r.kind == THD || r.kind == FALLOFF || r.kind == CHEMACT) {
    // third-body concentration, Sec. 2.3.2
    if (r.collider_species) v.E = st.X[r.m];
    else { v.E = S(0); for (int j = 0; j < m.N; ++j) v.E += S(r.alpha[j]) * st.X[j]; }
  }
  if (r.kind == THD) v.c = v.E;
  if (r.kind == FALLOFF || r.kind == CHEMACT) {
    v.Pr = v.k0 / v.kinf * v.E;                                     // Eq. (pr_i)
    // P_r <= 0 (an absent single-species collider, or one driven slightly
    // negative by rounding): F takes its limit as P_r -> 0+, where log10 P_r
    // -> -inf.  Troe: A/B -> 1/(-0.14), so F -> F_cent^(1/(1 + 1/0.14^2));
    // SRI: X -> 0, so F -> d T^e.
    double Ere = 0;
    if (r.collider_species) Ere = st.Xre[r.m];
    else for (int j = 0; j < m.N; ++j) Ere += r.alpha[j] * st.Xre[j];
    const bool pos = double(re(v.k0 / v.kinf)) * Ere > 0;
    if (r.blend == LIND) v.F = S(1);
    else if (r.blend == TROE) {
      const auto& t = r.troe;
      v.Fcent = S(1 - t[0]) * exp(-T / S(t[1])) + S(t[0]) * exp(-T / S(t[2]));
      if (t.size() > 3) v.Fcent += exp(-S(t[3]) / T);
      if (pos) {
        S lF = log10s(v.Fcent), lP = log10s(v.Pr);
        v.At = lP - S(0.67) * lF - S(0.4);
        v.Bt = S(0.806) - S(1.1762) * lF - S(0.14) * lP;
        v.F = pow(v.Fcent, S(1) / (S(1) + (v.At / v.Bt) * (v.At / v.Bt)));
      } else {
        v.F = pow(v.Fcent, S(1) / (S(1) + S(1.0 / (0.14 * 0.14))));
      }
    } else {
      const auto& s = r.sri;
      double d = s.size() > 3 ? s[3] : 1.0, e = s.size() > 4 ? s[4] : 0.0;
      if (pos) {
        S lP = log10s(v.Pr);
        v.Xs = S(1) / (S(1) + lP * lP);
      } else {
        v.Xs = S(0);
      }
      v.sri_base = S(s[0]) * exp(-S(s[1]) / T) + exp(-T / S(s[2]));
      v.F = S(d) * pow(T, S(e)) * pow(v.sri_base, v.Xs);
    }
    v.c = (r.kind == FALLOFF) ? v.Pr / (S(1) + v.Pr) * v.F : S(1) / (S(1) + v.Pr) * v.F;   // Eq. (rxn_pressure)
  }
  // reverse rate coefficient, Sec. 2.3.1
  if (r.rev == KC) {
    int dnu = 0;
    S sum = S(0);
    for (int k : m.rxn_species[i]) {
      int n = m.nu(k, i);
      if (n) { dnu += n; sum += S(n) * (st.sR[k] - st.hRT[k]); }
    }
    v.Kc = pow(S(kPatm) / (S(kR) * T), S(dnu)) * exp(sum);          // K_c = K_p (p_atm/RT)^{sum nu}
    v.kr = v.kf / v.Kc;
  } else if (r.rev == EXPLICIT) { v.Kc = S(0); v.kr = arrhenius(r.revarr, T); }
  else { v.Kc = S(0); v.kr = S(0); }
  S pf = S(1), pr = S(1);
  for (auto& [k, n] : r.reac) pf *= ipow(st.X[k], n);
  for (auto& [k, n] : r.prod) pr *= ipow(st.X[k], n);
  v.Rf = v.kf * pf;
  v.Rr = v.kr * pr;
}

// RHS, Eqs. (ode), (dTdt).  out: wdot[N], dphi[N]; optional per-reaction terms.
template <class S> void rhs(const Mech& m, const S& T, double p, const S* y, S* wdot, S* dphi,
                            S* rop_f, S* rop_r, S* pmod) {
  State<S> st;
  make_state(m, T, p, y, st);
  const int N = m.N;
  for (int k = 0; k < N; ++k) wdot[k] = S(0);
  RxnVals<S> v;
  std::vector<S> q(m.NR);
  const S pS(p);
  for (int i = 0; i < m.NR; ++i) {
    reaction_values(m, i, st, pS, v);
    q[i] = v.c * (v.Rf - v.Rr);
    if (rop_f) rop_f[i] = v.Rf;
    if (rop_r) rop_r[i] = v.Rr;
    if (pmod) pmod[i] = v.c;
  }
  for (int k = 0; k < N; ++k) {
    S acc = S(0);
    for (int i : m.species_rxns[k]) acc += S(m.nu(k, i)) * q[i];
    wdot[k] = acc;
  }
  S hsum = S(0);
  for (int k = 0; k < N; ++k) hsum += st.hRT[k] * S(kR) * T * wdot[k];    // h_k W_k wdot_k
  dphi[0] = -hsum / (st.rho * st.cp);
  for (int k = 0; k < N - 1; ++k) dphi[k + 1] = S(m.W[k]) * wdot[k] / st.rho;
}

// dF/dT and (dF/dP_r)/F of the blending function of a falloff or chemically
// activated reaction (Sec. 2.3.3 definitions, differentiated as in Sec. 3.1),
// given dP_r/dT along the path of the formulation (it differs between the
// constant-pressure and the constant-volume forms).
void blend_derivs(const Rxn& r, const RxnVals<double>& x, double T, double dPrdT, double& dFdT,
                  double& dFdPr_over_F) {
  dFdT = 0;
  dFdPr_over_F = 0;
  if (x.Pr <= 0) {
    // P_r -> 0+ limit (see reaction_values): F depends on T alone, and
    // every P_r-derivative of ln F vanishes in the limit
    if (r.blend == TROE) {
      const auto& t = r.troe;
      double dFc_dT = -(1 - t[0]) / t[1] * std::exp(-T / t[1]) - t[0] / t[2] * std::exp(-T / t[2]);
      if (t.size() > 3) dFc_dT += t[3] / (T * T) * std::exp(-t[3] / T);
      dFdT = x.F / (x.Fcent * (1 + 1 / (0.14 * 0.14))) * dFc_dT;
    } else if (r.blend == SRI) {
      dFdT = x.F * ((r.sri.size() > 4 ? r.sri[4] : 0.0) / T);
    }
  } else if (r.blend == TROE) {
    const auto& t = r.troe;
    double ratio2 = (x.At / x.Bt) * (x.At / x.Bt);
    double dA_dFc = -0.67 / (x.Fcent * kLn10), dB_dFc = -1.1762 / (x.Fcent * kLn10);
    double dA_dPr = 1.0 / (x.Pr * kLn10), dB_dPr = -0.14 / (x.Pr * kLn10);
    double lnFc = std::log(x.Fcent);
    double dF_dFc = x.F * (1.0 / (x.Fcent * (1 + ratio2)) -
                           lnFc * 2 * x.At / (x.Bt * x.Bt * x.Bt) * (dA_dFc * x.Bt - x.At * dB_dFc) /
                               ((1 + ratio2) * (1 + ratio2)));
    double dFc_dT = -(1 - t[0]) / t[1] * std::exp(-T / t[1]) - t[0] / t[2] * std::exp(-T / t[2]);
    if (t.size() > 3) dFc_dT += t[3] / (T * T) * std::exp(-t[3] / T);
    double dF_dPr = -x.F * lnFc * 2 * x.At / (x.Bt * x.Bt * x.Bt) * (dA_dPr * x.Bt - x.At * dB_dPr) /
                    ((1 + ratio2) * (1 + ratio2));
    dFdT = dF_dFc * dFc_dT + dF_dPr * dPrdT;
    dFdPr_over_F = dF_dPr / x.F;
  } else if (r.blend == SRI) {
    const auto& s = r.sri;
    double e = s.size() > 4 ? s[4] : 0.0;
    double lP = std::log10(x.Pr);
    double dX_dPr = -x.Xs * x.Xs * 2 * lP / (x.Pr * kLn10);
    double num = s[0] * s[1] / (T * T) * std::exp(-s[1] / T) - 1.0 / s[2] * std::exp(-T / s[2]);
    dFdT = x.F * (e / T + x.Xs * num / x.sri_base + dX_dPr * dPrdT * std::log(x.sri_base));
    dFdPr_over_F = dX_dPr * std::log(x.sri_base);
  }
}

// ---------------------------------------------------------- analytical Jacobian (Sec. 3)
void jacobian(const Mech& m, double T, double p, const double* y, double* J /* N*N row-major */) {
  const int N = m.N, NR = m.NR;
  State<double> st;
  make_state(m, T, p, y, st);
  const double rho = st.rho, W = st.W, cp = st.cp;
  std::vector<double> v(N);                        // 1/W_j - 1/W_N
  for (int j = 0; j < N; ++j) v[j] = 1.0 / m.W[j] - 1.0 / m.W[N - 1];
  // dc_p/dT (Eq. dcpdT) and dc_{p,k}/dT
  double dcpdT = 0;
  std::vector<double> cpk(N), hk(N);
  for (int k = 0; k < N; ++k) {
    const auto& a = (T <= m.tmid[k]) ? m.lo[k] : m.hi[k];
    double dcpk = kR / m.W[k] * (a[1] + T * (2 * a[2] + T * (3 * a[3] + 4 * a[4] * T)));
    dcpdT += st.Y[k] * dcpk;
    cpk[k] = st.cpR[k] * kR / m.W[k];
    hk[k] = st.hRT[k] * kR * T / m.W[k];
  }
  // dB_k/dT (Sec. 2.3.1)
  std::vector<double> dBdT(N);
  for (int k = 0; k < N; ++k) {
    const auto& a = (T <= m.tmid[k]) ? m.lo[k] : m.hi[k];
    dBdT[k] = (a[0] - 1 + a[5] / T) / T + a[1] / 2 + T * (a[2] / 3 + T * (a[3] / 4 + a[4] / 5 * T));
  }
  // partial derivatives of concentrations w.r.t. Y_j (j = 0..N-2 here means Y_{j+1})
  auto dX_dY = [&](int i_sp, int j) {
    double dij = (i_sp == j) ? 1.0 : 0.0, diN = (i_sp == N - 1) ? 1.0 : 0.0;
    return -st.X[i_sp] * W * v[j] + (dij - diN) * rho / m.W[i_sp];
  };
  std::vector<RxnVals<double>> vals(NR);
  std::vector<double> dcdT(NR), dRdT(NR);
  std::vector<double> dcdY((size_t)NR * (N - 1), 0.0), dRdY((size_t)NR * (N - 1), 0.0);
  std::vector<double> wdot(N, 0.0);
  for (int i = 0; i < NR; ++i) {
    const Rxn& r = m.rxn[i];
    RxnVals<double>& x = vals[i];
    reaction_values(m, i, st, p, x);
    // --- dk_f/dT
    double dkfdT = 0;
    switch (r.kind) {
      case ELEM: case THD: dkfdT = x.kf / T * (r.arr.b + r.arr.Ta / T); break;         // Eq. (dkfdT)
      case FALLOFF: dkfdT = x.kf / T * (r.high.b + r.high.Ta / T); break;
      case CHEMACT: dkfdT = x.kf / T * (r.low.b + r.low.Ta / T); break;
      case PLOG: {
        int lo; double frac;
        plog_kf(r, T, p, &lo, &frac);
        const auto& a1 = r.plog[lo];
        if (frac < 0) dkfdT = x.kf / T * (a1[2] + a1[3] / T);
        else {
          const auto& a2 = r.plog[lo + 1];
          dkfdT = x.kf / T * (a1[2] + a1[3] / T + (a2[2] - a1[2] + (a2[3] - a1[3]) / T) * frac);
        }
        break;
      }
      case CHEB: {
        double Tr = (2 / T - 1 / r.Tmin - 1 / r.Tmax) / (1 / r.Tmax - 1 / r.Tmin);
        double pr = (2 * std::log10(p) - std::log10(r.Pmin) - std::log10(r.Pmax)) /
                    (std::log10(r.Pmax) - std::log10(r.Pmin));
        std::vector<double> tT(r.nT), uT(r.nT), tP(r.nP), uP(r.nP);
        cheb_polys(r.nT, Tr, tT.data(), uT.data());
        cheb_polys(r.nP, pr, tP.data(), uP.data());
        double sum = 0;
        for (int a = 1; a < r.nT; ++a)                      // (i-1) U_{i-2}(T~) with i-1 = a
          for (int b = 0; b < r.nP; ++b)
            sum += r.eta[a * r.nP + b] * a * uT[a - 1] * tP[b] * (-2 / T) / (1 / r.Tmax - 1 / r.Tmin);
        dkfdT = x.kf / T * kLn10 * sum;
        break;
      }
    }
    // --- dk_r/dT
    double dkrdT = 0;
    if (r.rev == KC) {
      double snu = 0;
      for (int k : m.rxn_species[i]) { int n = m.nu(k, i); if (n) snu += n * dBdT[k]; }
      dkrdT = x.kr * (dkfdT / x.kf - snu);                               // Eq. (dkrdT_general) with dK_c/dT
    } else if (r.rev == EXPLICIT) dkrdT = x.kr / T * (r.revarr.b + r.revarr.Ta / T);
    // --- dR/dT: product rule with d[X]/dT = -[X]/T (Eqs. dRfdT-orig, dRdT_explicit_rev_general)
    int sf = 0, sr = 0;
    double pf = 1, pr = 1;
    for (auto& [k, n] : r.reac) { sf += n; pf *= ipow(st.X[k], n); }
    for (auto& [k, n] : r.prod) { sr += n; pr *= ipow(st.X[k], n); }
    dRdT[i] = dkfdT * pf - x.kf * pf * sf / T - (dkrdT * pr - x.kr * pr * sr / T);
    // --- dc/dT and dc/dY (Sec. 3.1)
    double dPrdT = 0, dlnPrdT = 0, dFdT = 0, dFdPr_over_F = 0;   // dF/dPr / F
    if (r.kind == FALLOFF || r.kind == CHEMACT) {
      dlnPrdT = (r.low.b - r.high.b + (r.low.Ta - r.high.Ta) / T - 1) / T;       // Eq. (dPridT) / P_r
      dPrdT = x.Pr * dlnPrdT;
      blend_derivs(r, x, T, dPrdT, dFdT, dFdPr_over_F);
    }
    if (r.kind == THD) dcdT[i] = -x.c / T;
    else if (r.kind == FALLOFF) dcdT[i] = x.c * (dlnPrdT / (1 + x.Pr) + dFdT / x.F);
    else if (r.kind == CHEMACT) dcdT[i] = x.c * (-dPrdT / (1 + x.Pr) + dFdT / x.F);
    else dcdT[i] = 0;
    double* dc = &dcdY[(size_t)i * (N - 1)];
    double* dR = &dRdY[(size_t)i * (N - 1)];
    for (int j = 0; j < N - 1; ++j) {
      if (r.kind == THD || r.kind == FALLOFF || r.kind == CHEMACT) {
        double dE;
        if (r.collider_species) dE = dX_dY(r.m, j);
        else dE = -x.E * W * v[j] + rho * (r.alpha[j] / m.W[j] - r.alpha[N - 1] / m.W[N - 1]);
        if (r.kind == THD) dc[j] = dE;
        else {
          double dPr = x.k0 / x.kinf * dE;                                  // Eq. (dPridY)
          double dFoverF = dFdPr_over_F * dPr;                               // dF/dY_j / F
          // d/dY_j of P_r/(1+P_r) F and of F/(1+P_r): (1+P_r)^-2 dP_r F plus c dF/F
          if (r.kind == FALLOFF) dc[j] = x.F / ((1 + x.Pr) * (1 + x.Pr)) * dPr + x.c * dFoverF;
          else dc[j] = x.c * (-dPr / (1 + x.Pr) + dFoverF);
        }
      }
      // dR_i/dY_j: product rule over every species of the reaction (Sec. 3.1, reversible form)
      double acc = 0;
      for (int k : m.rxn_species[i]) {
        int a = m.nuf(k, i), b = m.nur(k, i);
        double dkj = (k == j) ? 1.0 : 0.0, dkN = (k == N - 1) ? 1.0 : 0.0;
        if (a) {
          double other = 1;
          for (auto& [l, n] : r.reac) if (l != k) other *= ipow(st.X[l], n);
          acc += a * (-x.Rf * W * v[j] + (dkj - dkN) * x.kf * rho / m.W[k] * ipow(st.X[k], a - 1) * other);
        }
        if (b) {
          double other = 1;
          for (auto& [l, n] : r.prod) if (l != k) other *= ipow(st.X[l], n);
          acc -= b * (-x.Rr * W * v[j] + (dkj - dkN) * x.kr * rho / m.W[k] * ipow(st.X[k], b - 1) * other);
        }
      }
      dR[j] = acc;
    }
  }
  for (int k = 0; k < N; ++k) {
    double acc = 0;
    for (int i : m.species_rxns[k]) acc += m.nu(k, i) * vals[i].c * (vals[i].Rf - vals[i].Rr);
    wdot[k] = acc;
  }
  // Species rows k = 1..N (row N is the placeholder for the last species), Eqs. (jac_dydt), (jac_dydy)
  std::vector<double> JT(N), JY((size_t)N * (N - 1));
  for (int k = 0; k < N; ++k) {
    double acc = 0;
    for (int i : m.species_rxns[k]) {
      int n = m.nu(k, i);
      const auto& x = vals[i];
      acc += n * (dcdT[i] * (x.Rf - x.Rr) + x.c * (dRdT[i] + (x.Rf - x.Rr) / T));
    }
    JT[k] = m.W[k] / rho * acc;
    for (int j = 0; j < N - 1; ++j) {
      double s = 0;
      for (int i : m.species_rxns[k]) {
        int n = m.nu(k, i);
        const auto& x = vals[i];
        s += n * (dcdY[(size_t)i * (N - 1) + j] * (x.Rf - x.Rr) + x.c * dRdY[(size_t)i * (N - 1) + j]);
      }
      JY[(size_t)k * (N - 1) + j] = m.W[k] / rho * (wdot[k] * W * v[j] + s);
    }
  }
  // Temperature row, Sec. 3.2 Eq. (jac_dt) and the J_{1,1} expression before it
  double sum00 = 0, hw = 0;
  for (int k = 0; k < N; ++k) {
    sum00 += (cpk[k] - hk[k] / cp * dcpdT) * m.W[k] * wdot[k] / rho + hk[k] * JT[k];
    hw += hk[k] * m.W[k] * wdot[k];
  }
  J[0] = -sum00 / cp;
  for (int j = 0; j < N - 1; ++j) {
    double s = 0;
    for (int k = 0; k < N; ++k) s += hk[k] * JY[(size_t)k * (N - 1) + j];
    J[j + 1] = -1.0 / cp * (-(cpk[j] - cpk[N - 1]) / (rho * cp) * hw + s);
  }
  for (int k = 0; k < N - 1; ++k) {
    J[(size_t)(k + 1) * N] = JT[k];
    for (int j = 0; j < N - 1; ++j) J[(size_t)(k + 1) * N + j + 1] = JY[(size_t)k * (N - 1) + j];
  }
}

// ------------------------------------- constant-volume, concentration-based form
// State Phi_C = {T, [X_1], ..., [X_N]} of a constant-volume reactor: Sec. 3.3
// names this formulation (concentrations as state variables, no density in
// the cross-species elements) as the route to a sparse Jacobian, and Sec. 6
// plans it.  The rate laws are those of Sec. 2.3 evaluated at p = R T sum [X_k]
// (Eq. state); the ODE is
//   d[X_k]/dt = wdot_k,
//   dT/dt = -sum_k U_k wdot_k / sum_k [X_k] C_v,k,
// with molar internal energies U_k = H_k - R T and heat capacities
// C_v,k = C_p,k - R (Sec. 2.2 polynomials): energy conservation at constant
// volume.  Its Jacobian is the plain definition J = d f / d Phi_C.

template <class S> S make_state_conc(const Mech& m, const S& T, const S* C, State<S>& st) {
  const int N = m.N;
  st.N = N;
  st.T = T;
  st.X.assign(C, C + N);
  st.Xre.resize(N);
  for (int k = 0; k < N; ++k) st.Xre[k] = double(re(C[k]));
  st.cpR.resize(N); st.hRT.resize(N); st.sR.resize(N);
  thermo(m, T, st.cpR.data(), st.hRT.data(), st.sR.data());
  S sum = S(0);
  for (int k = 0; k < N; ++k) sum += C[k];
  return S(kR) * T * sum;                                          // p, Eq. (state)
}

template <class S> void rhs_conc(const Mech& m, const S& T, const S* C, S* f /* N + 1 */) {
  State<S> st;
  const S p = make_state_conc(m, T, C, st);
  const int N = m.N;
  std::vector<S> q(m.NR);
  RxnVals<S> v;
  for (int i = 0; i < m.NR; ++i) {
    reaction_values(m, i, st, p, v);
    q[i] = v.c * (v.Rf - v.Rr);
  }
  S num = S(0), den = S(0);
  for (int k = 0; k < N; ++k) {
    S w = S(0);
    for (int i : m.species_rxns[k]) w += S(m.nu(k, i)) * q[i];
    f[k + 1] = w;
    const S U = S(kR) * T * (st.hRT[k] - S(1));                   // molar internal energy
    const S Cv = S(kR) * (st.cpR[k] - S(1));                      // molar C_v
    num += U * w;
    den += C[k] * Cv;
  }
  f[0] = -num / den;
}

// d ln k_f / dT at fixed p and d ln k_f / d ln p of the forward rate coefficient
// (Sec. 2.3 Arrhenius, Sec. 2.3.4 PLOG and Chebyshev).  PLOG: ln k is linear in
// ln p inside a bracket (the last grid point p_n <= p), flat outside the grid;
// Chebyshev: d log10 k / d log10 p from the U-polynomial derivative of T_b.
void kf_log_derivs(const Rxn& r, double T, double p, double& dlnk_dT, double& dlnk_dlnp) {
  dlnk_dlnp = 0;
  switch (r.kind) {
    case ELEM: case THD: dlnk_dT = (r.arr.b + r.arr.Ta / T) / T; break;
    case FALLOFF: dlnk_dT = (r.high.b + r.high.Ta / T) / T; break;
    case CHEMACT: dlnk_dT = (r.low.b + r.low.Ta / T) / T; break;
    case PLOG: {
      const auto& pts = r.plog;
      const int n = (int)pts.size();
      auto lnk = [&](int q) { return std::log(pts[q][1]) + pts[q][2] * std::log(T) - pts[q][3] / T; };
      auto dlnk = [&](int q) { return (pts[q][2] + pts[q][3] / T) / T; };
      if (n == 1 || p <= pts[0][0]) dlnk_dT = dlnk(0);
      else if (p >= pts[n - 1][0]) dlnk_dT = dlnk(n - 1);
      else {
        int lo = 0;
        for (int q = 0; q < n - 1; ++q) if (pts[q][0] <= p) lo = q;
        const double w = (std::log(p) - std::log(pts[lo][0])) / (std::log(pts[lo + 1][0]) - std::log(pts[lo][0]));
        dlnk_dT = dlnk(lo) + (dlnk(lo + 1) - dlnk(lo)) * w;
        dlnk_dlnp = (lnk(lo + 1) - lnk(lo)) / (std::log(pts[lo + 1][0]) - std::log(pts[lo][0]));
      }
      break;
    }
    case CHEB: {
      const double span_T = 1 / r.Tmax - 1 / r.Tmin, span_p = std::log10(r.Pmax) - std::log10(r.Pmin);
      const double Tr = (2 / T - 1 / r.Tmin - 1 / r.Tmax) / span_T;
      const double pr = (2 * std::log10(p) - std::log10(r.Pmin) - std::log10(r.Pmax)) / span_p;
      std::vector<double> tT(r.nT), uT(r.nT), tP(r.nP), uP(r.nP);
      cheb_polys(r.nT, Tr, tT.data(), uT.data());
      cheb_polys(r.nP, pr, tP.data(), uP.data());
      double dT_sum = 0, dp_sum = 0;
      for (int a = 0; a < r.nT; ++a)
        for (int b = 0; b < r.nP; ++b) {
          const double eta = r.eta[a * r.nP + b];
          if (a > 0) dT_sum += eta * a * uT[a - 1] * tP[b];           // dT_a/dx = a U_{a-1}
          if (b > 0) dp_sum += eta * tT[a] * b * uP[b - 1];
        }
      dlnk_dT = kLn10 * dT_sum * (-2 / (T * T)) / span_T;
      dlnk_dlnp = dp_sum * 2 / span_p;                           // d log10 k / d log10 p
      break;
    }
  }
}

// J = d f / d Phi_C, (N+1) x (N+1) row-major: row 0 and column 0 are T, row and
// column k+1 the concentration of species k.  Element by element: per-reaction
// derivative vectors dq_i/dT and dq_i/d[X_j] from the product and chain rules,
// then each species row summed over its reactions, then the temperature row.
void jacobian_conc(const Mech& m, double T, const double* C, double* J) {
  const int N = m.N, NR = m.NR, N1 = N + 1;
  State<double> st;
  const double p = make_state_conc(m, T, C, st);
  double Msum = 0;
  for (int k = 0; k < N; ++k) Msum += C[k];
  // d ln p / dT = 1/T and d ln p / d[X_j] = 1/sum[X] at constant volume
  std::vector<double> dBdT(N);
  for (int k = 0; k < N; ++k) {
    const auto& a = (T <= m.tmid[k]) ? m.lo[k] : m.hi[k];
    dBdT[k] = (a[0] - 1 + a[5] / T) / T + a[1] / 2 + T * (a[2] / 3 + T * (a[3] / 4 + a[4] / 5 * T));
  }
  std::vector<double> dqdT(NR), dqdC((size_t)NR * N, 0.0), q(NR);
  for (int i = 0; i < NR; ++i) {
    const Rxn& r = m.rxn[i];
    RxnVals<double> x;
    reaction_values(m, i, st, p, x);
    q[i] = x.c * (x.Rf - x.Rr);
    double dlnkf_dT = 0, dlnkf_dlnp = 0;
    kf_log_derivs(r, T, p, dlnkf_dT, dlnkf_dlnp);
    const double dlnkf_dT_C = dlnkf_dT + dlnkf_dlnp / T;           // along constant concentrations
    double dkr_dT = 0, dkr_dlnp = 0;
    if (r.rev == KC) {
      double snu = 0;
      for (int k : m.rxn_species[i]) { int n = m.nu(k, i); if (n) snu += n * dBdT[k]; }
      dkr_dT = x.kr * (dlnkf_dT_C - snu);                            // K_c depends on T only
      dkr_dlnp = x.kr * dlnkf_dlnp;
    } else if (r.rev == EXPLICIT) {
      dkr_dT = x.kr * (r.revarr.b + r.revarr.Ta / T) / T;
    }
    double pf = 1, pr = 1;
    for (auto& [k, n] : r.reac) pf *= ipow(C[k], n);
    for (auto& [k, n] : r.prod) pr *= ipow(C[k], n);
    const double dRf_dT = x.kf * dlnkf_dT_C * pf, dRr_dT = dkr_dT * pr;
    // pressure modification
    double dcdT = 0, dPrdT = 0, dFdT = 0, dFdPr_over_F = 0;
    if (r.kind == FALLOFF || r.kind == CHEMACT) {
      const double dlnPrdT = (r.low.b - r.high.b + (r.low.Ta - r.high.Ta) / T) / T;   // [X]_i fixed
      dPrdT = x.Pr * dlnPrdT;
      blend_derivs(r, x, T, dPrdT, dFdT, dFdPr_over_F);
      if (r.kind == FALLOFF) dcdT = x.c * (dlnPrdT / (1 + x.Pr) + dFdT / x.F);
      else dcdT = x.c * (-dPrdT / (1 + x.Pr) + dFdT / x.F);
    }
    dqdT[i] = dcdT * (x.Rf - x.Rr) + x.c * (dRf_dT - dRr_dT);
    double* dq = &dqdC[(size_t)i * N];
    for (int j = 0; j < N; ++j) {
      // d[X]_i / d[X_j]
      double dE = 0;
      if (r.kind == THD || r.kind == FALLOFF || r.kind == CHEMACT)
        dE = r.collider_species ? (j == r.m ? 1.0 : 0.0) : r.alpha[j];
      double dc = 0;
      if (r.kind == THD) dc = dE;
      else if (r.kind == FALLOFF || r.kind == CHEMACT) {
        const double dPr = x.k0 / x.kinf * dE;
        if (r.kind == FALLOFF) dc = x.F / ((1 + x.Pr) * (1 + x.Pr)) * dPr + x.c * dFdPr_over_F * dPr;
        else dc = x.c * (-dPr / (1 + x.Pr) + dFdPr_over_F * dPr);
      }
      // dR/d[X_j]: mass-action product rule plus the pressure dependence of k
      double dpf = 0, dpr = 0;
      for (auto& [k, n] : r.reac)
        if (k == j) {
          double other = 1;
          for (auto& [l, nl] : r.reac) if (l != k) other *= ipow(C[l], nl);
          dpf = n * ipow(C[k], n - 1) * other;
        }
      for (auto& [k, n] : r.prod)
        if (k == j) {
          double other = 1;
          for (auto& [l, nl] : r.prod) if (l != k) other *= ipow(C[l], nl);
          dpr = n * ipow(C[k], n - 1) * other;
        }
      const double dRf = x.kf * dlnkf_dlnp / Msum * pf + x.kf * dpf;
      const double dRr = dkr_dlnp / Msum * pr + x.kr * dpr;
      dq[j] = dc * (x.Rf - x.Rr) + x.c * (dRf - dRr);
    }
  }
  std::vector<double> wdot(N, 0.0), U(N), Cv(N), dCv(N);
  for (int k = 0; k < N; ++k) {
    for (int i : m.species_rxns[k]) wdot[k] += m.nu(k, i) * q[i];
    const auto& a = (T <= m.tmid[k]) ? m.lo[k] : m.hi[k];
    U[k] = kR * T * (st.hRT[k] - 1);
    Cv[k] = kR * (st.cpR[k] - 1);
    dCv[k] = kR * (a[1] + T * (2 * a[2] + T * (3 * a[3] + 4 * a[4] * T)));
  }
  // species rows
  for (int k = 0; k < N; ++k) {
    double acc = 0;
    for (int i : m.species_rxns[k]) acc += m.nu(k, i) * dqdT[i];
    J[(size_t)(k + 1) * N1] = acc;
    for (int j = 0; j < N; ++j) {
      double s = 0;
      for (int i : m.species_rxns[k]) s += m.nu(k, i) * dqdC[(size_t)i * N + j];
      J[(size_t)(k + 1) * N1 + j + 1] = s;
    }
  }
  // temperature row: f_0 = -num / den, num = sum U_k wdot_k, den = sum [X_k] C_v,k;
  // dU_k/dT = C_v,k
  double num = 0, den = 0, dden_dT = 0;
  for (int k = 0; k < N; ++k) { num += U[k] * wdot[k]; den += C[k] * Cv[k]; dden_dT += C[k] * dCv[k]; }
  {
    double dnum = 0;
    for (int k = 0; k < N; ++k) dnum += Cv[k] * wdot[k] + U[k] * J[(size_t)(k + 1) * N1];
    J[0] = -dnum / den + num * dden_dT / (den * den);
  }
  for (int j = 0; j < N; ++j) {
    double dnum = 0;
    for (int k = 0; k < N; ++k) dnum += U[k] * J[(size_t)(k + 1) * N1 + j + 1];
    J[j + 1] = -dnum / den + num * Cv[j] / (den * den);
  }
}

int nthreads_or_default(int nt) {
#ifdef _OPENMP
  return nt > 0 ? nt : omp_get_max_threads();
#else
  (void)nt; return 1;
#endif
}

Mech* as_mech(void* h) { return static_cast<Mech*>(h); }

}  // namespace

extern "C" {

const char* pyjac_ref_last_error(void) { return g_err.c_str(); }

int pyjac_ref_mech_load_string(const char* text, void** out) {
  try {
    if (!text || !out) { g_err = "null argument"; return -1; }
    *out = new Mech(parse(text));
    return 0;
  } catch (const std::exception& e) { g_err = e.what(); return -2; }
}

int pyjac_ref_mech_load(const char* path, void** out) {
  if (!path) { g_err = "null path"; return -1; }
  std::ifstream f(path);
  if (!f) { g_err = std::string("cannot open ") + path; return -6; }
  std::stringstream ss; ss << f.rdbuf();
  return pyjac_ref_mech_load_string(ss.str().c_str(), out);
}

void pyjac_ref_mech_free(void* h) { delete as_mech(h); }

int pyjac_ref_mech_info(void* h, int* n_species, int* n_reactions) {
  if (!h) return -1;
  if (n_species) *n_species = as_mech(h)->N;
  if (n_reactions) *n_reactions = as_mech(h)->NR;
  return 0;
}

// Rates and RHS for n states; layout e*ld + s.  Any output may be NULL.
int pyjac_ref_eval_rates(void* h, int64_t n, int64_t ld, const double* phi, const double* p,
                         double* rop_f, double* rop_r, double* pres_mod, double* wdot, double* dphi,
                         int nthreads) {
  if (!h || !phi || !p || n < 0 || ld < n) { g_err = "bad argument"; return -1; }
  const Mech& m = *as_mech(h);
  const int N = m.N, NR = m.NR;
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads_or_default(nthreads))
  for (int64_t s = 0; s < n; ++s) {
    std::vector<double> y(N - 1), w(N), f(N), rf(NR), rr(NR), pm(NR);
    for (int j = 0; j < N - 1; ++j) y[j] = phi[(j + 1) * ld + s];
    rhs<double>(m, phi[s], p[s], y.data(), w.data(), f.data(), rf.data(), rr.data(), pm.data());
    for (int i = 0; i < NR; ++i) {
      if (rop_f) rop_f[i * ld + s] = rf[i];
      if (rop_r) rop_r[i * ld + s] = rr[i];
      if (pres_mod) pres_mod[i * ld + s] = pm[i];
    }
    for (int k = 0; k < N; ++k) {
      if (wdot) wdot[k * ld + s] = w[k];
      if (dphi) dphi[k * ld + s] = f[k];
    }
  }
  return 0;
}

// RHS in extended precision (long double) for finite-difference references.
int pyjac_ref_eval_rhs_ld(void* h, int64_t n, int64_t ld, const long double* phi, const double* p,
                          long double* dphi, int nthreads) {
  if (!h || !phi || !p || !dphi || n < 0 || ld < n) { g_err = "bad argument"; return -1; }
  const Mech& m = *as_mech(h);
  const int N = m.N;
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads_or_default(nthreads))
  for (int64_t s = 0; s < n; ++s) {
    std::vector<long double> y(N - 1), w(N), f(N);
    for (int j = 0; j < N - 1; ++j) y[j] = phi[(j + 1) * ld + s];
    rhs<long double>(m, phi[s], p[s], y.data(), w.data(), f.data(), nullptr, nullptr, nullptr);
    for (int k = 0; k < N; ++k) dphi[k * ld + s] = f[k];
  }
  return 0;
}

// Analytical Jacobian, layout jac[(i*N + j)*ld + s].
int pyjac_ref_eval_jacobian(void* h, int64_t n, int64_t ld, const double* phi, const double* p,
                            double* jac, int nthreads) {
  if (!h || !phi || !p || !jac || n < 0 || ld < n) { g_err = "bad argument"; return -1; }
  const Mech& m = *as_mech(h);
  const int N = m.N;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads_or_default(nthreads))
  for (int64_t s = 0; s < n; ++s) {
    std::vector<double> y(N - 1), J((size_t)N * N);
    for (int j = 0; j < N - 1; ++j) y[j] = phi[(j + 1) * ld + s];
    jacobian(m, phi[s], p[s], y.data(), J.data());
    for (size_t e = 0; e < (size_t)N * N; ++e) jac[e * ld + s] = J[e];
  }
  return 0;
}

// Complex-step Jacobian of the RHS: column j = Im f(Phi + i h e_j) / h.
int pyjac_ref_eval_jacobian_cs(void* h, int64_t n, int64_t ld, const double* phi, const double* p,
                               double* jac, double step, int nthreads) {
  if (!h || !phi || !p || !jac || n < 0 || ld < n || !(step > 0)) { g_err = "bad argument"; return -1; }
  const Mech& m = *as_mech(h);
  const int N = m.N;
  using C = std::complex<double>;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads_or_default(nthreads))
  for (int64_t s = 0; s < n; ++s) {
    std::vector<C> y(N - 1), w(N), f(N);
    for (int col = 0; col < N; ++col) {
      C T(phi[s], col == 0 ? step : 0.0);
      for (int j = 0; j < N - 1; ++j) y[j] = C(phi[(j + 1) * ld + s], (col == j + 1) ? step : 0.0);
      rhs<C>(m, T, p[s], y.data(), w.data(), f.data(), nullptr, nullptr, nullptr);
      for (int row = 0; row < N; ++row) jac[((size_t)row * N + col) * ld + s] = f[row].imag() / step;
    }
  }
  return 0;
}

// Constant-volume, concentration-based form: phi_c [(N+1)][ld] holds T and
// [X_1..X_N]; f [(N+1)][ld]; jac [(N+1)^2][ld] row-major per state.
int pyjac_ref_eval_rhs_conc(void* h, int64_t n, int64_t ld, const double* phi_c, double* f, int nthreads) {
  if (!h || !phi_c || !f || n < 0 || ld < n) { g_err = "bad argument"; return -1; }
  const Mech& m = *as_mech(h);
  const int N1 = m.N + 1;
#pragma omp parallel for schedule(dynamic, 8) num_threads(nthreads_or_default(nthreads))
  for (int64_t s = 0; s < n; ++s) {
    std::vector<double> C(m.N), out(N1);
    for (int k = 0; k < m.N; ++k) C[k] = phi_c[(k + 1) * ld + s];
    rhs_conc<double>(m, phi_c[s], C.data(), out.data());
    for (int e = 0; e < N1; ++e) f[e * ld + s] = out[e];
  }
  return 0;
}

int pyjac_ref_eval_jacobian_conc(void* h, int64_t n, int64_t ld, const double* phi_c, double* jac, int nthreads) {
  if (!h || !phi_c || !jac || n < 0 || ld < n) { g_err = "bad argument"; return -1; }
  const Mech& m = *as_mech(h);
  const size_t N1 = m.N + 1;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads_or_default(nthreads))
  for (int64_t s = 0; s < n; ++s) {
    std::vector<double> C(m.N), J(N1 * N1);
    for (int k = 0; k < m.N; ++k) C[k] = phi_c[(k + 1) * ld + s];
    jacobian_conc(m, phi_c[s], C.data(), J.data());
    for (size_t e = 0; e < N1 * N1; ++e) jac[e * ld + s] = J[e];
  }
  return 0;
}

int pyjac_ref_eval_jacobian_conc_cs(void* h, int64_t n, int64_t ld, const double* phi_c, double* jac, double step,
                                    int nthreads) {
  if (!h || !phi_c || !jac || n < 0 || ld < n || !(step > 0)) { g_err = "bad argument"; return -1; }
  const Mech& m = *as_mech(h);
  const int N1 = m.N + 1;
  using Cx = std::complex<double>;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nthreads_or_default(nthreads))
  for (int64_t s = 0; s < n; ++s) {
    std::vector<Cx> C(m.N), f(N1);
    for (int col = 0; col < N1; ++col) {
      Cx T(phi_c[s], col == 0 ? step : 0.0);
      for (int k = 0; k < m.N; ++k) C[k] = Cx(phi_c[(k + 1) * ld + s], (col == k + 1) ? step : 0.0);
      rhs_conc<Cx>(m, T, C.data(), f.data());
      for (int row = 0; row < N1; ++row) jac[((size_t)row * N1 + col) * ld + s] = f[row].imag() / step;
    }
  }
  return 0;
}

// Per-species NASA-7 values at one temperature (for formula pins).
int pyjac_ref_species_thermo(void* h, double T, double* cpR, double* hRT, double* sR) {
  if (!h) return -1;
  thermo<double>(*as_mech(h), T, cpR, hRT, sR);
  return 0;
}

// Per-reaction intermediate values at one state (for formula pins).
// out arrays of length NR: kf, kr, c, Rf, Rr, Kc, Pr, F.  Any may be NULL.
int pyjac_ref_reaction_terms(void* h, double T, double p, const double* y, double* kf, double* kr,
                             double* c, double* Rf, double* Rr, double* Kc, double* Pr, double* F) {
  if (!h || !y) return -1;
  const Mech& m = *as_mech(h);
  State<double> st;
  make_state(m, T, p, y, st);
  RxnVals<double> v;
  for (int i = 0; i < m.NR; ++i) {
    reaction_values(m, i, st, p, v);
    if (kf) kf[i] = v.kf;
    if (kr) kr[i] = v.kr;
    if (c) c[i] = v.c;
    if (Rf) Rf[i] = v.Rf;
    if (Rr) Rr[i] = v.Rr;
    if (Kc) Kc[i] = v.Kc;
    if (Pr) Pr[i] = v.Pr;
    if (F) F[i] = v.F;
  }
  return 0;
}

}  // extern "C"
