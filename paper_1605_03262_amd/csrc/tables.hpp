// Mechanism tables of the MI355X library: host-side packing result and the
// device view passed to the kernels by value.
//
// Reactions are stored in a sorted order (by rate class, falloff blending,
// collider kind and reverse treatment) so that lanes evaluating neighbouring
// reactions take the same branches; rorig maps a sorted slot back to the
// mechanism file's reaction index for the per-reaction outputs.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace pyjac {

constexpr double kGasConstant = 8314.462618;   // J / (kmol K), exact SI value
constexpr double kOneAtm = 101325.0;           // Pa

// reaction class codes (low 4 bits of rinfo)
enum : int { K_ELEM = 0, K_THD = 1, K_FALLOFF = 2, K_CHEMACT = 3, K_PLOG = 4, K_CHEB = 5 };
// blending (bits 4..7)
enum : int { B_NONE = 0, B_LIND = 1, B_TROE = 2, B_SRI = 3 };
// reverse treatment (bits 8..11)
enum : int { R_KC = 0, R_EXPLICIT = 1, R_IRREV = 2 };
// collider (bits 12..15)
enum : int { C_NONE = 0, C_UNITY = 1, C_EFF = 2, C_SPECIES = 3 };
// flags (bits 16..)
constexpr int F_LAST_SPECIES = 1 << 16;   // the last species (index N-1) takes part
constexpr int F_TROE_T2 = 1 << 17;        // Troe with the optional T** term

constexpr int kMaxSide = 3;     // distinct species per side
constexpr int kMaxNet = 6;      // species with nonzero net coefficient
constexpr int kArrStride = 9;   // primary (A,b,Ta), secondary (ratio A, db, dTa), reverse (A,b,Ta)
constexpr int kFparStride = 5;
constexpr int kSideStride = 2 * kMaxSide;   // (species, nu) pairs packed as sp | nu << 16
constexpr int kNetStride = kMaxNet;

inline int rinfo_kind(int v) { return v & 0xF; }

// Host-side packed tables (sorted reaction order).
struct PackedMech {
  int N = 0, NR = 0, NG = 0;
  uint64_t hash = 0;
  std::vector<double> W, invW, nasa, tmid, vcol;          // species
  std::vector<int> rinfo, rorig, side, net, coll_m, gslot, sum_f, sum_r;
  std::vector<double> arr, fpar, dnu_lnpr, alphaN_m1;
  std::vector<int> eff_ptr, eff_sp;
  std::vector<double> eff_am1;
  std::vector<int> plog_ptr;
  std::vector<double> plog;                               // (ln p, ln A, b, Ta) per point
  std::vector<int> cheb_off;
  std::vector<double> cheb;                               // nT, nP, c1, c0, pc1, pc0, eta...
  std::vector<int> spg_ptr, spg_rxn;                      // per-species reaction lists
  std::vector<double> spg_nu;
  std::vector<int> col_ptr, term_src, term_x;             // Jacobian column terms
  std::vector<double> term_coef;
};

// Parse + validate + pack.  Returns 0 or a PYJAC_E_* code with msg set.
int build_tables(const std::string& text, PackedMech& out, std::string& msg);

// Device view (all pointers into one device allocation).
struct MechDev {
  int N, NR, NG;
  const double* __restrict__ W;
  const double* __restrict__ invW;
  const double* __restrict__ nasa;      // [N][2][7]
  const double* __restrict__ tmid;
  const double* __restrict__ vcol;      // [N-1]
  const int* __restrict__ rinfo;
  const int* __restrict__ rorig;
  const int* __restrict__ side;         // [NR][6]
  const int* __restrict__ net;          // [NR][6]
  const int* __restrict__ coll_m;
  const int* __restrict__ gslot;
  const int* __restrict__ sum_f;
  const int* __restrict__ sum_r;
  const double* __restrict__ arr;       // [NR][9]
  const double* __restrict__ fpar;      // [NR][5]
  const double* __restrict__ dnu_lnpr;  // sum(nu) * ln(p_atm / R)
  const double* __restrict__ alphaN_m1;
  const int* __restrict__ eff_ptr;
  const int* __restrict__ eff_sp;
  const double* __restrict__ eff_am1;
  const int* __restrict__ plog_ptr;
  const double* __restrict__ plog;
  const int* __restrict__ cheb_off;
  const double* __restrict__ cheb;
  const int* __restrict__ spg_ptr;
  const int* __restrict__ spg_rxn;
  const double* __restrict__ spg_nu;
  const int* __restrict__ col_ptr;      // [(N-1)*N + 1]
  const int* __restrict__ term_src;
  const int* __restrict__ term_x;       // x1 | x2 << 16 (index N means "1")
  const double* __restrict__ term_coef;
};

}  // namespace pyjac
