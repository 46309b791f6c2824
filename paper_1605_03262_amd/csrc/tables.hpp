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

inline int rinfo_kind(int v) { return v & 0xF; }

// Everything one reaction needs, in one 256-byte record so that a lane fetches
// it with independent wide loads before any branch (sorted reaction order).
struct alignas(16) RxnRec {
  int info, sum_f, sum_r, gslot;          // class/flags, sum nu', sum nu'', G slot or -1
  int mol[2 * kMaxSide];                  // reactant then product molecules (species index,
                                          // repeated per unit of nu); N = none (X[N] = 1)
  int net[kMaxNet];                       // sp | nu << 16 (nu signed), -1 = none
  int coll_m, aux0, aux1, orig;           // collider species; efficiency or PLOG range or
                                          // Chebyshev offset; file index of the reaction
  double dnu_lnpr, alphaN_m1;             // sum(nu) ln(p_atm/R); alpha_N - 1
  double arr[kArrStride];
  double fpar[kFparStride];
  double frcp[2];                         // Troe 1/T***, 1/T*; SRI 1/c (fpar[2])
  double pad[4];
};
static_assert(sizeof(RxnRec) == 256, "RxnRec must stay 256 bytes");

// One entry of a Jacobian column stream.  Every entry contributes
// coef * X[src] * X[x & 0x7FFF] * X[(x >> 15) & 0x7FFF] to the current element,
// where X[0..N] are the concentrations (X[N] = 1) and the rate products P
// follow directly, so src = N + 1 + (index into P).  An entry with bit
// kColMark set in x ends a row after its own contribution; a marker is such an
// entry with coef = 0; padding has coef = 0 and src = N.  Two forms:
//  * every row (col_split = 0): for rows k = 0..N-1 in order, the terms of
//    (k, j); for k < N - 1 the row's last term carries the mark, and a row
//    without terms is a marker (src = N) alone (the placeholder row N - 1 is
//    finished after the stream); padding to a multiple of kColBatch.
//  * present rows only (col_split = 1): bit k of the column's col_flags words
//    marks row k as present (streamed); the other rows hold the dense part
//    alone.  The stream is a marker, then for each present row in ascending
//    order its terms and a marker, padded to a multiple of 2 kColBatch; a
//    marker's src is the next present row (N after the last): it ends the open
//    row and opens that one.
// The loader takes the second form when most (row, column) pairs have no
// terms (large mechanisms), where it saves a marker per empty row.
struct alignas(16) ColRec {
  double coef;
  int src, x;
};
constexpr int kColMark = 1 << 30;
constexpr int kColBatch = 4;

// Every-row form: a column's stream may be cut at row boundaries into
// segments that separate groups stream.  Segment: rows [k0, ...) of column j,
// records [rec, rec + cnt) (cnt a multiple of kColBatch); last = 1 when it
// holds the placeholder row N - 1.  slot < 0: the column is one segment and
// its temperature-row element is finished at once; otherwise the partial
// temperature-row sum goes to that slot and the column's ColJoin adds its
// nslot slots (slot0 ...) in row order.
struct alignas(16) ColItem {
  int j, k0, rec, cnt, slot, last, pad0, pad1;
};
struct alignas(16) ColJoin {
  int j, slot0, nslot, pad;
};

// Host-side packed tables (sorted reaction order).
struct PackedMech {
  int N = 0, NR = 0, NG = 0;
  uint64_t hash = 0;
  std::vector<double> W, invW, nasa, tmid, vcol;          // species
  std::vector<RxnRec> rx;
  std::vector<int> eff_sp;
  std::vector<double> eff_am1;
  std::vector<double> plog;                               // (ln p, ln A, b, Ta) per point
  std::vector<double> cheb;                               // nT, nP, c1, c0, pc1, pc0, eta...
  std::vector<int> spg_ptr, spg_ent;                      // per-species reaction lists:
                                                          // slot | nu << 16 (nu signed)
  std::vector<int> col_start;                             // [N] stream offsets per column
  std::vector<ColRec> colrec;
  std::vector<int> col_order;                             // [N-1] columns, longest stream first
  std::vector<ColItem> col_item;                          // every-row form: segments, longest first
  std::vector<ColJoin> col_join;                          // every-row form: columns in several segments
  std::vector<uint32_t> col_flags;                        // [N-1][colFlagWords(N)] present rows
  int col_split = 0;                                      // column-stream form (see ColRec)
  // Concentration-based, constant-volume Jacobian: species block
  // J[k][j] = u_k + S[k][j] with S sparse.  Per species column j (all N):
  // a present-rows stream (as col_split = 1, without the dense pass; coef
  // without molecular-weight ratios, every species a state variable) and
  // the compressed-column pattern of S (rows with terms, ascending).
  std::vector<int> cv_col_start;                          // [N + 1]
  std::vector<ColRec> cv_colrec;
  std::vector<int> cv_col_order;                          // [N] longest stream first
  std::vector<int> cv_colptr, cv_rowidx;                  // [N + 1], [nnz]
};

constexpr int colFlagWords(int N) { return (N + 31) / 32; }

// Per-chunk bounds of the species reaction lists for reaction chunks of size
// `chunk`: entry [c * N + k] is the first list index of species k whose
// reaction slot is >= c * chunk; there are ceil(NR / chunk) + 1 rows.
std::vector<int> species_chunk_bounds(const PackedMech& P, int chunk);

// Parse + validate + pack.  Returns 0 or a PYJAC_E_* code with msg set.
int build_tables(const std::string& text, PackedMech& out, std::string& msg);

// Device view (all pointers into one device allocation).
struct MechDev {
  int N, NR, NG;
  int col_split;                        // column-stream form (see ColRec)
  const double* __restrict__ W;
  const double* __restrict__ invW;
  const double* __restrict__ nasa;      // [N][2][7]
  const double* __restrict__ tmid;
  const double* __restrict__ vcol;      // [N-1]
  const RxnRec* __restrict__ rx;        // [NR]
  const int* __restrict__ eff_sp;
  const double* __restrict__ eff_am1;
  const double* __restrict__ plog;
  const double* __restrict__ cheb;
  const int* __restrict__ spg_ent;
  const int* __restrict__ spg_chunk;    // species_chunk_bounds for the launch's chunk size
  const int* __restrict__ col_start;    // [N]
  const ColRec* __restrict__ colrec;
  const int* __restrict__ col_order;    // [N-1] longest column stream first
  const ColItem* __restrict__ col_item; // [n_col_item] every-row form, longest first
  const ColJoin* __restrict__ col_join; // [n_col_join]
  int n_col_item, n_col_join;
  const uint32_t* __restrict__ col_flags;  // [N-1][colFlagWords(N)]
  const int* __restrict__ cv_col_start;    // [N + 1]
  const ColRec* __restrict__ cv_colrec;
  const int* __restrict__ cv_col_order;    // [N]
  const int* __restrict__ cv_colptr;       // [N + 1]
};

// One batch of a multi-mechanism work-list launch:
// the mechanism's device view (with the species-list chunk bounds of the
// launch shape), the batch's arrays and size, and its first tile in the grid.
struct WorkItem {
  MechDev md;
  const double* phi;
  const double* p;
  double* jac;
  int64_t n, ld, tile0;
};
// The work list travels as a kernel argument (no device copy, so a launch can
// be captured into a graph as is): at most kMaxWorkItems batches per launch.
constexpr int kMaxWorkItems = 8;
struct WorkList {
  WorkItem item[kMaxWorkItems];
  int n_items;
};

}  // namespace pyjac
