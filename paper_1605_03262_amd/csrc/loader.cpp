// Mechanism text -> packed device tables (host code of libpyjac_mi355x).
//
// The text format is token based ('#' starts a comment):
//   pyjac-mech 1
//   elements <n>  (<symbol> <atomic weight>)*n
//   species <n>   (<name> <W> <T_mid> <n_el> (<el> <count>)*n_el <7 low a> <7 high a>)*n
//   reactions <n> (reaction <class> <reverse> <keyword blocks>)*n
//   end
// Reaction classes: elementary thirdbody falloff chemact plog cheb; reverse
// treatments: kc explicit irrev.  Keyword blocks: reactants/products <n>
// (<species> <nu>)*n, arrhenius A b Ta, low/high A b Ta (falloff/chemact),
// lindemann | troe <3|4> a T*** T* [T**] | sri <3|5> a b c [d e],
// collider mix <n> (<species> <alpha>)* | collider species <name>,
// plog <n> (p A b Ta)*n, cheb nT nP Tmin Tmax Pmin Pmax eta(nT*nP),
// reverse A b Ta.  SI-kmol units; Ta is the activation temperature in K.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <numeric>
#include <sstream>
#include <stdexcept>

#include "../../include/pyjac.h"
#include "tables.hpp"

namespace pyjac {
namespace {

struct LoadError : std::runtime_error {
  int code;
  LoadError(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

class Reader {
 public:
  explicit Reader(const std::string& text) {
    size_t i = 0, n = text.size();
    while (i < n) {
      char ch = text[i];
      if (ch == '#') { while (i < n && text[i] != '\n') ++i; continue; }
      if (std::isspace(static_cast<unsigned char>(ch))) { ++i; continue; }
      size_t j = i;
      while (j < n && !std::isspace(static_cast<unsigned char>(text[j])) && text[j] != '#') ++j;
      toks_.emplace_back(text, i, j - i);
      i = j;
    }
  }
  bool at_end() const { return pos_ >= toks_.size(); }
  const std::string& look() const {
    if (at_end()) throw LoadError(PYJAC_E_PARSE, "mechanism text ends early");
    return toks_[pos_];
  }
  std::string word() { std::string w = look(); ++pos_; return w; }
  void keyword(const char* k) {
    std::string w = word();
    if (w != k) throw LoadError(PYJAC_E_PARSE, std::string("expected '") + k + "' but found '" + w + "'");
  }
  double real() {
    std::string w = word();
    char* e = nullptr;
    double v = std::strtod(w.c_str(), &e);
    if (e == w.c_str() || *e != '\0' || !std::isfinite(v))
      throw LoadError(PYJAC_E_PARSE, "bad number '" + w + "'");
    return v;
  }
  long count() {
    std::string w = word();
    char* e = nullptr;
    long v = std::strtol(w.c_str(), &e, 10);
    if (e == w.c_str() || *e != '\0') throw LoadError(PYJAC_E_PARSE, "bad integer '" + w + "'");
    return v;
  }

 private:
  std::vector<std::string> toks_;
  size_t pos_ = 0;
};

struct Arrh { double A = 0, b = 0, Ta = 0; bool set = false; };

struct RawRxn {
  int cls = K_ELEM, rev = R_KC, blend = B_NONE, coll = C_NONE, m = -1;
  std::vector<std::pair<int, int>> reac, prod;
  Arrh arr, low, high, revr;
  std::vector<double> troe, sri;
  std::map<int, double> eff;
  std::vector<std::array<double, 4>> plog;
  int nT = 0, nP = 0;
  double Tmin = 0, Tmax = 0, Pmin = 0, Pmax = 0;
  std::vector<double> eta;
  int file_index = 0;
};

struct RawMech {
  std::vector<std::string> elements;
  std::vector<std::string> names;
  std::vector<double> W, tmid;
  std::vector<std::array<double, 14>> nasa;
  std::vector<std::vector<int>> comp;      // [species][element]
  std::vector<RawRxn> rxn;
};

Arrh read_arrh(Reader& rd) { Arrh a; a.A = rd.real(); a.b = rd.real(); a.Ta = rd.real(); a.set = true; return a; }

RawMech read_mech(const std::string& text) {
  Reader rd(text);
  RawMech m;
  rd.keyword("pyjac-mech");
  if (rd.count() != 1) throw LoadError(PYJAC_E_UNSUPPORTED, "mechanism format version is not 1");
  rd.keyword("elements");
  long ne = rd.count();
  if (ne < 1) throw LoadError(PYJAC_E_PARSE, "no elements");
  for (long e = 0; e < ne; ++e) { m.elements.push_back(rd.word()); rd.real(); }
  rd.keyword("species");
  long ns = rd.count();
  if (ns < 2) throw LoadError(PYJAC_E_UNSUPPORTED, "at least two species are required");
  std::map<std::string, int> sidx;
  for (long k = 0; k < ns; ++k) {
    std::string name = rd.word();
    if (sidx.count(name)) throw LoadError(PYJAC_E_PARSE, "species '" + name + "' defined twice");
    sidx[name] = (int)k;
    m.names.push_back(name);
    double W = rd.real(), tm = rd.real();
    if (!(W > 0) || !(tm > 0)) throw LoadError(PYJAC_E_PARSE, "species '" + name + "': W and T_mid must be positive");
    m.W.push_back(W);
    m.tmid.push_back(tm);
    std::vector<int> comp(m.elements.size(), 0);
    long nc = rd.count();
    for (long c = 0; c < nc; ++c) {
      std::string el = rd.word();
      long cnt = rd.count();
      auto it = std::find(m.elements.begin(), m.elements.end(), el);
      if (it == m.elements.end()) throw LoadError(PYJAC_E_PARSE, "species '" + name + "' uses undeclared element " + el);
      comp[it - m.elements.begin()] += (int)cnt;
    }
    m.comp.push_back(comp);
    std::array<double, 14> a{};
    for (auto& v : a) v = rd.real();
    m.nasa.push_back(a);
  }
  auto species = [&](const std::string& s) {
    auto it = sidx.find(s);
    if (it == sidx.end()) throw LoadError(PYJAC_E_PARSE, "unknown species '" + s + "'");
    return it->second;
  };
  rd.keyword("reactions");
  long nr = rd.count();
  if (nr < 1) throw LoadError(PYJAC_E_UNSUPPORTED, "no reactions");
  for (long i = 0; i < nr; ++i) {
    rd.keyword("reaction");
    RawRxn r;
    r.file_index = (int)i;
    std::string cls = rd.word(), rev = rd.word();
    static const std::map<std::string, int> cls_map = {
        {"elementary", K_ELEM}, {"thirdbody", K_THD}, {"falloff", K_FALLOFF},
        {"chemact", K_CHEMACT}, {"plog", K_PLOG}, {"cheb", K_CHEB}};
    static const std::map<std::string, int> rev_map = {{"kc", R_KC}, {"explicit", R_EXPLICIT}, {"irrev", R_IRREV}};
    if (!cls_map.count(cls)) throw LoadError(PYJAC_E_UNSUPPORTED, "reaction class '" + cls + "'");
    if (!rev_map.count(rev)) throw LoadError(PYJAC_E_UNSUPPORTED, "reverse treatment '" + rev + "'");
    r.cls = cls_map.at(cls);
    r.rev = rev_map.at(rev);
    while (!rd.at_end() && rd.look() != "reaction" && rd.look() != "end") {
      std::string kw = rd.word();
      if (kw == "reactants" || kw == "products") {
        long n = rd.count();
        auto& side = (kw == "reactants") ? r.reac : r.prod;
        for (long c = 0; c < n; ++c) {
          int k = species(rd.word());
          long nu = rd.count();
          if (nu < 1) throw LoadError(PYJAC_E_UNSUPPORTED, "stoichiometric coefficients must be positive integers");
          auto it = std::find_if(side.begin(), side.end(), [&](const std::pair<int, int>& q) { return q.first == k; });
          if (it != side.end()) it->second += (int)nu; else side.push_back({k, (int)nu});
        }
      } else if (kw == "arrhenius") r.arr = read_arrh(rd);
      else if (kw == "low") r.low = read_arrh(rd);
      else if (kw == "high") r.high = read_arrh(rd);
      else if (kw == "reverse") r.revr = read_arrh(rd);
      else if (kw == "lindemann") r.blend = B_LIND;
      else if (kw == "troe") {
        r.blend = B_TROE;
        long n = rd.count();
        if (n != 3 && n != 4) throw LoadError(PYJAC_E_UNSUPPORTED, "Troe needs 3 or 4 parameters");
        for (long c = 0; c < n; ++c) r.troe.push_back(rd.real());
      } else if (kw == "sri") {
        r.blend = B_SRI;
        long n = rd.count();
        if (n != 3 && n != 5) throw LoadError(PYJAC_E_UNSUPPORTED, "SRI needs 3 or 5 parameters");
        for (long c = 0; c < n; ++c) r.sri.push_back(rd.real());
      } else if (kw == "collider") {
        std::string how = rd.word();
        if (how == "mix") {
          long n = rd.count();
          for (long c = 0; c < n; ++c) { int k = species(rd.word()); r.eff[k] = rd.real(); }
          r.coll = C_UNITY;
          for (auto& [k, a] : r.eff) if (a != 1.0) r.coll = C_EFF;
        } else if (how == "species") {
          r.coll = C_SPECIES;
          r.m = species(rd.word());
        } else throw LoadError(PYJAC_E_UNSUPPORTED, "collider kind '" + how + "'");
      } else if (kw == "plog") {
        long n = rd.count();
        for (long c = 0; c < n; ++c) {
          std::array<double, 4> q{};
          for (auto& v : q) v = rd.real();
          r.plog.push_back(q);
        }
      } else if (kw == "cheb") {
        r.nT = (int)rd.count(); r.nP = (int)rd.count();
        r.Tmin = rd.real(); r.Tmax = rd.real(); r.Pmin = rd.real(); r.Pmax = rd.real();
        if (r.nT < 1 || r.nP < 1 || r.nT > 16 || r.nP > 16)
          throw LoadError(PYJAC_E_UNSUPPORTED, "Chebyshev grid must be 1..16 x 1..16");
        for (int c = 0; c < r.nT * r.nP; ++c) r.eta.push_back(rd.real());
      } else throw LoadError(PYJAC_E_PARSE, "unknown reaction keyword '" + kw + "'");
    }
    m.rxn.push_back(std::move(r));
  }
  rd.keyword("end");
  return m;
}

void validate(const RawMech& m) {
  const int N = (int)m.names.size();
  for (size_t i = 0; i < m.rxn.size(); ++i) {
    const RawRxn& r = m.rxn[i];
    std::string tag = "reaction " + std::to_string(i) + ": ";
    if (r.reac.empty() || r.prod.empty()) throw LoadError(PYJAC_E_UNSUPPORTED, tag + "needs reactants and products");
    if ((int)r.reac.size() > kMaxSide || (int)r.prod.size() > kMaxSide)
      throw LoadError(PYJAC_E_UNSUPPORTED, tag + "more than 3 distinct species on a side");
    int mf = 0, mr = 0;
    for (auto& q : r.reac) mf += q.second;
    for (auto& q : r.prod) mr += q.second;
    if (mf > 3 || mr > 3) throw LoadError(PYJAC_E_UNSUPPORTED, tag + "more than 3 molecules on a side");
    for (size_t e = 0; e < m.elements.size(); ++e) {
      long bal = 0;
      for (auto& q : r.reac) bal -= (long)q.second * m.comp[q.first][e];
      for (auto& q : r.prod) bal += (long)q.second * m.comp[q.first][e];
      if (bal != 0) throw LoadError(PYJAC_E_UNBALANCED, tag + "element " + m.elements[e] + " is not conserved");
    }
    int nnet = 0;
    for (int k = 0; k < N; ++k) {
      int nu = 0;
      for (auto& q : r.reac) if (q.first == k) nu -= q.second;
      for (auto& q : r.prod) if (q.first == k) nu += q.second;
      if (nu) ++nnet;
    }
    if (nnet > kMaxNet) throw LoadError(PYJAC_E_UNSUPPORTED, tag + "too many species");
    bool pdep = (r.cls == K_THD || r.cls == K_FALLOFF || r.cls == K_CHEMACT);
    if (pdep && r.coll == C_NONE) throw LoadError(PYJAC_E_PARSE, tag + "pressure-dependent reaction needs a collider");
    if (!pdep && r.coll != C_NONE) throw LoadError(PYJAC_E_UNSUPPORTED, tag + "collider on a class that takes none");
    if ((r.cls == K_ELEM || r.cls == K_THD) && !r.arr.set) throw LoadError(PYJAC_E_PARSE, tag + "missing arrhenius");
    if (r.cls == K_FALLOFF || r.cls == K_CHEMACT) {
      if (!r.low.set || !r.high.set) throw LoadError(PYJAC_E_PARSE, tag + "falloff needs low and high");
      if (!(r.low.A > 0) || !(r.high.A > 0)) throw LoadError(PYJAC_E_UNSUPPORTED, tag + "falloff A must be positive");
      if (r.blend == B_NONE) throw LoadError(PYJAC_E_PARSE, tag + "falloff needs lindemann/troe/sri");
      if (r.blend == B_SRI && r.sri.size() == 5 && !(r.sri[3] > 0)) throw LoadError(PYJAC_E_UNSUPPORTED, tag + "SRI d must be positive");
      if (r.blend == B_TROE && (r.troe[1] == 0 || r.troe[2] == 0)) throw LoadError(PYJAC_E_UNSUPPORTED, tag + "Troe T***, T* must be nonzero");
    }
    if (r.cls == K_PLOG) {
      if (r.plog.empty()) throw LoadError(PYJAC_E_PARSE, tag + "PLOG needs points");
      for (size_t a = 0; a < r.plog.size(); ++a) {
        if (!(r.plog[a][0] > 0) || !(r.plog[a][1] > 0)) throw LoadError(PYJAC_E_UNSUPPORTED, tag + "PLOG p and A must be positive");
        for (size_t b = 0; b < a; ++b)
          if (r.plog[a][0] == r.plog[b][0]) throw LoadError(PYJAC_E_UNSUPPORTED, tag + "duplicate PLOG pressure");
      }
    }
    if (r.cls == K_CHEB) {
      if (r.eta.empty()) throw LoadError(PYJAC_E_PARSE, tag + "Chebyshev needs coefficients");
      if (!(r.Tmin > 0 && r.Tmax > r.Tmin && r.Pmin > 0 && r.Pmax > r.Pmin))
        throw LoadError(PYJAC_E_UNSUPPORTED, tag + "bad Chebyshev range");
    }
    if (r.rev == R_EXPLICIT && !r.revr.set) throw LoadError(PYJAC_E_PARSE, tag + "explicit reverse needs 'reverse'");
    if (r.rev != R_EXPLICIT && r.revr.set) throw LoadError(PYJAC_E_PARSE, tag + "'reverse' given for a non-explicit reaction");
  }
}

uint64_t fnv1a(const std::string& s) {
  uint64_t h = 1469598103934665603ULL;
  for (unsigned char c : s) { h ^= c; h *= 1099511628211ULL; }
  return h;
}

int pack_side(int sp, int nu) { return sp | (nu << 16); }

// A piece of a Jacobian column stream: rows [k0, k1) of column j, len records.
struct ColSeg {
  int j, k0, k1, len;
};

// Longest segment a group would stream when segments, longest first, are dealt
// to `groups` groups in snake order (the order of the tile kernel's phase D),
// each segment costing its padded length plus a fixed set-up.
int snake_makespan(std::vector<int> len, int groups) {
  std::sort(len.rbegin(), len.rend());
  std::vector<int> load(groups, 0);
  for (size_t i = 0; i < len.size(); ++i) {
    const int m = (int)(i / groups), r = (int)(i % groups);
    load[(m & 1) ? groups - 1 - r : r] += (len[i] + kColBatch - 1) / kColBatch * kColBatch + 8;
  }
  return *std::max_element(load.begin(), load.end());
}

// Splits the every-row column streams at row boundaries so that 64 groups
// (the group count of the usual launch shapes) finish phase D together: the
// longest segment is halved while that lowers the snake makespan, as long as
// the partial sums of the split columns fit the 2N rows the tile kernel keeps
// for them.  The split depends on the mechanism only, never on the launch
// shape, so results stay identical across shapes.
std::vector<ColSeg> split_columns(const std::vector<std::vector<std::vector<ColRec>>>& rows, int N) {
  constexpr int kGroups = 64, kMinSplit = 32;
  std::vector<ColSeg> segs;
  for (int j = 0; j < N - 1; ++j) {
    int len = 0;
    for (int k = 0; k < N; ++k) len += (int)rows[j][k].size();
    segs.push_back(ColSeg{j, 0, N, len});
  }
  auto lens = [&](const std::vector<ColSeg>& v) {
    std::vector<int> l;
    for (auto& g : v) l.push_back(g.len);
    return l;
  };
  auto slots = [&](const std::vector<ColSeg>& v) {
    std::vector<int> n(N, 0);
    for (auto& g : v) ++n[g.j];
    int s = 0;
    for (int c : n) s += c > 1 ? c : 0;
    return s;
  };
  std::vector<ColSeg> best = segs;
  int best_ms = snake_makespan(lens(segs), kGroups);
  for (;;) {
    int w = -1;
    for (int i = 0; i < (int)segs.size(); ++i)
      if (segs[i].k1 - segs[i].k0 > 1 && segs[i].len >= kMinSplit && (w < 0 || segs[i].len > segs[w].len)) w = i;
    if (w < 0) break;
    // the row boundary that best halves the segment
    const ColSeg g = segs[w];
    int acc = 0, cut = g.k0 + 1, cut_acc = 0, err = 1 << 30;
    for (int k = g.k0; k < g.k1 - 1; ++k) {
      acc += (int)rows[g.j][k].size();
      const int e = std::abs(2 * acc - g.len);
      if (e < err) { err = e; cut = k + 1; cut_acc = acc; }
    }
    segs[w] = ColSeg{g.j, g.k0, cut, cut_acc};
    segs.push_back(ColSeg{g.j, cut, g.k1, g.len - cut_acc});
    if (slots(segs) > 2 * N) break;
    const int ms = snake_makespan(lens(segs), kGroups);
    if (ms < best_ms) { best_ms = ms; best = segs; }
    if ((int)segs.size() >= 4 * kGroups) break;
  }
  return best;
}

}  // namespace

int build_tables(const std::string& text, PackedMech& P, std::string& msg) {
  try {
    RawMech m = read_mech(text);
    validate(m);
    const int N = (int)m.names.size(), NR = (int)m.rxn.size();
    P = PackedMech();
    P.N = N; P.NR = NR; P.hash = fnv1a(text);
    // ---- species
    for (int k = 0; k < N; ++k) {
      P.W.push_back(m.W[k]);
      P.invW.push_back(1.0 / m.W[k]);
      P.tmid.push_back(m.tmid[k]);
      for (double a : m.nasa[k]) P.nasa.push_back(a);
    }
    for (int j = 0; j < N - 1; ++j) P.vcol.push_back(1.0 / m.W[j] - 1.0 / m.W[N - 1]);
    // ---- sort reactions so that neighbouring lanes share branches
    std::vector<int> order(NR);
    std::iota(order.begin(), order.end(), 0);
    auto key = [&](int i) {
      const RawRxn& r = m.rxn[i];
      return ((r.cls * 16 + r.blend) * 16 + r.coll) * 16 + r.rev;
    };
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return key(a) < key(b); });
    const double lnpr = std::log(kOneAtm / kGasConstant);
    int ng = 0;
    for (int slot = 0; slot < NR; ++slot) {
      const RawRxn& r = m.rxn[order[slot]];
      RxnRec rec;
      std::memset(&rec, 0, sizeof(rec));
      int info = r.cls | (r.blend << 4) | (r.rev << 8) | (r.coll << 12);
      for (auto& q : r.reac) if (q.first == N - 1) info |= F_LAST_SPECIES;
      for (auto& q : r.prod) if (q.first == N - 1) info |= F_LAST_SPECIES;
      if (r.blend == B_TROE && r.troe.size() == 4) info |= F_TROE_T2;
      rec.info = info;
      rec.orig = r.file_index;
      int sf = 0, sr = 0;
      for (int q = 0; q < 2 * kMaxSide; ++q) rec.mol[q] = N;      // X[N] = 1: an absent molecule
      for (auto& q : r.reac)
        for (int c = 0; c < q.second; ++c) rec.mol[sf++] = q.first;
      for (auto& q : r.prod)
        for (int c = 0; c < q.second; ++c) rec.mol[kMaxSide + sr++] = q.first;
      rec.sum_f = sf;
      rec.sum_r = sr;
      std::map<int, int> netnu;
      for (auto& q : r.reac) netnu[q.first] -= q.second;
      for (auto& q : r.prod) netnu[q.first] += q.second;
      int dnu = 0, c = 0;
      for (auto& [k, nu] : netnu) {
        if (!nu) continue;
        rec.net[c++] = pack_side(k, nu & 0xFFFF);
        dnu += nu;
      }
      for (; c < kMaxNet; ++c) rec.net[c] = -1;
      rec.dnu_lnpr = dnu * lnpr;
      // Arrhenius: primary rate coefficient (k_f), secondary ratio k0/kinf, reverse
      if (r.cls == K_ELEM || r.cls == K_THD) { rec.arr[0] = r.arr.A; rec.arr[1] = r.arr.b; rec.arr[2] = r.arr.Ta; }
      if (r.cls == K_FALLOFF || r.cls == K_CHEMACT) {
        const Arrh& pri = (r.cls == K_FALLOFF) ? r.high : r.low;
        rec.arr[0] = pri.A; rec.arr[1] = pri.b; rec.arr[2] = pri.Ta;
        rec.arr[3] = r.low.A / r.high.A; rec.arr[4] = r.low.b - r.high.b; rec.arr[5] = r.low.Ta - r.high.Ta;
      }
      if (r.rev == R_EXPLICIT) { rec.arr[6] = r.revr.A; rec.arr[7] = r.revr.b; rec.arr[8] = r.revr.Ta; }
      if (r.blend == B_TROE) {
        for (size_t q = 0; q < r.troe.size(); ++q) rec.fpar[q] = r.troe[q];
        rec.frcp[0] = 1.0 / r.troe[1];
        rec.frcp[1] = 1.0 / r.troe[2];
      }
      if (r.blend == B_SRI) {
        rec.fpar[0] = r.sri[0]; rec.fpar[1] = r.sri[1]; rec.fpar[2] = r.sri[2];
        rec.fpar[3] = r.sri.size() > 3 ? r.sri[3] : 1.0;
        rec.fpar[4] = r.sri.size() > 4 ? r.sri[4] : 0.0;
        rec.frcp[0] = 1.0 / r.sri[2];
      }
      // collider
      rec.coll_m = (r.coll == C_SPECIES) ? r.m : -1;
      double aN = 1.0;
      if (r.coll == C_EFF) {
        rec.aux0 = (int)P.eff_sp.size();
        for (auto& [k, a] : r.eff) {
          if (a == 1.0) continue;
          P.eff_sp.push_back(k);
          P.eff_am1.push_back(a - 1.0);
          if (k == N - 1) aN = a;
        }
        rec.aux1 = (int)P.eff_sp.size();
      }
      rec.alphaN_m1 = aN - 1.0;
      bool has_g = (r.coll == C_EFF) || (r.coll == C_SPECIES);
      rec.gslot = has_g ? ng++ : -1;
      if (r.cls == K_PLOG) {
        auto pts = r.plog;
        std::sort(pts.begin(), pts.end(), [](const std::array<double, 4>& a, const std::array<double, 4>& b) { return a[0] < b[0]; });
        rec.aux0 = (int)P.plog.size() / 4;
        for (auto& q : pts) { P.plog.push_back(std::log(q[0])); P.plog.push_back(std::log(q[1])); P.plog.push_back(q[2]); P.plog.push_back(q[3]); }
        rec.aux1 = (int)P.plog.size() / 4;
      }
      // Chebyshev: T~ = c1/T + c0, p~ = pc1 log10(p) + pc0
      if (r.cls == K_CHEB) {
        rec.aux0 = (int)P.cheb.size();
        double iTmin = 1.0 / r.Tmin, iTmax = 1.0 / r.Tmax;
        double lpmin = std::log10(r.Pmin), lpmax = std::log10(r.Pmax);
        P.cheb.push_back(r.nT);
        P.cheb.push_back(r.nP);
        P.cheb.push_back(2.0 / (iTmax - iTmin));
        P.cheb.push_back(-(iTmin + iTmax) / (iTmax - iTmin));
        P.cheb.push_back(2.0 / (lpmax - lpmin));
        P.cheb.push_back(-(lpmin + lpmax) / (lpmax - lpmin));
        for (double v : r.eta) P.cheb.push_back(v);
      }
      P.rx.push_back(rec);
    }
    P.NG = ng;
    if (P.cheb.empty()) P.cheb.push_back(0.0);
    if (P.plog.empty()) P.plog.push_back(0.0);
    // slack for the four-at-a-time efficiency loads
    for (int u = 0; u < 4; ++u) { P.eff_sp.push_back(0); P.eff_am1.push_back(0.0); }
    // ---- per-species reaction lists (sorted slots ascending), all N species
    std::vector<std::vector<std::pair<int, double>>> lists(N);
    for (int slot = 0; slot < NR; ++slot) {
      const RawRxn& r = m.rxn[order[slot]];
      std::map<int, int> netnu;
      for (auto& q : r.reac) netnu[q.first] -= q.second;
      for (auto& q : r.prod) netnu[q.first] += q.second;
      for (auto& [k, nu] : netnu) if (nu) lists[k].push_back({slot, (double)nu});
    }
    P.spg_ptr.push_back(0);
    for (int k = 0; k < N; ++k) {
      for (auto& e : lists[k]) P.spg_ent.push_back(e.first | ((int)e.second << 16));
      P.spg_ptr.push_back((int)P.spg_ent.size());
    }
    P.spg_ent.resize(P.spg_ent.size() + 4, 0);      // slack for the unrolled gather
    // ---- Jacobian column streams.  For species row k and species column j the
    // j-specific part of J[k+1][j+1] is sum_t coef_t * P[src_t] * X[x1_t] * X[x2_t]
    // with P = {c_i k_f,i (slots 0..NR-1), c_i k_r,i (NR..2NR-1), dc_i/dE_i * R_i (2NR..)}.
    struct Term { int j, k, src, x; double coef; };
    std::vector<Term> terms;
    auto cofactors = [&](const std::vector<std::pair<int, int>>& sidev, int l) {
      // molecules of the side other than one copy of species l; N means "1"
      std::vector<int> mol;
      bool removed = false;
      for (auto& q : sidev)
        for (int c = 0; c < q.second; ++c) {
          if (q.first == l && !removed) { removed = true; continue; }
          mol.push_back(q.first);
        }
      while (mol.size() < 2) mol.push_back(N);
      return mol[0] | (mol[1] << 15);
    };
    for (int slot = 0; slot < NR; ++slot) {
      const RawRxn& r = m.rxn[order[slot]];
      std::map<int, int> netnu;
      for (auto& q : r.reac) netnu[q.first] -= q.second;
      for (auto& q : r.prod) netnu[q.first] += q.second;
      for (auto& [k, nu_k] : netnu) {
        if (!nu_k) continue;
        for (auto& q : r.reac) {
          int l = q.first;
          if (l == N - 1) continue;
          terms.push_back({l, k, slot, cofactors(r.reac, l), m.W[k] / m.W[l] * nu_k * q.second});
        }
        if (r.rev != R_IRREV)
          for (auto& q : r.prod) {
            int l = q.first;
            if (l == N - 1) continue;
            terms.push_back({l, k, NR + slot, cofactors(r.prod, l), -m.W[k] / m.W[l] * nu_k * q.second});
          }
        int g = P.rx[slot].gslot;
        if (r.coll == C_EFF) {
          for (auto& [l, a] : r.eff) {
            if (l == N - 1 || a == 1.0) continue;
            terms.push_back({l, k, 2 * NR + g, N | (N << 15), m.W[k] / m.W[l] * nu_k * (a - 1.0)});
          }
        } else if (r.coll == C_SPECIES && r.m != N - 1) {
          terms.push_back({r.m, k, 2 * NR + g, N | (N << 15), m.W[k] / m.W[r.m] * nu_k});
        }
      }
    }
    std::stable_sort(terms.begin(), terms.end(), [](const Term& a, const Term& b) {
      return a.j != b.j ? a.j < b.j : a.k < b.k;
    });

    const int FW = colFlagWords(N);
    P.col_flags.assign((size_t)std::max(N - 1, 1) * FW, 0u);
    {
      // form of the streams: present rows only when most (row, column) pairs
      // have no terms, every row otherwise
      long long pairs = 0;
      for (size_t u = 0; u < terms.size(); ++u)
        pairs += (u == 0 || terms[u].j != terms[u - 1].j || terms[u].k != terms[u - 1].k);
      P.col_split = 2 * pairs < (long long)(N - 1) * N ? 1 : 0;
    }
    if (!P.col_split) {
      // records of every row of every column: the row's terms, the last one
      // carrying the mark for k < N - 1, or a marker alone for a row without
      // terms (the placeholder row N - 1 has none: the kernel finishes it after
      // the stream); markers and padding address X[N] = 1 and contribute 0
      std::vector<std::vector<std::vector<ColRec>>> rows(N - 1, std::vector<std::vector<ColRec>>(N));
      for (size_t t = 0; t < terms.size(); ++t)
        rows[terms[t].j][terms[t].k].push_back(ColRec{terms[t].coef, N + 1 + terms[t].src, terms[t].x});
      for (int j = 0; j < N - 1; ++j)
        for (int k = 0; k < N - 1; ++k) {
          if (rows[j][k].empty()) rows[j][k].push_back(ColRec{0.0, N, N | (N << 15)});
          rows[j][k].back().x |= kColMark;
        }
      const std::vector<ColSeg> segs = split_columns(rows, N);
      // emission: each column's segments in row order, each padded to a
      // multiple of kColBatch; a column in several segments gets consecutive
      // slots for its partial temperature-row sums, added in row order
      P.col_item.clear();
      P.col_join.clear();
      int slot = 0;
      for (int j = 0; j < N - 1; ++j) {
        P.col_start.push_back((int)P.colrec.size());
        std::vector<ColSeg> mine;
        for (const ColSeg& g : segs) if (g.j == j) mine.push_back(g);
        std::sort(mine.begin(), mine.end(), [](const ColSeg& a, const ColSeg& b) { return a.k0 < b.k0; });
        const bool joined = mine.size() > 1;
        if (joined) P.col_join.push_back(ColJoin{j, slot, (int)mine.size(), 0});
        for (size_t q = 0; q < mine.size(); ++q) {
          const int rec = (int)P.colrec.size();
          for (int k = mine[q].k0; k < mine[q].k1; ++k)
            P.colrec.insert(P.colrec.end(), rows[j][k].begin(), rows[j][k].end());
          while (P.colrec.size() % kColBatch) P.colrec.push_back(ColRec{0.0, N, N | (N << 15)});
          P.col_item.push_back(ColItem{j, mine[q].k0, rec, (int)P.colrec.size() - rec, joined ? slot++ : -1,
                                       mine[q].k1 == N ? 1 : 0, 0, 0});
        }
      }
      // longest first: the groups of a wavefront stream in lockstep
      std::stable_sort(P.col_item.begin(), P.col_item.end(),
                       [](const ColItem& a, const ColItem& b) { return a.cnt > b.cnt; });
      P.col_start.push_back((int)P.colrec.size());
      // one batch of slack: the kernel reads one batch past a segment's stream
      for (int u = 0; u < kColBatch; ++u) P.colrec.push_back(ColRec{0.0, N, N | (N << 15)});
    } else {
      size_t t = 0;
      for (int j = 0; j < N - 1; ++j) {
        P.col_start.push_back((int)P.colrec.size());
        // rows of column j with terms.  A row without terms costs a marker in
        // the stream but a full visit in the dense pass, so a block of 32 rows
        // goes to the dense pass only when most of its rows have no terms;
        // otherwise all its rows are streamed.
        std::vector<char> has(N, 0);
        for (size_t u = t; u < terms.size() && terms[u].j == j; ++u) has[terms[u].k] = 1;
        std::vector<int> rows;
        for (int w = 0; w < FW; ++w) {
          const int k0 = 32 * w, kn = std::min(32, N - k0);
          int absent = 0;
          for (int k = k0; k < k0 + kn; ++k) absent += !has[k];
          const bool split = 2 * absent > kn;
          for (int k = k0; k < k0 + kn; ++k)
            if (has[k] || !split) {
              rows.push_back(k);
              P.col_flags[(size_t)j * FW + w] |= 1u << (k - k0);
            }
        }
        P.colrec.push_back(ColRec{0.0, rows.empty() ? N : rows[0], N | (N << 15) | kColMark});
        for (size_t q = 0; q < rows.size(); ++q) {
          for (; t < terms.size() && terms[t].j == j && terms[t].k == rows[q]; ++t)
            P.colrec.push_back(ColRec{terms[t].coef, N + 1 + terms[t].src, terms[t].x});
          const int next = q + 1 < rows.size() ? rows[q + 1] : N;
          P.colrec.push_back(ColRec{0.0, next, N | (N << 15) | kColMark});
        }
        // padding addresses X[N] = 1 and contributes 0
        while (P.colrec.size() % (2 * kColBatch)) P.colrec.push_back(ColRec{0.0, N, N | (N << 15)});
      }
      P.col_start.push_back((int)P.colrec.size());
      // one batch of slack: the kernel reads one batch past a column's stream
      for (int u = 0; u < kColBatch; ++u) P.colrec.push_back(ColRec{0.0, N, N | (N << 15)});
    }
    // ---- concentration-based, constant-volume form (state {T, [X_1..X_N]}):
    // d wdot_k / d[X_l] = sum_i nu_ki dq_i/d[X_l]; the mass-action and
    // non-unit-collider parts are the sparse terms (every species l is a state
    // variable, no molecular-weight ratios); the all-species collider baseline
    // and the pressure dependence form the dense vector u computed per state.
    {
      std::vector<Term> tv;
      for (int slot = 0; slot < NR; ++slot) {
        const RawRxn& r = m.rxn[order[slot]];
        std::map<int, int> netnu;
        for (auto& q : r.reac) netnu[q.first] -= q.second;
        for (auto& q : r.prod) netnu[q.first] += q.second;
        for (auto& [k, nu_k] : netnu) {
          if (!nu_k) continue;
          for (auto& q : r.reac) tv.push_back({q.first, k, slot, cofactors(r.reac, q.first), (double)nu_k * q.second});
          if (r.rev != R_IRREV)
            for (auto& q : r.prod)
              tv.push_back({q.first, k, NR + slot, cofactors(r.prod, q.first), -(double)nu_k * q.second});
          const int g = P.rx[slot].gslot;
          if (r.coll == C_EFF) {
            for (auto& [l, a] : r.eff)
              if (a != 1.0) tv.push_back({l, k, 2 * NR + g, N | (N << 15), nu_k * (a - 1.0)});
          } else if (r.coll == C_SPECIES) {
            tv.push_back({r.m, k, 2 * NR + g, N | (N << 15), (double)nu_k});
          }
        }
      }
      std::stable_sort(tv.begin(), tv.end(), [](const Term& a, const Term& b) {
        return a.j != b.j ? a.j < b.j : a.k < b.k;
      });
      size_t t = 0;
      P.cv_colptr.push_back(0);
      for (int j = 0; j < N; ++j) {
        P.cv_col_start.push_back((int)P.cv_colrec.size());
        std::vector<int> rows;
        for (size_t u = t; u < tv.size() && tv[u].j == j; ++u)
          if (rows.empty() || rows.back() != tv[u].k) rows.push_back(tv[u].k);
        for (int k : rows) P.cv_rowidx.push_back(k);
        P.cv_colptr.push_back((int)P.cv_rowidx.size());
        P.cv_colrec.push_back(ColRec{0.0, rows.empty() ? N : rows[0], N | (N << 15) | kColMark});
        for (size_t q = 0; q < rows.size(); ++q) {
          for (; t < tv.size() && tv[t].j == j && tv[t].k == rows[q]; ++t)
            P.cv_colrec.push_back(ColRec{tv[t].coef, N + 1 + tv[t].src, tv[t].x});
          const int next = q + 1 < rows.size() ? rows[q + 1] : N;
          P.cv_colrec.push_back(ColRec{0.0, next, N | (N << 15) | kColMark});
        }
        while (P.cv_colrec.size() % (2 * kColBatch)) P.cv_colrec.push_back(ColRec{0.0, N, N | (N << 15)});
      }
      P.cv_col_start.push_back((int)P.cv_colrec.size());
      for (int u = 0; u < kColBatch; ++u) P.cv_colrec.push_back(ColRec{0.0, N, N | (N << 15)});
      P.cv_col_order.resize(N);
      std::iota(P.cv_col_order.begin(), P.cv_col_order.end(), 0);
      std::stable_sort(P.cv_col_order.begin(), P.cv_col_order.end(), [&](int a, int b) {
        return P.cv_col_start[a + 1] - P.cv_col_start[a] > P.cv_col_start[b + 1] - P.cv_col_start[b];
      });
    }
    // The groups of a wavefront stream their columns in lockstep, so columns
    // go out longest first: neighbouring groups get streams of similar length.
    P.col_order.resize(N - 1);
    std::iota(P.col_order.begin(), P.col_order.end(), 0);
    std::stable_sort(P.col_order.begin(), P.col_order.end(), [&](int a, int b) {
      return P.col_start[a + 1] - P.col_start[a] > P.col_start[b + 1] - P.col_start[b];
    });
    if (P.col_order.empty()) P.col_order.push_back(0);
    return PYJAC_OK;
  } catch (const LoadError& e) {
    msg = e.what();
    return e.code;
  } catch (const std::exception& e) {
    msg = e.what();
    return PYJAC_E_PARSE;
  }
}

std::vector<int> species_chunk_bounds(const PackedMech& P, int chunk) {
  const int N = P.N;
  const int nch = (P.NR + chunk - 1) / chunk;
  std::vector<int> b((size_t)(nch + 1) * N);
  for (int k = 0; k < N; ++k) {
    int e = P.spg_ptr[k];
    for (int c = 0; c <= nch; ++c) {
      const int lim = c * chunk;
      while (e < P.spg_ptr[k + 1] && (P.spg_ent[e] & 0xFFFF) < lim) ++e;
      b[(size_t)c * N + k] = e;
    }
  }
  return b;
}

}  // namespace pyjac
