// Reader for mechanisms in the Chemkin-II text format (the subset that the
// library's reaction classes cover), converted into the library's own token
// format so that one validating loader serves both.
//
// Accepted input:
//  * ELEMENTS (ELEM) block: names, optionally with an atomic weight "/w/";
//    names without one take the IUPAC abridged standard atomic weight.
//  * SPECIES (SPEC) block: names.
//  * THERMO [ALL] block, here or in a separate thermo text: an optional line
//    of default T_low T_mid T_high, then 4-line NASA-7 records in the fixed
//    columns of the format (name and composition on line 1, T_low, T_high,
//    T_mid in columns 46-73; upper-range a1..a7 then lower-range a1..a7 in
//    15-column fields on lines 2-4).
//  * REACTIONS (REAC) block with optional units (CAL/MOLE default, KCAL/MOLE,
//    JOULES/MOLE, KJOULES/MOLE, KELVINS, EVOLTS; MOLES default).  Each
//    reaction is "equation A b E" followed by auxiliary lines:
//    LOW/HIGH (falloff / chemically activated pressure limit), TROE, SRI, REV,
//    PLOG (p in atm), CHEB with TCHEB/PCHEB (p in atm), third-body
//    efficiencies "X/a/", DUPLICATE.  "+M" marks a third-body reaction,
//    "(+M)" or "(+X)" a pressure-dependent one (Sec. 2.3.2, 2.3.3), "=>" an
//    irreversible one.
//
// Unit conversion to SI-kmol: A is in (cm^3/mol)^(order-1)/s with order the
// molecularity of that rate coefficient (reactant coefficients, plus one for
// [M] in third-body and falloff low-pressure-limit coefficients, minus one
// for the high-pressure limit of a chemically activated reaction), so it is
// scaled by 1e-3^(order-1); activation energies become activation temperatures E/R;
// pressures go from atm to Pa.  Chebyshev fits give log10 k, so the same
// scaling shifts the (0, 0) coefficient by -3(order-1).
#include <array>
#include <cmath>
#include <cstdlib>
#include <cctype>
#include <map>
#include <sstream>
#include <string>
#include <vector>

#include "../../include/pyjac.h"
#include "tables.hpp"
#include "chemkin.hpp"

namespace pyjac {
namespace {

constexpr double kRmol = 8.314462618;      // J/(mol K)
constexpr double kAtm = 101325.0;          // Pa

struct CkError {
  int code;
  std::string msg;
};

[[noreturn]] void ck_fail(int code, int line, const std::string& m) {
  throw CkError{code, (line > 0 ? "line " + std::to_string(line) + ": " : std::string()) + m};
}

std::string upper(std::string s) {
  for (auto& c : s) c = (char)std::toupper((unsigned char)c);
  return s;
}

std::string trim(const std::string& s) {
  size_t a = s.find_first_not_of(" \t\r\n"), b = s.find_last_not_of(" \t\r\n");
  return a == std::string::npos ? std::string() : s.substr(a, b - a + 1);
}

bool parse_real(const std::string& t, double& v) {
  if (t.empty()) return false;
  std::string u = t;
  for (auto& c : u)
    if (c == 'd' || c == 'D') c = 'e';      // Fortran exponents
  char* end = nullptr;
  v = std::strtod(u.c_str(), &end);
  return end && *end == '\0';
}

double real_or_fail(const std::string& t, int line, const char* what) {
  double v;
  if (!parse_real(trim(t), v)) ck_fail(PYJAC_E_PARSE, line, std::string("bad number for ") + what + ": '" + t + "'");
  return v;
}

std::string num(double v) {
  std::ostringstream o;
  o.precision(17);
  o << v;
  return o.str();
}

double standard_weight(const std::string& e) {
  static const std::map<std::string, double> w = {
      {"H", 1.008}, {"D", 2.014}, {"HE", 4.0026}, {"C", 12.011}, {"N", 14.007}, {"O", 15.999},
      {"F", 18.998}, {"NE", 20.180}, {"SI", 28.085}, {"S", 32.06}, {"CL", 35.45}, {"AR", 39.95},
      {"KR", 83.798}, {"XE", 131.29}};
  auto it = w.find(upper(e));
  return it == w.end() ? -1.0 : it->second;
}

struct Line {
  int no;
  std::string text;      // comment stripped
  std::string raw;       // as read (fixed-column thermo records)
};

struct ThermoRec {
  std::vector<std::pair<std::string, double>> comp;
  double tmid;
  double low[7], high[7];
};

// Splits an auxiliary line into "KEY / values /" items; a key without a
// slash (DUPLICATE) has no values.
std::vector<std::pair<std::string, std::vector<std::string>>> aux_items(const std::string& s, int line) {
  std::vector<std::pair<std::string, std::vector<std::string>>> out;
  size_t i = 0;
  while (i < s.size()) {
    while (i < s.size() && std::isspace((unsigned char)s[i])) ++i;
    if (i >= s.size()) break;
    size_t k = i;
    while (k < s.size() && s[k] != '/' && !std::isspace((unsigned char)s[k])) ++k;
    std::string key = s.substr(i, k - i);
    size_t j = k;
    while (j < s.size() && std::isspace((unsigned char)s[j])) ++j;
    if (j < s.size() && s[j] == '/') {
      size_t e = s.find('/', j + 1);
      if (e == std::string::npos) ck_fail(PYJAC_E_PARSE, line, "unterminated '/' after " + key);
      std::istringstream vs(s.substr(j + 1, e - j - 1));
      std::vector<std::string> vals;
      for (std::string t; vs >> t;) vals.push_back(t);
      out.push_back({key, vals});
      i = e + 1;
    } else {
      out.push_back({key, {}});
      i = k;
    }
  }
  return out;
}

struct Side {
  std::vector<std::pair<std::string, int>> sp;   // species, coefficient (merged)
  bool plus_m = false;                            // "+M"
  std::string falloff;                            // "" | "M" | species of "(+X)"
};

Side parse_side(std::string s, const std::map<std::string, int>& known, int line) {
  Side out;
  // "(+X)" at the end of the side marks a pressure-dependent reaction
  const size_t fo = s.rfind("(+");
  if (fo != std::string::npos && !s.empty() && s.back() == ')') {
    const std::string inner = s.substr(fo + 2, s.size() - fo - 3);
    if (upper(inner) == "M" || known.count(inner)) {
      out.falloff = upper(inner) == "M" ? "M" : inner;
      s = s.substr(0, fo);
    }
  }
  // split on '+' (a '+' right after another '+' or at the start belongs to a name)
  std::vector<std::string> terms;
  std::string cur;
  for (size_t i = 0; i < s.size(); ++i) {
    if (s[i] == '+' && !cur.empty()) {
      terms.push_back(cur);
      cur.clear();
    } else {
      cur += s[i];
    }
  }
  if (!cur.empty()) terms.push_back(cur);
  std::map<std::string, int> merged;
  std::vector<std::string> order;
  for (const auto& t : terms) {
    if (upper(t) == "M") {
      out.plus_m = true;
      continue;
    }
    std::string name = t;
    int coef = 1;
    if (!known.count(name)) {
      size_t d = 0;
      while (d < t.size() && std::isdigit((unsigned char)t[d])) ++d;
      if (d > 0 && d < t.size() && known.count(t.substr(d))) {
        coef = std::atoi(t.substr(0, d).c_str());
        name = t.substr(d);
      } else {
        ck_fail(PYJAC_E_PARSE, line, "unknown species '" + t + "'");
      }
    }
    if (!merged.count(name)) order.push_back(name);
    merged[name] += coef;
  }
  for (const auto& n : order) out.sp.push_back({n, merged[n]});
  return out;
}

struct CkReaction {
  int line = 0;
  Side lhs, rhs;
  bool reversible = true;
  double A = 0, b = 0, E = 0;
  std::vector<double> low, high, troe, sri, rev;
  std::vector<std::array<double, 4>> plog;
  std::vector<double> cheb, tcheb, pcheb;
  std::vector<std::pair<std::string, double>> eff;
};

void convert(const std::string& mech, const std::string* thermo_text, std::string& out) {
  // ---- lines, comments stripped
  std::vector<Line> lines;
  {
    std::istringstream in(mech);
    int no = 0;
    for (std::string l; std::getline(in, l);) {
      ++no;
      const size_t c = l.find('!');
      lines.push_back({no, c == std::string::npos ? l : l.substr(0, c), l});
    }
  }
  std::vector<std::pair<std::string, double>> elements;     // name, weight
  std::vector<std::string> species;
  std::map<std::string, int> sp_index;
  std::map<std::string, ThermoRec> thermo;
  std::vector<CkReaction> rxns;
  double e_to_ta = 4.184 / kRmol;                             // CAL/MOLE

  auto parse_thermo = [&](const std::vector<Line>& tl, size_t i, size_t end) {
    double dmid = 1000.0;
    // optional default temperature line: three numbers
    while (i < end && trim(tl[i].text).empty()) ++i;
    if (i < end) {
      std::istringstream ts(tl[i].text);
      double a, m, c;
      std::string extra;
      if ((ts >> a >> m >> c) && !(ts >> extra)) {
        dmid = m;
        ++i;
      }
    }
    while (i < end) {
      if (trim(tl[i].text).empty()) { ++i; continue; }
      if (i + 3 >= end) ck_fail(PYJAC_E_PARSE, tl[i].no, "truncated thermo record");
      const std::string l1 = tl[i].raw + std::string(80, ' ');
      std::string name;
      std::istringstream(l1.substr(0, 18)) >> name;
      ThermoRec r;
      for (int f = 0; f < 4; ++f) {
        const std::string el = trim(l1.substr(24 + 5 * f, 2));
        const std::string cnt = trim(l1.substr(26 + 5 * f, 3));
        if (el.empty() || el == "0") continue;
        const double c = cnt.empty() ? 0.0 : real_or_fail(cnt, tl[i].no, "element count");
        if (c != 0.0) r.comp.push_back({el, c});
      }
      const std::string tm = trim(l1.substr(65, 8));
      r.tmid = tm.empty() ? dmid : real_or_fail(tm, tl[i].no, "T_mid");
      double a[15];
      int q = 0;
      for (int k = 1; k <= 3; ++k) {
        const std::string lk = tl[i + k].raw + std::string(80, ' ');
        const int nf = k < 3 ? 5 : 4;
        for (int f = 0; f < nf; ++f) a[q++] = real_or_fail(lk.substr(15 * f, 15), tl[i + k].no, "NASA coefficient");
      }
      for (int k = 0; k < 7; ++k) {
        r.high[k] = a[k];
        r.low[k] = a[7 + k];
      }
      thermo[name] = r;
      i += 4;
    }
  };

  size_t i = 0;
  while (i < lines.size()) {
    const std::string t = upper(trim(lines[i].text));
    if (t.empty()) { ++i; continue; }
    std::istringstream ts(t);
    std::string kw;
    ts >> kw;
    auto block_end = [&](size_t from) {
      size_t e = from;
      while (e < lines.size()) {
        std::istringstream ls(upper(lines[e].text));
        std::string f;
        if ((ls >> f) && f == "END") break;
        ++e;
      }
      if (e >= lines.size()) ck_fail(PYJAC_E_PARSE, lines[from - 1].no, kw + " block without END");
      return e;
    };
    if (kw == "ELEMENTS" || kw == "ELEM") {
      const size_t e = block_end(i + 1);
      // tokens of the header line after the keyword belong to the block too
      std::string body = trim(lines[i].text).substr(kw.size());
      for (size_t k = i + 1; k < e; ++k) body += " " + lines[k].text;
      for (const auto& it : aux_items(body, lines[i].no)) {
        const double w = it.second.empty() ? standard_weight(it.first)
                                           : real_or_fail(it.second.at(0), lines[i].no, "atomic weight");
        if (!(w > 0)) ck_fail(PYJAC_E_PARSE, lines[i].no, "no atomic weight for element " + it.first);
        elements.push_back({it.first, w});
      }
      i = e + 1;
    } else if (kw == "SPECIES" || kw == "SPEC") {
      const size_t e = block_end(i + 1);
      std::string body = trim(lines[i].text).substr(kw.size());
      for (size_t k = i + 1; k < e; ++k) body += " " + lines[k].text;
      std::istringstream bs(body);
      for (std::string s; bs >> s;) {
        if (sp_index.count(s)) ck_fail(PYJAC_E_PARSE, lines[i].no, "species " + s + " listed twice");
        sp_index[s] = (int)species.size();
        species.push_back(s);
      }
      i = e + 1;
    } else if (kw == "THERMO") {
      const size_t e = block_end(i + 1);
      parse_thermo(lines, i + 1, e);
      i = e + 1;
    } else if (kw == "REACTIONS" || kw == "REAC") {
      for (std::string u; ts >> u;) {
        if (u == "CAL/MOLE") e_to_ta = 4.184 / kRmol;
        else if (u == "KCAL/MOLE") e_to_ta = 4184.0 / kRmol;
        else if (u == "JOULES/MOLE") e_to_ta = 1.0 / kRmol;
        else if (u == "KJOULES/MOLE") e_to_ta = 1000.0 / kRmol;
        else if (u == "KELVINS") e_to_ta = 1.0;
        else if (u == "EVOLTS") e_to_ta = 1.602176634e-19 / 1.380649e-23;
        else if (u == "MOLES") {}
        else ck_fail(PYJAC_E_UNSUPPORTED, lines[i].no, "reaction units " + u);
      }
      const size_t e = block_end(i + 1);
      for (size_t k = i + 1; k < e; ++k) {
        const std::string s = trim(lines[k].text);
        if (s.empty()) continue;
        const int ln = lines[k].no;
        // a reaction line has an equation and three trailing numbers
        std::istringstream ls(s);
        std::vector<std::string> tok;
        for (std::string w; ls >> w;) tok.push_back(w);
        double A, b, E;
        const bool is_rxn = s.find('=') != std::string::npos && tok.size() >= 4 &&
                            parse_real(tok[tok.size() - 3], A) && parse_real(tok[tok.size() - 2], b) &&
                            parse_real(tok[tok.size() - 1], E);
        if (is_rxn) {
          CkReaction r;
          r.line = ln;
          r.A = A; r.b = b; r.E = E;
          std::string eq;
          for (size_t q = 0; q + 3 < tok.size(); ++q) eq += tok[q];
          size_t pos, len;
          if ((pos = eq.find("<=>")) != std::string::npos) len = 3;
          else if ((pos = eq.find("=>")) != std::string::npos) { len = 2; r.reversible = false; }
          else if ((pos = eq.find('=')) != std::string::npos) len = 1;
          else ck_fail(PYJAC_E_PARSE, ln, "no '=' in reaction");
          r.lhs = parse_side(eq.substr(0, pos), sp_index, ln);
          r.rhs = parse_side(eq.substr(pos + len), sp_index, ln);
          if (r.lhs.plus_m != r.rhs.plus_m || r.lhs.falloff != r.rhs.falloff)
            ck_fail(PYJAC_E_PARSE, ln, "third body must appear on both sides");
          rxns.push_back(r);
          continue;
        }
        if (rxns.empty()) ck_fail(PYJAC_E_PARSE, ln, "auxiliary data before the first reaction");
        CkReaction& r = rxns.back();
        for (const auto& it : aux_items(s, ln)) {
          const std::string key = upper(it.first);
          if (key == "DUPLICATE" || key == "DUP") continue;
          static const char* const kKeys[] = {"LOW", "HIGH", "TROE", "SRI", "REV", "PLOG", "CHEB", "TCHEB", "PCHEB"};
          bool known = sp_index.count(it.first) > 0;
          for (const char* kk : kKeys) known = known || key == kk;
          if (!known) ck_fail(PYJAC_E_UNSUPPORTED, ln, "auxiliary keyword " + it.first);
          std::vector<double> v;
          for (const auto& x : it.second) v.push_back(real_or_fail(x, ln, key.c_str()));
          if (key == "LOW") r.low = v;
          else if (key == "HIGH") r.high = v;
          else if (key == "TROE") r.troe = v;
          else if (key == "SRI") r.sri = v;
          else if (key == "REV") r.rev = v;
          else if (key == "PLOG") {
            if (v.size() != 4) ck_fail(PYJAC_E_PARSE, ln, "PLOG needs p A b E");
            r.plog.push_back({v[0], v[1], v[2], v[3]});
          } else if (key == "CHEB") r.cheb.insert(r.cheb.end(), v.begin(), v.end());
          else if (key == "TCHEB") r.tcheb = v;
          else if (key == "PCHEB") r.pcheb = v;
          else {   // a species: third-body efficiency
            if (v.size() != 1) ck_fail(PYJAC_E_PARSE, ln, "efficiency of " + it.first + " needs one value");
            r.eff.push_back({it.first, v[0]});
          }
        }
      }
      i = e + 1;
    } else {
      ck_fail(PYJAC_E_PARSE, lines[i].no, "unexpected '" + trim(lines[i].text) + "' outside a block");
    }
  }
  if (thermo_text) {
    std::vector<Line> tl;
    std::istringstream in(*thermo_text);
    int no = 0;
    for (std::string l; std::getline(in, l);) {
      ++no;
      const size_t c = l.find('!');
      tl.push_back({no, c == std::string::npos ? l : l.substr(0, c), l});
    }
    size_t a = 0, e = tl.size();
    // a separate thermo text may carry its own THERMO ... END wrapper
    for (size_t k = 0; k < tl.size(); ++k) {
      std::istringstream ls(upper(tl[k].text));
      std::string f;
      if (!(ls >> f)) continue;
      if (f == "THERMO") a = k + 1;
      else if (f == "END") { e = k; break; }
    }
    parse_thermo(tl, a, e);
  }
  if (elements.empty()) ck_fail(PYJAC_E_PARSE, 0, "no ELEMENTS block");
  if (species.empty()) ck_fail(PYJAC_E_PARSE, 0, "no SPECIES block");

  // ---- token text
  std::ostringstream o;
  o << "pyjac-mech 1\n# converted from Chemkin format\n";
  o << "elements " << elements.size() << "\n";
  std::map<std::string, double> ew;
  for (const auto& e : elements) {
    o << "  " << e.first << " " << num(e.second) << "\n";
    ew[upper(e.first)] = e.second;
  }
  o << "species " << species.size() << "\n";
  for (const auto& s : species) {
    auto it = thermo.find(s);
    if (it == thermo.end()) ck_fail(PYJAC_E_PARSE, 0, "no thermo data for species " + s);
    const ThermoRec& r = it->second;
    double W = 0.0;
    std::string comp;
    for (const auto& c : r.comp) {
      auto w = ew.find(upper(c.first));
      if (w == ew.end()) ck_fail(PYJAC_E_PARSE, 0, "species " + s + " uses undeclared element " + c.first);
      if (c.second != std::floor(c.second)) ck_fail(PYJAC_E_UNSUPPORTED, 0, "fractional element count in " + s);
      W += w->second * c.second;
      // element names as declared in ELEMENTS
      std::string en = c.first;
      for (const auto& e : elements)
        if (upper(e.first) == upper(c.first)) en = e.first;
      comp += " " + en + " " + std::to_string((long)c.second);
    }
    o << "  " << s << " " << num(W) << " " << num(r.tmid) << " " << r.comp.size() << comp << "\n    ";
    for (int k = 0; k < 7; ++k) o << num(r.low[k]) << (k < 6 ? " " : "\n    ");
    for (int k = 0; k < 7; ++k) o << num(r.high[k]) << (k < 6 ? " " : "\n");
  }
  o << "reactions " << rxns.size() << "\n";
  for (const auto& r : rxns) {
    const int ln = r.line;
    auto side = [&](const Side& sd) {
      std::string t = std::to_string(sd.sp.size());
      for (const auto& p : sd.sp) t += " " + p.first + " " + std::to_string(p.second);
      return t;
    };
    int nf = 0, nr = 0;
    for (const auto& p : r.lhs.sp) nf += p.second;
    for (const auto& p : r.rhs.sp) nr += p.second;
    auto scaleA = [&](double A, int order) { return A * std::pow(1e-3, order - 1); };
    auto arr = [&](double A, double b, double E, int order) {
      return num(scaleA(A, order)) + " " + num(b) + " " + num(E * e_to_ta);
    };
    const bool pdep = !r.lhs.falloff.empty();
    std::string kind;
    if (!r.plog.empty()) {
      if (r.lhs.plus_m || pdep) ck_fail(PYJAC_E_UNSUPPORTED, ln, "PLOG with a third body");
      kind = "plog";
    } else if (!r.cheb.empty()) {
      if (r.lhs.plus_m) ck_fail(PYJAC_E_UNSUPPORTED, ln, "CHEB with +M");
      kind = "cheb";
    } else if (pdep) {
      if (r.low.empty() == r.high.empty()) ck_fail(PYJAC_E_PARSE, ln, "(+M) reaction needs exactly one of LOW and HIGH");
      kind = r.low.empty() ? "chemact" : "falloff";
    } else {
      kind = r.lhs.plus_m ? "thirdbody" : "elementary";
    }
    const std::string rev = !r.reversible ? "irrev" : (r.rev.empty() ? "kc" : "explicit");
    if (!r.reversible && !r.rev.empty()) ck_fail(PYJAC_E_PARSE, ln, "REV on an irreversible reaction");
    o << "  reaction " << kind << " " << rev << "\n    reactants " << side(r.lhs) << "\n    products "
      << side(r.rhs) << "\n";
    if (kind == "elementary") o << "    arrhenius " << arr(r.A, r.b, r.E, nf) << "\n";
    else if (kind == "thirdbody") o << "    arrhenius " << arr(r.A, r.b, r.E, nf + 1) << "\n";
    else if (kind == "falloff" || kind == "chemact") {
      const std::vector<double>& aux = kind == "falloff" ? r.low : r.high;
      if (aux.size() != 3) ck_fail(PYJAC_E_PARSE, ln, "LOW/HIGH needs A b E");
      // falloff: main line k_inf (order nf), LOW k0 (order nf + 1, [M] counted);
      // chemically activated: main line k0 (the rate's own order nf), HIGH
      // k_inf (order nf - 1, so that P_r = k0 [M] / k_inf is dimensionless)
      const bool fo = kind == "falloff";
      const double k0[3] = {fo ? aux[0] : r.A, fo ? aux[1] : r.b, fo ? aux[2] : r.E};
      const double ki[3] = {fo ? r.A : aux[0], fo ? r.b : aux[1], fo ? r.E : aux[2]};
      o << "    low " << arr(k0[0], k0[1], k0[2], fo ? nf + 1 : nf) << "\n    high "
        << arr(ki[0], ki[1], ki[2], fo ? nf : nf - 1) << "\n";
      if (!r.troe.empty() && !r.sri.empty()) ck_fail(PYJAC_E_PARSE, ln, "both TROE and SRI");
      if (!r.troe.empty()) {
        if (r.troe.size() != 3 && r.troe.size() != 4) ck_fail(PYJAC_E_PARSE, ln, "TROE needs 3 or 4 values");
        o << "    troe " << r.troe.size();
        for (double v : r.troe) o << " " << num(v);
        o << "\n";
      } else if (!r.sri.empty()) {
        if (r.sri.size() != 3 && r.sri.size() != 5) ck_fail(PYJAC_E_PARSE, ln, "SRI needs 3 or 5 values");
        o << "    sri " << r.sri.size();
        for (double v : r.sri) o << " " << num(v);
        o << "\n";
      } else {
        o << "    lindemann\n";
      }
    } else if (kind == "plog") {
      o << "    plog " << r.plog.size();
      for (const auto& pt : r.plog) o << " " << num(pt[0] * kAtm) << " " << arr(pt[1], pt[2], pt[3], nf);
      o << "\n";
    } else {   // cheb
      if (r.cheb.size() < 2) ck_fail(PYJAC_E_PARSE, ln, "CHEB needs the basis sizes");
      const int nT = (int)r.cheb[0], nP = (int)r.cheb[1];
      if (nT < 1 || nP < 1 || r.cheb[0] != nT || r.cheb[1] != nP || (int)r.cheb.size() != 2 + nT * nP)
        ck_fail(PYJAC_E_PARSE, ln, "CHEB needs nT nP and nT*nP coefficients");
      const double Tmin = r.tcheb.size() == 2 ? r.tcheb[0] : 300.0, Tmax = r.tcheb.size() == 2 ? r.tcheb[1] : 2500.0;
      const double Pmin = r.pcheb.size() == 2 ? r.pcheb[0] : 0.001, Pmax = r.pcheb.size() == 2 ? r.pcheb[1] : 100.0;
      o << "    cheb " << nT << " " << nP << " " << num(Tmin) << " " << num(Tmax) << " " << num(Pmin * kAtm) << " "
        << num(Pmax * kAtm);
      for (int q = 0; q < nT * nP; ++q) o << " " << num(r.cheb[2 + q] + (q == 0 ? -3.0 * (nf - 1) : 0.0));
      o << "\n";
    }
    // a Chebyshev fit already holds the pressure dependence: "(+M)" on it adds no collider
    if (kind != "cheb" && (r.lhs.plus_m || (pdep && r.lhs.falloff == "M"))) {
      o << "    collider mix " << r.eff.size();
      for (const auto& e : r.eff) o << " " << e.first << " " << num(e.second);
      o << "\n";
    } else if (pdep && kind != "cheb") {
      if (!r.eff.empty()) ck_fail(PYJAC_E_PARSE, ln, "efficiencies with a single collider species");
      o << "    collider species " << r.lhs.falloff << "\n";
    } else if (!r.eff.empty()) {
      ck_fail(PYJAC_E_PARSE, ln, "efficiencies on a reaction without a third body");
    }
    if (!r.rev.empty()) {
      if (r.rev.size() != 3) ck_fail(PYJAC_E_PARSE, ln, "REV needs A b E");
      o << "    reverse " << arr(r.rev[0], r.rev[1], r.rev[2], nr + (r.lhs.plus_m ? 1 : 0)) << "\n";
    }
  }
  o << "end\n";
  out = o.str();
}

}  // namespace

int chemkin_to_tokens(const std::string& mech, const std::string* thermo, std::string& out, std::string& msg) {
  try {
    convert(mech, thermo, out);
    return PYJAC_OK;
  } catch (const CkError& e) {
    msg = "Chemkin: " + e.msg;
    return e.code;
  } catch (const std::exception& e) {
    msg = std::string("Chemkin: ") + e.what();
    return PYJAC_E_PARSE;
  }
}

}  // namespace pyjac
