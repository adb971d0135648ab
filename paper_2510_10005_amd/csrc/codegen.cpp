// Per-mechanism HIP source generation: the code-generation step of the paper (Section 4.3),
// re-targeted to gfx950.  Like ChemGen, every reaction becomes straight-line code with its
// constants folded (A, b, Ea/R, stoichiometry, efficiencies, Troe parameters), the integer
// powers of concentrations and of (p_ref/RT) are unrolled into products or a single ln term,
// efficiencies equal to the default are dropped (eq. TB_optimization), and the analytic Jacobian
// is emitted from the chain rules of each rate form (Section 4.2) with only the entries the
// reaction touches.  Unlike ChemGen, ln A stays a runtime array (it is a differentiable
// parameter), and the emitted code is device code for one cell per GPU lane.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <set>
#include <sstream>
#include <stdexcept>
#include <string>
#include <type_traits>
#include <vector>

#include "mechanism.hpp"

namespace chem {

static const char* kPrelude =
#include "device_prelude.inc"
    ;
static const char* kKernels =
#include "device_kernels.inc"
    ;
static const char* kWave =
#include "device_wave.inc"
    ;
static const char* kBlock =
#include "device_block.inc"
    ;

// Rows of the Jacobian assembled per LDS part in the block form: the whole padded matrix when it
// is at most 64 (the factors then stay in LDS), else what fits the workgroup's LDS (160 KiB on
// gfx950) beside the records and vectors; mirrors the size of BkShared in device_block.inc.
static int block_part_rows(int n, int nr, int md) {
  const int np = (n + 15) / 16 * 16, js = np + 1;
  if (np <= 64) return np;
  // LDS of the block form outside the Jacobian part for n_pad > 64 (the BkShared members): 14
  // vectors, reductions, the records and the zero record, LU panel + pivot rows + 1/u_kk + T-row
  // sums, scalars; ints: pivot step of each row, row of each step, scalars
  const long fixed = 8L * (14L * np + 16 + static_cast<long>(nr + 1) * (3 + md) + 10L * np + 8) + 4L * (2L * np + 8) + 64;
  const long budget = 163840 - 1024 - fixed;
  long rows = budget / (8L * js);
  if (rows > np) rows = np;
  if (rows < 16) throw std::runtime_error("mechanism too large for the block form's LDS");
  return static_cast<int>(rows);
}

static std::string num(double v) {
  char buf[64];
  std::snprintf(buf, sizeof(buf), "%.17g", v);
  std::string s(buf);
  if (s.find_first_of(".eEn") == std::string::npos) s += ".0";  // keep it a double literal
  if (v < 0) return "(" + s + ")";
  return s;
}

// product of C[i]^nu over a side, as "C[a]*C[a]*C[b]" (or "1.0")
static std::string conc_product(const std::vector<std::pair<int, int>>& side, int skip = -1, int* coef = nullptr) {
  std::string out;
  for (auto& p : side) {
    int e = p.second;
    if (p.first == skip) {
      if (coef) *coef = e;
      e -= 1;
    }
    for (int r = 0; r < e; ++r) {
      if (!out.empty()) out += "*";
      out += "C[" + std::to_string(p.first) + "]";
    }
  }
  return out.empty() ? "1.0" : out;
}

// Jacobian element reference for full state index (rf, cf): in the reduced (active-species)
// system a column of a species that never changes is dropped; its rows are zero anyway.
static std::string jref(int rf, int cf, const std::vector<int>& red) {
  const int rr = red[rf], cr = red[cf];
  return "J(RED ? " + std::to_string(rr) + " : " + std::to_string(rf) + ", RED ? " + std::to_string(cr) + " : " +
         std::to_string(cf) + ")";
}

// One reaction's rate (kf, kr, q).  jac: also its production-rate and Jacobian contributions
// (mech_eval).  vjp: generic value type R and, instead of Jacobian entries, the contraction
// with the adjoint weights of mech_vjp: sig = sum_i nu_ij ut_i, g_j += q sig, v_k += sig dq/dy_k
// (the default-efficiency part of d[M]/dC goes to tbs, added to every species column at the end).
static void emit_rate(std::ostringstream& os, const Mechanism& m, int j, bool jac, const std::vector<int>& red,
                      bool vjp = false) {
  const Reaction& r = m.reactions[j];
  const std::string J = std::to_string(j);
  const std::string ty = vjp ? "R" : "double";
  os << "  { // reaction " << j << ": " << r.equation << "\n";
  // ln k = ln A + b ln T - (Ea/R) / T   (log form of the Arrhenius law, Section 2.2.1)
  os << "    const " << ty << " lnk = lnA[" << J << "]";
  if (r.k.b != 0.0) os << " + " << num(r.k.b) << "*lnT";
  if (r.k.theta != 0.0) os << " - " << num(r.k.theta) << "*invT";
  os << ";\n";
  const bool pd = r.kind != RxKind::Elementary;
  if (pd) {
    // [M] = default * M_c + sum over listed species of (alpha - default) C_i
    os << "    const " << ty << " M = ";
    if (r.default_eff == 1.0)
      os << "Mc";
    else if (r.default_eff == 0.0)
      os << "0.0";
    else
      os << num(r.default_eff) << "*Mc";
    for (auto& e : r.eff) os << " + " << num(e.second - r.default_eff) << "*C[" << e.first << "]";
    os << ";\n";
  }
  if (r.kind == RxKind::Elementary) {
    os << "    const " << ty << " kf = exp(lnk);\n";
  } else if (r.kind == RxKind::ThirdBody) {
    os << "    const " << ty << " kf = M*exp(lnk);\n";
  } else if (r.kind == RxKind::Plog) {
    // ln k linear in ln p between the tabulated sets around p = R T sum C, the end sets outside;
    // set i relative to the first: ln k_i = lnk + (lnA_i - lnA_0) + (b_i - b_0) ln T - (th_i - th_0)/T
    const auto& P = r.plog;
    const int np = static_cast<int>(P.size());
    os << "    " << ty << " kf, dlnkf_dT_fo, dlnkf_dM_fo;\n    {\n";
    os << "      const " << ty << " lnp = log(CHEM_R*T*M);\n";
    os << "      " << ty << " lk, dkT, dkp;\n";
    auto set_lnk = [&](int i) {
      const Arrhenius& k = P[i].second;
      return std::string("(lnk + ") + num(k.lnA - P[0].second.lnA) + " + " + num(k.b - P[0].second.b) + "*lnT - " +
             num(k.theta - P[0].second.theta) + "*invT)";
    };
    auto set_dT = [&](int i) {
      const Arrhenius& k = P[i].second;
      return std::string("((") + num(k.b) + " + " + num(k.theta) + "*invT)*invT)";
    };
    // !(lnp > p_0): a non-finite ln p (sum C <= 0 at a trial state) takes the lowest-pressure set,
    // the rule of the table-driven form and of the reference evaluation
    os << "      if (!(chem_val(lnp) > " << num(P[0].first) << ")) { lk = " << set_lnk(0) << "; dkT = " << set_dT(0)
       << "; dkp = 0.0; }\n";
    for (int i = 0; i + 1 < np; ++i) {
      const double inv = 1.0 / (P[i + 1].first - P[i].first);
      os << "      else if (chem_val(lnp) <= " << num(P[i + 1].first) << ") {\n";
      os << "        const " << ty << " k0 = " << set_lnk(i) << ", k1 = " << set_lnk(i + 1) << ";\n";
      os << "        const " << ty << " w = (lnp - " << num(P[i].first) << ")*" << num(inv) << ";\n";
      os << "        lk = k0 + w*(k1 - k0);\n        dkp = (k1 - k0)*" << num(inv) << ";\n";
      os << "        dkT = (1.0 - w)*" << set_dT(i) << " + w*" << set_dT(i + 1) << ";\n      }\n";
    }
    os << "      else { lk = " << set_lnk(np - 1) << "; dkT = " << set_dT(np - 1) << "; dkp = 0.0; }\n";
    os << "      kf = exp(lk);\n      dlnkf_dT_fo = dkT + dkp*invT;\n      dlnkf_dM_fo = dkp/M;\n    }\n";
  } else if (r.sri) {
    const double db = r.k0.b - r.k.b, dth = r.k0.theta - r.k.theta, dlnA = r.k0.lnA - r.k.lnA;
    os << "    " << ty << " kf, dlnkf_dT_fo, dlnkf_dM_fo;\n";
    os << "    chem_falloff_sri<" << (vjp ? "true" : (jac ? "JAC" : "false")) << ">(lnk, " << num(dlnA) << " + "
       << num(db) << "*lnT - " << num(dth) << "*invT, M, T, invT, lnT, " << num(r.k.b) << ", " << num(r.k.theta)
       << ", " << num(db) << ", " << num(dth) << ", " << num(r.sri_a) << ", " << num(r.sri_b) << ", "
       << num(1.0 / r.sri_c) << ", " << num(std::log(r.sri_d)) << ", " << num(r.sri_e)
       << ", kf, dlnkf_dT_fo, dlnkf_dM_fo);\n";
  } else {
    const double db = r.k0.b - r.k.b, dth = r.k0.theta - r.k.theta, dlnA = r.k0.lnA - r.k.lnA;
    os << "    " << ty << " kf, dlnkf_dT_fo, dlnkf_dM_fo;\n";
    os << "    chem_falloff<" << (vjp ? "true" : (jac ? "JAC" : "false")) << ", " << (r.troe ? "true" : "false") << ", "
       << (r.troe && r.troe_has_T2 ? "true" : "false") << ">(lnk, " << num(dlnA) << " + " << num(db) << "*lnT - "
       << num(dth) << "*invT, M, T, invT, " << num(r.k.b) << ", " << num(r.k.theta) << ", " << num(db) << ", "
       << num(dth) << ", " << num(r.troe ? r.troe_alpha : 0.0) << ", " << num(r.troe ? 1.0 / r.troe_T3 : 0.0) << ", "
       << num(r.troe ? 1.0 / r.troe_T1 : 0.0) << ", " << num(r.troe && r.troe_has_T2 ? r.troe_T2 : 0.0)
       << ", kf, dlnkf_dT_fo, dlnkf_dM_fo);\n";
  }
  auto nu = m.net(j);
  int dnu = 0;
  for (auto& p : nu) dnu += p.second;
  os << "    const " << ty << " Rf = kf*" << conc_product(r.reactants) << ";\n";
  if (r.reversible) {
    // ln K = -sum nu g/RT + (sum nu) ln(p_ref/(R T))   (eq. equilibrium-constant)
    os << "    const " << ty << " lnKc = -(";
    bool first = true;
    for (auto& p : nu) {
      if (!first) os << " + ";
      first = false;
      if (p.second == 1)
        os << "gRT[" << p.first << "]";
      else
        os << num(static_cast<double>(p.second)) << "*gRT[" << p.first << "]";
    }
    if (first) os << "0.0";
    os << ")";
    if (dnu != 0) os << " + " << num(static_cast<double>(dnu)) << "*(LNPREF_R - lnT)";
    os << ";\n";
    os << "    const " << ty << " kr = kf*exp(-lnKc);\n";
    os << "    const " << ty << " Rr = kr*" << conc_product(r.products) << ";\n";
  } else {
    os << "    const " << ty << " Rr = 0.0;\n";
  }
  os << "    const " << ty << " q = Rf - Rr;\n";
  if (!jac && !vjp) return;  // caller closes the block
  if (vjp) {
    os << "    const R sig = ";
    bool first = true;
    for (auto& p : nu) {
      os << (first ? "" : " + ") << num(static_cast<double>(p.second)) << "*ut[" << p.first << "]";
      first = false;
    }
    if (first) os << "0.0";
    os << ";\n    g[" << J << "] += chem_gpart(q*sig, gmode);\n";
    for (auto& p : nu) os << "    w[" << p.first << "] += " << num(static_cast<double>(p.second)) << "*q;\n";
  }
  for (auto& p : nu) {
    if (vjp) break;
    if (p.second == 1)
      os << "    w[" << p.first << "] += q;\n";
    else if (p.second == -1)
      os << "    w[" << p.first << "] -= q;\n";
    else
      os << "    w[" << p.first << "] = fma(" << num(static_cast<double>(p.second)) << ", q, w[" << p.first << "]);\n";
  }
  os << (vjp ? "    {\n" : "    if (JAC) {\n");
  if (r.kind == RxKind::Falloff || r.kind == RxKind::Plog) {
    os << "      const " << ty << " dlnkf_dT = dlnkf_dT_fo;\n";
  } else {
    os << "      const " << ty << " dlnkf_dT = (" << num(r.k.b) << " + " << num(r.k.theta) << "*invT)*invT;\n";
  }
  if (r.reversible) {
    os << "      const " << ty << " dlnKc_dT = (";
    bool first = true;
    for (auto& p : nu) {
      if (!first) os << " + ";
      first = false;
      if (p.second == 1)
        os << "hRT[" << p.first << "]";
      else
        os << num(static_cast<double>(p.second)) << "*hRT[" << p.first << "]";
    }
    if (first) os << "0.0";
    os << " - " << num(static_cast<double>(dnu)) << ")*invT;\n";
    os << "      const " << ty << " dqdT = q*dlnkf_dT + Rr*dlnKc_dT;\n";
  } else {
    os << "      const " << ty << " dqdT = q*dlnkf_dT;\n";
  }
  // d q / d C_k from mass action on each side
  std::map<int, std::string> dq;
  for (auto& p : r.reactants) {
    int c = 0;
    std::string pr = conc_product(r.reactants, p.first, &c);
    std::string t = "kf*" + (c > 1 ? num(static_cast<double>(c)) + "*" : std::string()) + pr;
    dq[p.first] = dq.count(p.first) ? dq[p.first] + " + " + t : t;
  }
  if (r.reversible) {
    for (auto& p : r.products) {
      int c = 0;
      std::string pr = conc_product(r.products, p.first, &c);
      std::string t = "kr*" + (c > 1 ? num(static_cast<double>(c)) + "*" : std::string()) + pr;
      dq[p.first] = dq.count(p.first) ? dq[p.first] + " - " + t : "-(" + t + ")";
    }
  }
  if (pd) {
    if (r.kind == RxKind::ThirdBody)
      os << "      const " << ty << " qM = q/M;\n";
    else
      os << "      const " << ty << " qM = q*dlnkf_dM_fo;\n";
    for (auto& e : r.eff) {
      std::string t = "qM*" + num(e.second - r.default_eff);
      dq[e.first] = dq.count(e.first) ? dq[e.first] + " + " + t : t;
    }
    if (vjp && r.default_eff != 0.0) os << "      tbs += " << num(r.default_eff) << "*(sig*qM);\n";
    if (!vjp && r.default_eff != 0.0) {
      for (auto& p : nu) {
        os << "      tbr[" << p.first << "] = fma(" << num(p.second * r.default_eff) << ", qM, tbr[" << p.first
           << "]);\n";
      }
    }
  }
  for (auto& d : dq) os << "      const " << ty << " dq" << d.first << " = " << d.second << ";\n";
  if (vjp) {
    os << "      v[0] += sig*dqdT;\n";
    for (auto& d : dq) os << "      v[" << 1 + d.first << "] += sig*dq" << d.first << ";\n";
    os << "    }\n";
    return;
  }
  for (auto& p : nu) {
    const std::string nv = num(static_cast<double>(p.second));
    auto acc = [&](int colf, const std::string& val) {
      const int rowf = 1 + p.first;
      const std::string ref = jref(rowf, colf, red);
      const std::string guard = red[colf] < 0 ? "if (!RED) " : "";
      if (p.second == 1)
        os << "      " << guard << ref << " += " << val << ";\n";
      else if (p.second == -1)
        os << "      " << guard << ref << " -= " << val << ";\n";
      else
        os << "      " << guard << ref << " = fma(" << nv << ", " << val << ", " << ref << ");\n";
    };
    acc(0, "dqdT");
    for (auto& d : dq) acc(1 + d.first, "dq" + std::to_string(d.first));
  }
  os << "    }\n";
}

// Constant tables of the one-wave-per-cell form (large mechanisms): reactions at positions sorted
// by rate form (elementary, third-body, Lindemann, Troe, Troe with T**, SRI, P-log) so that a round of 64
// lanes mostly runs one branch; species reaction lists (CSR over positions) for the gathers.
template <class T>
static void emit_array(std::ostringstream& os, const char* type, const char* name, const std::vector<T>& v) {
  os << "static __device__ const " << type << " " << name << "[" << (v.empty() ? 1 : v.size()) << "] = {";
  if (v.empty()) os << "0";
  for (size_t i = 0; i < v.size(); ++i) {
    if (i) os << ", ";
    if constexpr (std::is_floating_point<T>::value)
      os << num(v[i]);
    else
      os << v[i];
  }
  os << "};\n";
}

static int rate_kind(const Reaction& r) {
  if (r.kind == RxKind::Elementary) return 0;
  if (r.kind == RxKind::ThirdBody) return 1;
  if (r.kind == RxKind::Plog) return 6;
  if (r.sri) return 5;
  if (!r.troe) return 2;
  return r.troe_has_T2 ? 4 : 3;
}

// table position p -> reaction index (reactions grouped by rate kind, stable)
static std::vector<int> table_positions(const Mechanism& m) {
  std::vector<int> pos(m.nr());
  for (int j = 0; j < m.nr(); ++j) pos[j] = j;
  std::stable_sort(pos.begin(), pos.end(),
                   [&](int a, int b) { return rate_kind(m.reactions[a]) < rate_kind(m.reactions[b]); });
  return pos;
}

// species whose concentration a reaction's rate of progress depends on (its record lists dq/dC of
// these, ascending): reactants, products of reversible reactions, enhanced colliders
static std::vector<std::vector<int>> record_species(const Mechanism& m) {
  std::vector<std::vector<int>> dsp(m.nr());
  for (int j = 0; j < m.nr(); ++j) {
    const Reaction& r = m.reactions[j];
    std::set<int> d;
    for (auto& p : r.reactants) d.insert(p.first);
    if (r.reversible)
      for (auto& p : r.products) d.insert(p.first);
    if (r.kind != RxKind::Elementary)
      for (auto& e : r.eff) d.insert(e.first);
    dsp[j].assign(d.begin(), d.end());
  }
  return dsp;
}

// returns the number of derivative-record species per reaction (WV_MD)
static int emit_wave_tables(std::ostringstream& os, const Mechanism& m) {
  const int ns = m.ns(), nr = m.nr();
  for (const Species& sp : m.species)
    if (sp.poly)
      throw std::runtime_error("polynomial-cp thermo is supported for mechanisms of at most 24 state components");
  auto kind_of = [&](const Reaction& r) { return rate_kind(r); };
  const std::vector<int> pos = table_positions(m);
  const std::vector<std::vector<int>> dsp = record_species(m);
  int MR = 1, MP = 1, MN = 1, ME = 1, MD = 1;
  for (int j = 0; j < nr; ++j) {
    const Reaction& r = m.reactions[j];
    MR = std::max(MR, static_cast<int>(r.reactants.size()));
    MP = std::max(MP, static_cast<int>(r.products.size()));
    MN = std::max(MN, static_cast<int>(m.net(j).size()));
    ME = std::max(ME, static_cast<int>(r.eff.size()));
    MD = std::max(MD, static_cast<int>(dsp[j].size()));
  }
  os << "#define WV_MR " << MR << "\n#define WV_MP " << MP << "\n#define WV_MN " << MN << "\n#define WV_ME " << ME
     << "\n#define WV_MD " << MD << "\n";
  std::vector<int> rx, kind, rev, rs, rc, ps, pc, nus, es, ds, plo, pln;
  std::vector<double> b, th, fo, tr, dnu, nuv, deff, ev, sri, pl;
  for (int p = 0; p < nr; ++p) {
    const int j = pos[p];
    const Reaction& r = m.reactions[j];
    rx.push_back(j);
    kind.push_back(kind_of(r));
    rev.push_back(r.reversible ? 1 : 0);
    b.push_back(r.k.b);
    th.push_back(r.k.theta);
    const bool fall = r.kind == RxKind::Falloff;
    fo.push_back(fall ? r.k0.lnA - r.k.lnA : 0.0);
    fo.push_back(fall ? r.k0.b - r.k.b : 0.0);
    fo.push_back(fall ? r.k0.theta - r.k.theta : 0.0);
    tr.push_back(r.troe ? r.troe_alpha : 0.0);
    tr.push_back(r.troe ? 1.0 / r.troe_T3 : 0.0);
    tr.push_back(r.troe ? 1.0 / r.troe_T1 : 0.0);
    tr.push_back(r.troe && r.troe_has_T2 ? r.troe_T2 : 0.0);
    // SRI constants (a, b, 1/c, ln d, e) and P-log slices (ln p, ln A, b and Ea/R relative to the
    // first set, then b and Ea/R) of the shared table
    sri.push_back(r.sri ? r.sri_a : 0.0);
    sri.push_back(r.sri ? r.sri_b : 0.0);
    sri.push_back(r.sri ? 1.0 / r.sri_c : 0.0);
    sri.push_back(r.sri ? std::log(r.sri_d) : 0.0);
    sri.push_back(r.sri ? r.sri_e : 0.0);
    plo.push_back(static_cast<int>(pl.size() / 6));
    pln.push_back(static_cast<int>(r.plog.size()));
    for (auto& e : r.plog) {
      pl.push_back(e.first);
      pl.push_back(e.second.lnA - r.plog.front().second.lnA);
      pl.push_back(e.second.b - r.plog.front().second.b);
      pl.push_back(e.second.theta - r.plog.front().second.theta);
      pl.push_back(e.second.b);
      pl.push_back(e.second.theta);
    }
    deff.push_back(r.default_eff);
    for (int i = 0; i < MR; ++i) {
      const bool u = i < static_cast<int>(r.reactants.size());
      rs.push_back(u ? r.reactants[i].first : -1);
      rc.push_back(u ? r.reactants[i].second : 0);
    }
    for (int i = 0; i < MP; ++i) {
      const bool u = i < static_cast<int>(r.products.size());
      ps.push_back(u ? r.products[i].first : -1);
      pc.push_back(u ? r.products[i].second : 0);
    }
    auto nu = m.net(j);
    int dn = 0, i = 0;
    for (auto& q : nu) {
      nus.push_back(q.first);
      nuv.push_back(static_cast<double>(q.second));
      dn += q.second;
      ++i;
    }
    for (; i < MN; ++i) {
      nus.push_back(-1);
      nuv.push_back(0.0);
    }
    dnu.push_back(static_cast<double>(dn));
    i = 0;
    if (r.kind != RxKind::Elementary)
      for (auto& e : r.eff) {
        es.push_back(e.first);
        ev.push_back(e.second - r.default_eff);
        ++i;
      }
    for (; i < ME; ++i) {
      es.push_back(-1);
      ev.push_back(0.0);
    }
    for (i = 0; i < MD; ++i) ds.push_back(i < static_cast<int>(dsp[j].size()) ? dsp[j][i] : -1);
  }
  emit_array(os, "int", "wv_rx", rx);
  emit_array(os, "int", "wv_kind", kind);
  emit_array(os, "int", "wv_rev", rev);
  emit_array(os, "double", "wv_b", b);
  emit_array(os, "double", "wv_th", th);
  emit_array(os, "double", "wv_fo", fo);
  emit_array(os, "double", "wv_tr", tr);
  emit_array(os, "double", "wv_sri", sri);
  emit_array(os, "int", "wv_plo", plo);
  emit_array(os, "int", "wv_pln", pln);
  if (pl.empty()) pl.assign(6, 0.0);
  emit_array(os, "double", "wv_pl", pl);
  emit_array(os, "double", "wv_deff", deff);
  emit_array(os, "double", "wv_dnu", dnu);
  emit_array(os, "int", "wv_rs", rs);
  emit_array(os, "int", "wv_rc", rc);
  emit_array(os, "int", "wv_ps", ps);
  emit_array(os, "int", "wv_pc", pc);
  emit_array(os, "int", "wv_nus", nus);
  emit_array(os, "double", "wv_nuv", nuv);
  emit_array(os, "int", "wv_es", es);
  emit_array(os, "double", "wv_ev", ev);
  emit_array(os, "int", "wv_ds", ds);
  // species s: positions p (ascending) with nu_sp != 0
  std::vector<int> ptr(1, 0), sp_p;
  std::vector<double> sp_v;
  for (int s = 0; s < ns; ++s) {
    for (int p = 0; p < nr; ++p) {
      auto nu = m.net(pos[p]);
      auto it = nu.find(s);
      if (it != nu.end()) {
        sp_p.push_back(p);
        sp_v.push_back(static_cast<double>(it->second));
      }
    }
    ptr.push_back(static_cast<int>(sp_p.size()));
  }
  emit_array(os, "int", "wv_sp_ptr", ptr);
  // gather entries, 16 bytes each: x = position | (nu & 255) << 16, y..z = the record species
  // (s + 1, 0 = none) of that position, one byte each (MD <= 8)
  if (MD > 8) throw std::runtime_error("more than 8 derivative-record species per reaction");
  std::vector<unsigned> sp_e;
  for (size_t i = 0; i < sp_p.size(); ++i) {
    const int nu = static_cast<int>(sp_v[i]);
    if (nu < -128 || nu > 127 || sp_p[i] > 65535) throw std::runtime_error("gather entry out of range");
    const int j = pos[sp_p[i]];
    unsigned w[4] = {static_cast<unsigned>(sp_p[i]) | (static_cast<unsigned>(nu & 255) << 16), 0u, 0u, 0u};
    for (int d = 0; d < static_cast<int>(dsp[j].size()); ++d)
      w[1 + d / 4] |= static_cast<unsigned>(dsp[j][d] + 1) << (8 * (d % 4));
    sp_e.insert(sp_e.end(), w, w + 4);
  }
  if (sp_e.empty()) sp_e.assign(4, 0u);
  os << "static __device__ const unsigned wv_sp_e[" << sp_e.size() << "] __attribute__((aligned(16))) = {";
  for (size_t i = 0; i < sp_e.size(); ++i) os << (i ? ", " : "") << sp_e[i] << "u";
  os << "};\n";
  int maxc = 0;
  for (auto& r : m.reactions) {
    for (auto& q : r.reactants) maxc = std::max(maxc, q.second);
    for (auto& q : r.products) maxc = std::max(maxc, q.second);
  }
  os << "#define WV_MAXC " << maxc << "\n";
  std::vector<double> nasa, tmid;
  for (int s = 0; s < ns; ++s) {
    for (int c = 0; c < 7; ++c) nasa.push_back(m.species[s].lo[c]);
    for (int c = 0; c < 7; ++c) nasa.push_back(m.species[s].hi[c]);
    tmid.push_back(m.species[s].T_mid);
  }
  emit_array(os, "double", "wv_nasa", nasa);
  emit_array(os, "double", "wv_tmid", tmid);
  return MD;
}

// Assembly tables of the block form, stored interleaved by thread (entry j of thread t at
// j * 256 + t, every thread padded to the same count) so that a step of the loops over them is one
// coalesced load for the workgroup and the loops have a uniform trip count.  Padding refers to the
// zero record after the last reaction (position NR).
//  * bk_sp_ops [BK_SPN][256]: for species t, its table positions p (ascending) with nonzero net
//    coefficient: p << 8 | (nu & 255); the production rate, dS/dT and the default-efficiency
//    third-body part of its row are sums over these.
//  * bk_cs_ops [BK_CS_PARTS][BK_CSN][256]: the listed-species part of the Jacobian.  The species
//    rows are assembled in parts of `part` matrix rows (row 1 + s for species s, parts starting at
//    row 1); every structural nonzero (1 + s, 1 + k) of a part is one slot, the sum over the
//    positions p (ascending) whose net coefficient of s is nonzero and whose record lists k of
//    nu_sp times that record entry.  Slots go longest first to the least loaded thread; a thread's
//    slots are consecutive runs of its ops.  Op: low word record index << 8 | (nu & 255), high
//    word the slot's destination (row in the part << 16 | column) on its last term, else ~0.
static void emit_block_jac_tables(std::ostringstream& os, const Mechanism& m, int part, int md) {
  constexpr int kThreads = 256;   // the block form's workgroup size (BK_T)
  const int ns = m.ns(), nr = m.nr(), n = m.n(), rec = 3 + md;
  const std::vector<int> pos = table_positions(m);
  const std::vector<std::vector<int>> dsp = record_species(m);
  const int nparts = (n - 1 + part - 1) / part;
  if (static_cast<long>(nr + 1) * rec >= (1L << 24)) throw std::runtime_error("reaction record table too large");
  const unsigned zero_rec = static_cast<unsigned>(nr) * static_cast<unsigned>(rec);
  // species sums
  std::vector<std::vector<unsigned>> sp_ops(kThreads);
  struct Slot {
    int row, col;
    std::vector<unsigned> terms;
  };
  std::vector<std::vector<Slot>> parts(nparts);
  for (int s = 0; s < ns; ++s) {
    std::vector<std::vector<unsigned>> by_col(ns);
    for (int p = 0; p < nr; ++p) {
      const int j = pos[p];
      const auto nu = m.net(j);
      const auto it = nu.find(s);
      if (it == nu.end()) continue;
      if (it->second < -128 || it->second > 127) throw std::runtime_error("net coefficient out of range");
      const unsigned c = static_cast<unsigned>(it->second & 255);
      sp_ops[s].push_back((static_cast<unsigned>(p) << 8) | c);
      for (size_t d = 0; d < dsp[j].size(); ++d)
        by_col[dsp[j][d]].push_back(((static_cast<unsigned>(p) * rec + 3 + static_cast<unsigned>(d)) << 8) | c);
    }
    const int row = 1 + s, pi = (row - 1) / part;
    for (int k = 0; k < ns; ++k)
      if (!by_col[k].empty()) parts[pi].push_back(Slot{row - (1 + pi * part), 1 + k, by_col[k]});
  }
  size_t spn = 1;
  for (auto& v : sp_ops) spn = std::max(spn, v.size());
  std::vector<unsigned> sp_flat(spn * kThreads, static_cast<unsigned>(nr) << 8);
  for (int t = 0; t < kThreads; ++t)
    for (size_t j = 0; j < sp_ops[t].size(); ++j) sp_flat[j * kThreads + t] = sp_ops[t][j];
  // slots
  std::vector<std::vector<std::vector<unsigned long long>>> th_ops(nparts, std::vector<std::vector<unsigned long long>>(kThreads));
  size_t csn = 1;
  for (int pi = 0; pi < nparts; ++pi) {
    std::vector<Slot>& sl = parts[pi];
    std::vector<int> order(sl.size());
    for (size_t i = 0; i < sl.size(); ++i) order[i] = static_cast<int>(i);
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return sl[a].terms.size() > sl[b].terms.size(); });
    std::vector<size_t> load(kThreads, 0);
    std::vector<std::vector<int>> own(kThreads);
    for (int i : order) {
      const int th = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
      load[th] += sl[i].terms.size();
      own[th].push_back(i);
    }
    for (int th = 0; th < kThreads; ++th) {
      std::sort(own[th].begin(), own[th].end());
      for (int i : own[th]) {
        const unsigned long long dst = (static_cast<unsigned long long>(sl[i].row) << 16) | static_cast<unsigned>(sl[i].col);
        for (size_t e = 0; e < sl[i].terms.size(); ++e) {
          const unsigned long long hi = e + 1 == sl[i].terms.size() ? dst : 0xffffffffull;
          th_ops[pi][th].push_back((hi << 32) | sl[i].terms[e]);
        }
      }
      csn = std::max(csn, th_ops[pi][th].size());
    }
  }
  const unsigned long long pad = (0xffffffffull << 32) | (static_cast<unsigned long long>(zero_rec) << 8);
  std::vector<unsigned long long> cs_flat(static_cast<size_t>(nparts) * csn * kThreads, pad);
  for (int pi = 0; pi < nparts; ++pi)
    for (int th = 0; th < kThreads; ++th)
      for (size_t j = 0; j < th_ops[pi][th].size(); ++j)
        cs_flat[(static_cast<size_t>(pi) * csn + j) * kThreads + th] = th_ops[pi][th][j];
  os << "#define BK_SPN " << spn << "\n#define BK_CS_PARTS " << nparts << "\n#define BK_CSN " << csn << "\n";
  emit_array(os, "unsigned", "bk_sp_ops", sp_flat);
  os << "static __device__ const unsigned long long bk_cs_ops[" << cs_flat.size() << "] = {";
  for (size_t i = 0; i < cs_flat.size(); ++i) os << (i ? ", " : "") << cs_flat[i] << "ull";
  os << "};\n";
}

std::string generate_source(const Mechanism& m, int dense_limit, bool full_system) {
  std::ostringstream os;
  const int ns = m.ns(), nr = m.nr(), n = m.n();
  full_system = full_system && n <= dense_limit;
  os << kPrelude;
  os << "// ---------------------------------------------------------------- generated mechanism block\n";
  os << "#define NS " << ns << "\n#define NY " << n << "\n#define NR " << (nr > 0 ? nr : 1) << "\n";
  os << "#define CHEM_DENSE " << (n <= dense_limit ? 1 : 0) << "\n";
  // full-system build: the integrators solve for every state component (the reactor energy mode)
  os << "#define CHEM_FULL_SYSTEM " << (full_system ? 1 : 0) << "\n";
  os << "#if CHEM_DENSE\n#define CHEM_MUNROLL _Pragma(\"unroll\")\n#define CHEM_EVAL_INLINE __forceinline__\n"
        "#else\n#define CHEM_MUNROLL _Pragma(\"unroll 1\")\n#define CHEM_EVAL_INLINE __noinline__\n#endif\n";
  os << "#define CHEM_R 8314.462618\n";
  // The Rosenbrock adjoint kernel calls the mechanism evaluation and the vector-Jacobian product out
  // of line for mechanisms with P-log reactions (fully inlined there it computed wrong values on the
  // GPU); inline otherwise.
  bool any_plog = false;
  for (auto& r : m.reactions) any_plog = any_plog || r.kind == RxKind::Plog;
  os << "#define CHEM_ADJ_CALL " << (any_plog ? "__noinline__" : "CHEM_EVAL_INLINE") << "\n";
  os << "#define LNPREF_R " << num(std::log(m.p_ref / kR)) << "\n";
  os << "static __device__ const double mech_W[NS] = {";
  for (int i = 0; i < ns; ++i) os << (i ? ", " : "") << num(m.species[i].W);
  os << "};\n";
  os << "static __device__ const double mech_RW[NS] = {";
  for (int i = 0; i < ns; ++i) os << (i ? ", " : "") << num(kR / m.species[i].W);
  os << "};\n";

  // ---- thermo: NASA-7 (Table 1, n_p = 4) in Horner form; each lane selects the coefficient set of
  // its range (T < T_mid: low, else high).  Variants return only what a caller needs.
  std::map<double, std::vector<int>> groups;
  for (int i = 0; i < ns; ++i) groups[m.species[i].T_mid].push_back(i);
  // Single-range polynomial species (Section 2.1): cp/R = sum a_k T^k, h/RT = sum a_k T^k/(k+1)
  // + h0/T, s/R = a_0 ln T + sum_(k>=1) a_k T^k/k + s0, d(cp/R)/dT = sum k a_k T^(k-1), in Horner form
  auto horner = [&](const std::vector<double>& c) {
    std::string e = num(c.back());
    for (int k = static_cast<int>(c.size()) - 2; k >= 0; --k) e = num(c[k]) + " + T*(" + e + ")";
    return e;
  };
  auto poly_cp = [&](const Species& s) { return horner(s.cp); };
  auto poly_h = [&](const Species& s) {
    std::vector<double> b(s.cp.size());
    for (size_t k = 0; k < b.size(); ++k) b[k] = s.cp[k] / static_cast<double>(k + 1);
    return horner(b) + " + " + num(s.h0) + "*invT";
  };
  auto poly_s = [&](const Species& s) {
    std::string e = num(s.cp[0]) + "*lnT + " + num(s.s0);
    if (s.cp.size() > 1) {
      std::vector<double> c(s.cp.size() - 1);
      for (size_t k = 1; k < s.cp.size(); ++k) c[k - 1] = s.cp[k] / static_cast<double>(k);
      e += " + T*(" + horner(c) + ")";
    }
    return e;
  };
  auto poly_dcp = [&](const Species& s) {
    if (s.cp.size() < 2) return std::string("0.0");
    std::vector<double> d(s.cp.size() - 1);
    for (size_t k = 1; k < s.cp.size(); ++k) d[k - 1] = static_cast<double>(k) * s.cp[k];
    return horner(d);
  };
  // what: bit 1 = cp, 2 = h, 4 = s, 8 = g (needs h and s), 16 = dcp
  auto emit_thermo = [&](const std::string& name, const std::string& params, int what) {
    os << "__device__ __forceinline__ void " << name << "(" << params << ") {\n";
    for (auto& g : groups) {
      os << "  {\n    const bool hi = T >= " << num(g.first) << ";\n";
      for (int i : g.second) {
        const Species& s = m.species[i];
        const std::string I = std::to_string(i);
        os << "    { // " << s.name << "\n";
        if (s.poly) {
          if (what & 1) os << "      cpR[" << I << "] = " << poly_cp(s) << ";\n";
          if (what & 2 || what & 8) os << "      const double h_ = " << poly_h(s) << ";\n";
          if (what & 2) os << "      hRT[" << I << "] = h_;\n";
          if (what & 4 || what & 8) os << "      const double s_ = " << poly_s(s) << ";\n";
          if (what & 4) os << "      sR[" << I << "] = s_;\n";
          if (what & 8) os << "      gRT[" << I << "] = h_ - s_;\n";
          if (what & 16) os << "      dcpR[" << I << "] = " << poly_dcp(s) << ";\n";
        } else {  // select the coefficient set per lane, then Horner
          auto a = [&](int k) { return std::string("(hi ? ") + num(s.hi[k]) + " : " + num(s.lo[k]) + ")"; };
          if (what & 1) os << "      cpR[" << I << "] = " << a(0) << " + T*(" << a(1) << " + T*(" << a(2) << " + T*(" << a(3) << " + T*" << a(4) << ")));\n";
          if (what & 2 || what & 8)
            os << "      const double h_ = " << a(0) << " + T*(0.5*" << a(1) << " + T*((1.0/3.0)*" << a(2)
               << " + T*(0.25*" << a(3) << " + T*(0.2*" << a(4) << ")))) + " << a(5) << "*invT;\n";
          if (what & 2) os << "      hRT[" << I << "] = h_;\n";
          if (what & 4 || what & 8)
            os << "      const double s_ = " << a(0) << "*lnT + T*(" << a(1) << " + T*(0.5*" << a(2) << " + T*((1.0/3.0)*"
               << a(3) << " + T*(0.25*" << a(4) << ")))) + " << a(6) << ";\n";
          if (what & 4) os << "      sR[" << I << "] = s_;\n";
          if (what & 8) os << "      gRT[" << I << "] = h_ - s_;\n";
          if (what & 16) os << "      dcpR[" << I << "] = " << a(1) << " + T*(2.0*" << a(2) << " + T*(3.0*" << a(3) << " + T*(4.0*" << a(4) << ")));\n";
        }
        os << "    }\n";
      }
      os << "  }\n";
    }
    os << "}\n";
  };
  emit_thermo("mech_thermo", "double T, double lnT, double invT, double (&cpR)[NS], double (&hRT)[NS], "
              "double (&sR)[NS], double (&gRT)[NS], double (&dcpR)[NS]", 1 | 2 | 4 | 8 | 16);
  emit_thermo("mech_thermo_hg", "double T, double lnT, double invT, double (&hRT)[NS], double (&gRT)[NS]", 2 | 8);
  emit_thermo("mech_thermo_g", "double T, double lnT, double invT, double (&gRT)[NS]", 8);
  emit_thermo("mech_thermo_cp", "double T, double (&cpR)[NS], double (&dcpR)[NS]", 1 | 16);
  emit_thermo("mech_thermo_hcp", "double T, double invT, double (&hRT)[NS], double (&cpR)[NS]", 1 | 2);

  bool any_pd = false;
  for (auto& r : m.reactions) any_pd = any_pd || r.kind != RxKind::Elementary;
  // active state components: T and every species with a non-zero net coefficient somewhere
  std::vector<int> red(n, -1);
  std::vector<int> act;
  std::vector<bool> sp_active(ns, false);
  for (int j = 0; j < nr; ++j)
    for (auto& p : m.net(j)) sp_active[p.first] = true;
  if (full_system) std::fill(sp_active.begin(), sp_active.end(), true);
  red[0] = 0;
  act.push_back(0);
  for (int i = 0; i < ns; ++i)
    if (sp_active[i]) {
      red[1 + i] = static_cast<int>(act.size());
      act.push_back(1 + i);
    }
  os << "#define NA " << act.size() << "\n";
  os << "__device__ __forceinline__ constexpr int act_full(int a) {\n  constexpr int t[NA] = {";
  for (size_t a = 0; a < act.size(); ++a) os << (a ? ", " : "") << act[a];
  os << "};\n  return t[a];\n}\n";

  const bool wave = n > dense_limit;
  os << "#define CHEM_WAVE " << (wave ? 1 : 0) << "\n";
  // n <= 64: the API kernels of the one-wavefront-per-cell form; larger: those of the block form
  const bool wave_api = n <= 64;
  os << "#define CHEM_WAVE_API " << (wave && wave_api ? 1 : 0) << "\n";
  if (wave && wave_api) {
    // source terms alone need only C, g/RT and the production rates per cell, few enough values
    // for one cell per lane with the constants folded into straight-line code (API kernel)
    os << "__device__ void mech_source_lane(const double (&y)[NY], const double* __restrict__ lnA, int energy,"
          " double (&S)[NY]) {\n";
    os << "  const double T = y[0];\n  const double lnT = log(T);\n  const double invT = 1.0 / T;\n";
    os << "  double C[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) C[i] = y[1 + i];\n";
    os << "  double gRT[NS];\n  mech_thermo_g(T, lnT, invT, gRT);\n";
    if (any_pd) os << "  double Mc = 0.0;\n#pragma unroll\n  for (int i = 0; i < NS; ++i) Mc += C[i];\n";
    os << "  double w[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) w[i] = 0.0;\n";
    for (int j = 0; j < nr; ++j) {
      emit_rate(os, m, j, false, red);
      for (auto& p : m.net(j)) {
        if (p.second == 1)
          os << "    w[" << p.first << "] += q;\n";
        else if (p.second == -1)
          os << "    w[" << p.first << "] -= q;\n";
        else
          os << "    w[" << p.first << "] = fma(" << num(static_cast<double>(p.second)) << ", q, w[" << p.first << "]);\n";
      }
      os << "  }\n";
    }
    os << "  double hRT[NS], cpR[NS];\n  mech_thermo_hcp(T, invT, hRT, cpR);\n";
    os << "  const double off = energy == 1 ? 1.0 : 0.0;\n  double N = 0.0, D = 0.0;\n";
    os << "#pragma unroll\n  for (int i = 0; i < NS; ++i) {\n    N = fma(hRT[i] - off, w[i], N);\n"
          "    D = fma(C[i], cpR[i] - off, D);\n  }\n";
    os << "  S[0] = -T * N / D;\n#pragma unroll\n  for (int i = 0; i < NS; ++i) S[1 + i] = w[i];\n}\n";
  }
  if (wave) {
    const int md = emit_wave_tables(os, m);
    const int part = block_part_rows(n, nr > 0 ? nr : 1, md);
    os << "#define BK_PART " << part << "\n";
    emit_block_jac_tables(os, m, part, md);
    os << kKernels;
    os << kWave;
    os << kBlock;
    return os.str();
  }

  // ---- source terms and Jacobian
  os << "// RED: J is the active-component system (NA x NA); otherwise the full NY x NY matrix\n";
  os << "template <bool JAC, class MAT, bool RED = false>\n"
        "__device__ CHEM_EVAL_INLINE void mech_eval(const double (&y)[NY], const double* __restrict__ lnA, int energy,"
        " double (&S)[NY], MAT& J) {\n";
  os << "  const double T = y[0];\n  const double lnT = log(T);\n  const double invT = 1.0 / T;\n";
  os << "  double C[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) C[i] = y[1 + i];\n";
  os << "  double hRT[NS], gRT[NS];\n";
  os << "  if (JAC) mech_thermo_hg(T, lnT, invT, hRT, gRT); else mech_thermo_g(T, lnT, invT, gRT);\n";
  if (any_pd) os << "  double Mc = 0.0;\n#pragma unroll\n  for (int i = 0; i < NS; ++i) Mc += C[i];\n";
  os << "  double w[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) w[i] = 0.0;\n";
  if (any_pd) os << "  double tbr[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) tbr[i] = 0.0;\n";
  os << "  if (JAC) {\n    CHEM_MUNROLL\n    for (int i = 0; i < MAT::DIM; ++i) {\n      CHEM_MUNROLL\n"
        "      for (int k = 0; k < MAT::DIM; ++k) J(i, k) = 0.0;\n    }\n  }\n";
  for (int j = 0; j < nr; ++j) {
    emit_rate(os, m, j, true, red);
    os << "  }\n";
  }
  os << "  double cpR[NS], dcpR[NS];\n";
  os << "  if (JAC) mech_thermo_cp(T, cpR, dcpR); else mech_thermo_hcp(T, invT, hRT, cpR);\n";
  os << "  const double off = energy == 1 ? 1.0 : 0.0;\n";
  os << "  double hw[NS], cw[NS], N = 0.0, D = 0.0;\n";
  os << "#pragma unroll\n  for (int i = 0; i < NS; ++i) {\n    hw[i] = hRT[i] - off;\n    cw[i] = cpR[i] - off;\n"
        "    N = fma(hw[i], w[i], N);\n    D = fma(C[i], cw[i], D);\n  }\n";
  os << "  const double invD = 1.0 / D;\n";
  os << "  S[0] = -T * N * invD;\n#pragma unroll\n  for (int i = 0; i < NS; ++i) S[1 + i] = w[i];\n";
  os << "  if (JAC) {\n";
  // dense part of the third-body/falloff derivatives: d[M]/dC_k = default efficiency
  if (any_pd) {
    for (int i = 0; i < ns; ++i) {
      if (!sp_active[i]) continue;
      for (int k = 0; k < ns; ++k) {
        const std::string ref = jref(1 + i, 1 + k, red);
        os << "    " << (red[1 + k] < 0 ? "if (!RED) " : "") << ref << " += tbr[" << i << "];\n";
      }
    }
  }
  os << "    const double A = T * N * invD * invD;\n";
  os << "    double s1 = 0.0, s2 = 0.0, s3 = 0.0;\n";
  os << "#pragma unroll\n    for (int i = 0; i < NS; ++i) {\n      s1 = fma(cw[i], w[i], s1);\n      s3 = fma(C[i], dcpR[i], s3);\n    }\n";
  for (int i = 0; i < ns; ++i)
    if (sp_active[i]) os << "    s2 = fma(hw[" << i << "], " << jref(1 + i, 0, red) << ", s2);\n";
  os << "    " << jref(0, 0, red) << " = -(s1 + T * s2) * invD + A * s3;\n";
  for (int k = 0; k < ns; ++k) {
    os << "    " << (red[1 + k] < 0 ? "if (!RED) " : "") << "{\n      double t = 0.0;\n";
    for (int i = 0; i < ns; ++i)
      if (sp_active[i]) os << "      t = fma(hw[" << i << "], " << jref(1 + i, 1 + k, red) << ", t);\n";
    os << "      " << jref(0, 1 + k, red) << " = -T * t * invD + A * cw[" << k << "];\n    }\n";
  }
  os << "  }\n}\n\n";
  // ---- d/d lnA contraction for the adjoint: g_j += q_j (sum_i nu_ij mu_i - mu_T T sum_i nu_ij hw_i / D)
  os << "template <class GACC>\n"
        "__device__ CHEM_EVAL_INLINE void mech_grad(const double (&y)[NY], const double* __restrict__ lnA, int energy,"
        " const double (&mu)[NY], GACC& g) {\n";
  os << "  const double T = y[0];\n  const double lnT = log(T);\n  const double invT = 1.0 / T;\n";
  os << "  double C[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) C[i] = y[1 + i];\n";
  os << "  double cpR[NS], hRT[NS], sR[NS], gRT[NS], dcpR[NS];\n";
  os << "  mech_thermo(T, lnT, invT, cpR, hRT, sR, gRT, dcpR);\n";
  if (any_pd) os << "  double Mc = 0.0;\n#pragma unroll\n  for (int i = 0; i < NS; ++i) Mc += C[i];\n";
  os << "  const double off = energy == 1 ? 1.0 : 0.0;\n  double D = 0.0;\n"
        "#pragma unroll\n  for (int i = 0; i < NS; ++i) D = fma(C[i], cpR[i] - off, D);\n";
  os << "  const double muT = -T * mu[0] / D;\n";
  if (full_system) {
    // reactor mode (full-system build): d g / d lnA_j = q_j (sum_i nu_ij / sum C - dH_j / D) adds
    // -(mu . C) times that to the contraction
    os << "  double aC = 0.0, aH = 0.0;\n  if (energy == 2) {\n    double muC = 0.0, c = 0.0;\n"
          "#pragma unroll\n    for (int i = 0; i < NS; ++i) {\n      muC = fma(mu[1 + i], C[i], muC);\n"
          "      c += C[i];\n    }\n    aC = muC / c;\n    aH = muC / D;\n  }\n";
  }
  for (int j = 0; j < nr; ++j) {
    emit_rate(os, m, j, false, red);
    auto nu = m.net(j);
    os << "    const double dH = ";
    bool first = true;
    for (auto& p : nu) {
      if (!first) os << " + ";
      first = false;
      os << num(static_cast<double>(p.second)) << "*(hRT[" << p.first << "] - off)";
    }
    if (first) os << "0.0";
    os << ";\n    const double sm = ";
    first = true;
    for (auto& p : nu) {
      if (!first) os << " + ";
      first = false;
      os << num(static_cast<double>(p.second)) << "*mu[" << 1 + p.first << "]";
    }
    if (first) os << "0.0";
    if (full_system) {
      int dnu = 0;
      for (auto& p : nu) dnu += p.second;
      os << ";\n    g[" << j << "] += q * (fma(-aC, " << num(static_cast<double>(dnu)) << ", sm) + (muT + aH) * dH);\n  }\n";
    } else {
      os << ";\n    g[" << j << "] += q * (sm + muT * dH);\n  }\n";
    }
  }
  os << "}\n";
  // ---- NASA-7 values for a generic value type (plain or dual numbers); the range is chosen by
  // the value of T
  os << "template <class R>\n__device__ __forceinline__ void mech_thermo_t(R T, R lnT, R invT, R (&cpR)[NS], R (&hRT)[NS],"
        " R (&gRT)[NS], R (&dcpR)[NS]) {\n";
  for (auto& g : groups) {
    os << "  {\n    const bool hi = chem_val(T) >= " << num(g.first) << ";\n";
    for (int i : g.second) {
      const Species& sp = m.species[i];
      const std::string I = std::to_string(i);
      auto a = [&](int k) { return std::string("(hi ? ") + num(sp.hi[k]) + " : " + num(sp.lo[k]) + ")"; };
      os << "    { // " << sp.name << "\n";
      if (sp.poly) {
        os << "      cpR[" << I << "] = " << poly_cp(sp) << ";\n";
        os << "      hRT[" << I << "] = " << poly_h(sp) << ";\n";
        os << "      gRT[" << I << "] = hRT[" << I << "] - (" << poly_s(sp) << ");\n";
        os << "      dcpR[" << I << "] = " << poly_dcp(sp) << ";\n    }\n";
        continue;
      }
      os << "      cpR[" << I << "] = " << a(0) << " + T*(" << a(1) << " + T*(" << a(2) << " + T*(" << a(3) << " + T*"
         << a(4) << ")));\n";
      os << "      hRT[" << I << "] = " << a(0) << " + T*(0.5*" << a(1) << " + T*((1.0/3.0)*" << a(2) << " + T*(0.25*"
         << a(3) << " + T*(0.2*" << a(4) << ")))) + " << a(5) << "*invT;\n";
      os << "      gRT[" << I << "] = hRT[" << I << "] - (" << a(0) << "*lnT + T*(" << a(1) << " + T*(0.5*" << a(2)
         << " + T*((1.0/3.0)*" << a(3) << " + T*(0.25*" << a(4) << ")))) + " << a(6) << ");\n";
      os << "      dcpR[" << I << "] = " << a(1) << " + T*(2.0*" << a(2) << " + T*(3.0*" << a(3) << " + T*(4.0*" << a(4)
         << ")));\n    }\n";
    }
    os << "  }\n";
  }
  os << "}\n";
  // ---- vector-Jacobian product for the Rosenbrock adjoint, without forming J:
  //   v = J(y)^T u,  g_j += q_j(y) (u^T dS/dlnA_j(y)) / q_j = q_j sig_j
  // With ut_s = u_{1+s} - u_0 T hw_s / D (the T row folded into the species weights, omega_T =
  // -T N / D), (J^T u)_k = sum_j sig_j dq_j/dy_k + [k >= 1] sum_s ut_s tbr_s + u_0 x (the T row's
  // own terms: -s1/D + A s3 for k = 0, A cw_{k-1} otherwise), sig_j = sum_s nu_sj ut_s.  For
  // dual-number states y + eps d the dual parts are the directional derivatives along d.
  os << "template <class R, class GACC>\n"
        "__device__ CHEM_ADJ_CALL void mech_vjp(const R (&y)[NY], const double* __restrict__ lnA, int energy,"
        " const double (&u)[NY], R (&v)[NY], GACC& g, int gmode) {\n";
  os << "  const R T = y[0];\n  const R lnT = log(T);\n  const R invT = 1.0 / T;\n";
  os << "  R C[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) C[i] = y[1 + i];\n";
  os << "  R cpR[NS], hRT[NS], gRT[NS], dcpR[NS];\n  mech_thermo_t(T, lnT, invT, cpR, hRT, gRT, dcpR);\n";
  if (any_pd) os << "  R Mc = 0.0;\n#pragma unroll\n  for (int i = 0; i < NS; ++i) Mc += C[i];\n";
  os << "  const double off = energy == 1 ? 1.0 : 0.0;\n  R D = 0.0;\n"
        "#pragma unroll\n  for (int i = 0; i < NS; ++i) D += C[i] * (cpR[i] - off);\n";
  os << "  const R invD = 1.0 / D;\n  const R uT = -u[0] * T * invD;\n";
  os << "  R ut[NS], w[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) {\n    ut[i] = u[1 + i] + uT * (hRT[i] - off);\n"
        "    w[i] = 0.0;\n  }\n";
  os << "#pragma unroll\n  for (int k = 0; k < NY; ++k) v[k] = 0.0;\n  R tbs = 0.0;\n";
  for (int j = 0; j < nr; ++j) {
    emit_rate(os, m, j, false, red, true);
    os << "  }\n";
  }
  os << "  R N = 0.0, s1 = 0.0, s3 = 0.0;\n#pragma unroll\n  for (int i = 0; i < NS; ++i) {\n"
        "    N += (hRT[i] - off) * w[i];\n    s1 += (cpR[i] - off) * w[i];\n    s3 += C[i] * dcpR[i];\n  }\n";
  os << "  const R A = T * N * invD * invD;\n  v[0] += u[0] * (A * s3 - s1 * invD);\n";
  os << "#pragma unroll\n  for (int k = 0; k < NS; ++k) v[1 + k] += tbs + u[0] * (A * (cpR[k] - off));\n}\n";
  os << kKernels;
  return os.str();
}

}  // namespace chem
