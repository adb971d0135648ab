// Per-mechanism HIP source generation: the code-generation step of the paper (Section 4.3),
// re-targeted to gfx950.  Like ChemGen, every reaction becomes straight-line code with its
// constants folded (A, b, Ea/R, stoichiometry, efficiencies, Troe parameters), the integer
// powers of concentrations and of (p_ref/RT) are unrolled into products or a single ln term,
// efficiencies equal to the default are dropped (eq. TB_optimization), and the analytic Jacobian
// is emitted from the chain rules of each rate form (Section 4.2) with only the entries the
// reaction touches.  Unlike ChemGen, ln A stays a runtime array (it is a differentiable
// parameter), and the emitted code is device code for one cell per GPU lane.
#include <cmath>
#include <cstdio>
#include <set>
#include <sstream>
#include <string>

#include "mechanism.hpp"

namespace chem {

static const char* kPrelude =
#include "device_prelude.inc"
    ;
static const char* kKernels =
#include "device_kernels.inc"
    ;

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

static void emit_rate(std::ostringstream& os, const Mechanism& m, int j, bool jac) {
  const Reaction& r = m.reactions[j];
  const std::string J = std::to_string(j);
  os << "  { // reaction " << j << ": " << r.equation << "\n";
  // ln k = ln A + b ln T - (Ea/R) / T   (log form of the Arrhenius law, Section 2.2.1)
  os << "    const double lnk = lnA[" << J << "]";
  if (r.k.b != 0.0) os << " + " << num(r.k.b) << "*lnT";
  if (r.k.theta != 0.0) os << " - " << num(r.k.theta) << "*invT";
  os << ";\n";
  const bool pd = r.kind != RxKind::Elementary;
  if (pd) {
    // [M] = default * M_c + sum over listed species of (alpha - default) C_i
    os << "    const double M = ";
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
    os << "    const double kf = exp(lnk);\n";
  } else if (r.kind == RxKind::ThirdBody) {
    os << "    const double kf = M*exp(lnk);\n";
  } else {
    const double db = r.k0.b - r.k.b, dth = r.k0.theta - r.k.theta, dlnA = r.k0.lnA - r.k.lnA;
    os << "    double kf, dlnkf_dT_fo, dlnkf_dM_fo;\n";
    os << "    chem_falloff<" << (jac ? "JAC" : "false") << ", " << (r.troe ? "true" : "false") << ", "
       << (r.troe && r.troe_has_T2 ? "true" : "false") << ">(lnk, " << num(dlnA) << " + " << num(db) << "*lnT - "
       << num(dth) << "*invT, M, T, invT, " << num(r.k.b) << ", " << num(r.k.theta) << ", " << num(db) << ", "
       << num(dth) << ", " << num(r.troe ? r.troe_alpha : 0.0) << ", " << num(r.troe ? 1.0 / r.troe_T3 : 0.0) << ", "
       << num(r.troe ? 1.0 / r.troe_T1 : 0.0) << ", " << num(r.troe && r.troe_has_T2 ? r.troe_T2 : 0.0)
       << ", kf, dlnkf_dT_fo, dlnkf_dM_fo);\n";
  }
  auto nu = m.net(j);
  int dnu = 0;
  for (auto& p : nu) dnu += p.second;
  os << "    const double Rf = kf*" << conc_product(r.reactants) << ";\n";
  if (r.reversible) {
    // ln K = -sum nu g/RT + (sum nu) ln(p_ref/(R T))   (eq. equilibrium-constant)
    os << "    const double lnKc = -(";
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
    os << "    const double kr = kf*exp(-lnKc);\n";
    os << "    const double Rr = kr*" << conc_product(r.products) << ";\n";
  } else {
    os << "    const double Rr = 0.0;\n";
  }
  os << "    const double q = Rf - Rr;\n";
  if (!jac) return;  // caller closes the block
  for (auto& p : nu) {
    if (p.second == 1)
      os << "    w[" << p.first << "] += q;\n";
    else if (p.second == -1)
      os << "    w[" << p.first << "] -= q;\n";
    else
      os << "    w[" << p.first << "] = fma(" << num(static_cast<double>(p.second)) << ", q, w[" << p.first << "]);\n";
  }
  os << "    if (JAC) {\n";
  if (r.kind == RxKind::Falloff) {
    os << "      const double dlnkf_dT = dlnkf_dT_fo;\n";
  } else {
    os << "      const double dlnkf_dT = (" << num(r.k.b) << " + " << num(r.k.theta) << "*invT)*invT;\n";
  }
  if (r.reversible) {
    os << "      const double dlnKc_dT = (";
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
    os << "      const double dqdT = q*dlnkf_dT + Rr*dlnKc_dT;\n";
  } else {
    os << "      const double dqdT = q*dlnkf_dT;\n";
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
      os << "      const double qM = q/M;\n";
    else
      os << "      const double qM = q*dlnkf_dM_fo;\n";
    for (auto& e : r.eff) {
      std::string t = "qM*" + num(e.second - r.default_eff);
      dq[e.first] = dq.count(e.first) ? dq[e.first] + " + " + t : t;
    }
    if (r.default_eff != 0.0) {
      for (auto& p : nu) {
        os << "      tbr[" << p.first << "] = fma(" << num(p.second * r.default_eff) << ", qM, tbr[" << p.first
           << "]);\n";
      }
    }
  }
  for (auto& d : dq) os << "      const double dq" << d.first << " = " << d.second << ";\n";
  for (auto& p : nu) {
    const std::string row = std::to_string(1 + p.first);
    const std::string nv = num(static_cast<double>(p.second));
    auto acc = [&](const std::string& col, const std::string& val) {
      if (p.second == 1)
        os << "      J(" << row << "," << col << ") += " << val << ";\n";
      else if (p.second == -1)
        os << "      J(" << row << "," << col << ") -= " << val << ";\n";
      else
        os << "      J(" << row << "," << col << ") = fma(" << nv << ", " << val << ", J(" << row << "," << col << "));\n";
    };
    acc("0", "dqdT");
    for (auto& d : dq) acc(std::to_string(1 + d.first), "dq" + std::to_string(d.first));
  }
  os << "    }\n";
}

std::string generate_source(const Mechanism& m, int dense_limit) {
  std::ostringstream os;
  const int ns = m.ns(), nr = m.nr(), n = m.n();
  os << kPrelude;
  os << "// ---------------------------------------------------------------- generated mechanism block\n";
  os << "#define NS " << ns << "\n#define NY " << n << "\n#define NR " << (nr > 0 ? nr : 1) << "\n";
  os << "#define CHEM_DENSE " << (n <= dense_limit ? 1 : 0) << "\n";
  os << "#if CHEM_DENSE\n#define CHEM_MUNROLL _Pragma(\"unroll\")\n#define CHEM_EVAL_INLINE __forceinline__\n"
        "#else\n#define CHEM_MUNROLL _Pragma(\"unroll 1\")\n#define CHEM_EVAL_INLINE __noinline__\n#endif\n";
  os << "#define CHEM_R 8314.462618\n";
  os << "#define LNPREF_R " << num(std::log(m.p_ref / kR)) << "\n";
  os << "static __device__ const double mech_W[NS] = {";
  for (int i = 0; i < ns; ++i) os << (i ? ", " : "") << num(m.species[i].W);
  os << "};\n";
  os << "static __device__ const double mech_RW[NS] = {";
  for (int i = 0; i < ns; ++i) os << (i ? ", " : "") << num(kR / m.species[i].W);
  os << "};\n";

  // ---- thermo: NASA-7 in Horner form with the range chosen per T_mid (Table 1, n_p = 4)
  std::set<double> tmids;
  for (auto& s : m.species) tmids.insert(s.T_mid);
  os << "__device__ __forceinline__ void mech_thermo(double T, double lnT, double invT, double (&cpR)[NS], "
        "double (&hRT)[NS], double (&sR)[NS], double (&gRT)[NS], double (&dcpR)[NS]) {\n";
  int ti = 0;
  std::map<double, int> tidx;
  for (double t : tmids) {
    os << "  const bool hi" << ti << " = T >= " << num(t) << ";\n";
    tidx[t] = ti++;
  }
  for (int i = 0; i < ns; ++i) {
    const Species& s = m.species[i];
    const std::string h = "hi" + std::to_string(tidx[s.T_mid]);
    os << "  { // " << s.name << "\n";
    for (int k = 0; k < 7; ++k)
      os << "    const double a" << k << " = " << h << " ? " << num(s.hi[k]) << " : " << num(s.lo[k]) << ";\n";
    os << "    cpR[" << i << "] = a0 + T*(a1 + T*(a2 + T*(a3 + T*a4)));\n";
    os << "    hRT[" << i << "] = a0 + T*(a1*0.5 + T*(a2*(1.0/3.0) + T*(a3*0.25 + T*(a4*0.2)))) + a5*invT;\n";
    os << "    sR[" << i << "] = a0*lnT + T*(a1 + T*(a2*0.5 + T*(a3*(1.0/3.0) + T*(a4*0.25)))) + a6;\n";
    os << "    gRT[" << i << "] = hRT[" << i << "] - sR[" << i << "];\n";
    os << "    dcpR[" << i << "] = a1 + T*(2.0*a2 + T*(3.0*a3 + T*(4.0*a4)));\n";
    os << "  }\n";
  }
  os << "}\n";

  bool any_pd = false;
  for (auto& r : m.reactions) any_pd = any_pd || r.kind != RxKind::Elementary;

  // ---- source terms and Jacobian
  os << "template <bool JAC, class MAT>\n"
        "__device__ CHEM_EVAL_INLINE void mech_eval(const double (&y)[NY], const double* __restrict__ lnA, int energy,"
        " double (&S)[NY], MAT& J) {\n";
  os << "  const double T = y[0];\n  const double lnT = log(T);\n  const double invT = 1.0 / T;\n";
  os << "  double C[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) C[i] = y[1 + i];\n";
  os << "  double cpR[NS], hRT[NS], sR[NS], gRT[NS], dcpR[NS];\n";
  os << "  mech_thermo(T, lnT, invT, cpR, hRT, sR, gRT, dcpR);\n";
  if (any_pd) os << "  double Mc = 0.0;\n#pragma unroll\n  for (int i = 0; i < NS; ++i) Mc += C[i];\n";
  os << "  double w[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) w[i] = 0.0;\n";
  if (any_pd) os << "  double tbr[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) tbr[i] = 0.0;\n";
  os << "  if (JAC) {\n    CHEM_MUNROLL\n    for (int i = 0; i < NY; ++i) {\n      CHEM_MUNROLL\n"
        "      for (int k = 0; k < NY; ++k) J(i, k) = 0.0;\n    }\n  }\n";
  for (int j = 0; j < nr; ++j) {
    emit_rate(os, m, j, true);
    os << "  }\n";
  }
  os << "  const double off = energy ? 1.0 : 0.0;\n";
  os << "  double hw[NS], cw[NS], N = 0.0, D = 0.0;\n";
  os << "#pragma unroll\n  for (int i = 0; i < NS; ++i) {\n    hw[i] = hRT[i] - off;\n    cw[i] = cpR[i] - off;\n"
        "    N = fma(hw[i], w[i], N);\n    D = fma(C[i], cw[i], D);\n  }\n";
  os << "  S[0] = -T * N / D;\n#pragma unroll\n  for (int i = 0; i < NS; ++i) S[1 + i] = w[i];\n";
  os << "  if (JAC) {\n";
  if (any_pd) {
    os << "    CHEM_MUNROLL\n    for (int i = 0; i < NS; ++i) {\n      CHEM_MUNROLL\n"
          "      for (int k = 0; k < NS; ++k) J(1 + i, 1 + k) += tbr[i];\n    }\n";
  }
  os << "    const double A = T * N / (D * D);\n";
  os << "    double s1 = 0.0, s2 = 0.0, s3 = 0.0;\n";
  os << "#pragma unroll\n    for (int i = 0; i < NS; ++i) {\n      s1 = fma(cw[i], w[i], s1);\n"
        "      s2 = fma(hw[i], J(1 + i, 0), s2);\n      s3 = fma(C[i], dcpR[i], s3);\n    }\n";
  os << "    J(0, 0) = -(s1 + T * s2) / D + A * s3;\n";
  os << "    CHEM_MUNROLL\n    for (int k = 0; k < NS; ++k) {\n      double t = 0.0;\n      CHEM_MUNROLL\n"
        "      for (int i = 0; i < NS; ++i) t = fma(hw[i], J(1 + i, 1 + k), t);\n"
        "      J(0, 1 + k) = -T * t / D + A * cw[k];\n    }\n";
  os << "  }\n}\n";

  // ---- d/d lnA contraction for the adjoint: g_j += q_j (sum_i nu_ij mu_i - mu_T T sum_i nu_ij hw_i / D)
  os << "template <class GACC>\n"
        "__device__ CHEM_EVAL_INLINE void mech_grad(const double (&y)[NY], const double* __restrict__ lnA, int energy,"
        " const double (&mu)[NY], GACC& g) {\n";
  os << "  const double T = y[0];\n  const double lnT = log(T);\n  const double invT = 1.0 / T;\n";
  os << "  double C[NS];\n#pragma unroll\n  for (int i = 0; i < NS; ++i) C[i] = y[1 + i];\n";
  os << "  double cpR[NS], hRT[NS], sR[NS], gRT[NS], dcpR[NS];\n";
  os << "  mech_thermo(T, lnT, invT, cpR, hRT, sR, gRT, dcpR);\n";
  if (any_pd) os << "  double Mc = 0.0;\n#pragma unroll\n  for (int i = 0; i < NS; ++i) Mc += C[i];\n";
  os << "  const double off = energy ? 1.0 : 0.0;\n  double D = 0.0;\n"
        "#pragma unroll\n  for (int i = 0; i < NS; ++i) D = fma(C[i], cpR[i] - off, D);\n";
  os << "  const double muT = -T * mu[0] / D;\n";
  for (int j = 0; j < nr; ++j) {
    emit_rate(os, m, j, false);
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
    os << ";\n    g[" << j << "] += q * (sm + muT * dH);\n  }\n";
  }
  os << "}\n";
  os << kKernels;
  return os.str();
}

}  // namespace chem
