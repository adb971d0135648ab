// Mechanism file parsing and validation (Cantera-like JSON; Section 4.3 of the paper describes
// the same inputs: species thermo, stoichiometry, rate coefficients in SI units).
#include "mechanism.hpp"

#include <algorithm>
#include <cmath>
#include <stdexcept>

#include "json.hpp"

namespace chem {

std::map<int, int> Mechanism::net(int j) const {
  std::map<int, int> out;
  for (auto& p : reactions[j].reactants) out[p.first] -= p.second;
  for (auto& p : reactions[j].products) out[p.first] += p.second;
  for (auto it = out.begin(); it != out.end();) {
    if (it->second == 0)
      it = out.erase(it);
    else
      ++it;
  }
  return out;
}

static Arrhenius read_arrhenius(const chemjson::Value& v) {
  Arrhenius a;
  double A = v["A"].number();
  if (!(A > 0.0) || !std::isfinite(A)) throw std::runtime_error("Arrhenius prefactor A must be positive");
  a.lnA = std::log(A);
  a.b = v["b"].number();
  a.theta = v["Ea"].number() / kR;
  return a;
}

static std::vector<std::pair<int, int>> read_side(const chemjson::Value& v, const std::map<std::string, int>& idx) {
  std::vector<std::pair<int, int>> out;
  for (auto& kv : v.obj) {
    auto it = idx.find(kv.first);
    if (it == idx.end()) throw std::runtime_error("unknown species '" + kv.first + "' in reaction");
    double c = kv.second.number();
    if (c != std::floor(c) || c < 1 || c > 8)
      throw std::runtime_error("stoichiometric coefficients must be integers in [1, 8]");
    out.emplace_back(it->second, static_cast<int>(c));
  }
  if (out.empty()) throw std::runtime_error("empty reaction side");
  return out;
}

Mechanism parse_mechanism(const std::string& text) {
  chemjson::Value doc = chemjson::parse(text);
  Mechanism m;
  if (doc.has("reference-pressure")) m.p_ref = doc["reference-pressure"].number();
  if (doc.has("elements"))
    for (auto& e : doc["elements"].arr) m.elements.push_back(e["symbol"].string());
  std::map<std::string, int> idx;
  for (auto& s : doc["species"].arr) {
    Species sp;
    sp.name = s["name"].string();
    sp.W = s["molecular-weight"].number();
    if (!(sp.W > 0.0)) throw std::runtime_error("species '" + sp.name + "' has a non-positive molecular weight");
    if (s.has("inert") && s["inert"].kind == chemjson::Value::Bool) sp.inert = s["inert"].b;
    const auto& th = s["thermo"];
    const std::string model = th["model"].string();
    if (model == "polynomial-cp") {
      // single-range cp/R polynomial of degree n_p (Section 2.1) with its integration constants
      sp.poly = true;
      for (auto& v : th["cp-R"].arr) sp.cp.push_back(v.number());
      if (sp.cp.empty() || sp.cp.size() > 32) throw std::runtime_error("cp-R must hold 1 to 32 coefficients");
      sp.h0 = th["h0"].number();
      sp.s0 = th["s0"].number();
    } else if (model == "NASA7") {
      sp.T_mid = th["temperature-ranges"][1].number();
      const auto& data = th["data"];
      if (data.size() != 2 || data[0].size() != 7 || data[1].size() != 7)
        throw std::runtime_error("NASA7 data must be two lists of 7 coefficients");
      for (int k = 0; k < 7; ++k) {
        sp.lo[k] = data[0][k].number();
        sp.hi[k] = data[1][k].number();
      }
    } else {
      throw std::runtime_error("unsupported thermo model '" + model + "' (NASA7 or polynomial-cp)");
    }
    if (idx.count(sp.name)) throw std::runtime_error("duplicate species '" + sp.name + "'");
    idx[sp.name] = m.ns();
    m.species.push_back(sp);
  }
  if (m.species.empty()) throw std::runtime_error("mechanism has no species");
  for (auto& r : doc["reactions"].arr) {
    Reaction rx;
    std::string type = r["type"].string();
    if (type == "elementary")
      rx.kind = RxKind::Elementary;
    else if (type == "three-body")
      rx.kind = RxKind::ThirdBody;
    else if (type == "falloff")
      rx.kind = RxKind::Falloff;
    else if (type == "pressure-dependent-Arrhenius")
      rx.kind = RxKind::Plog;
    else
      throw std::runtime_error("unsupported reaction type '" + type + "'");
    if (r.has("equation")) rx.equation = r["equation"].string();
    rx.reversible = !r.has("reversible") || r["reversible"].b;
    rx.reactants = read_side(r["reactants"], idx);
    rx.products = read_side(r["products"], idx);
    if (rx.kind == RxKind::Falloff) {
      rx.k = read_arrhenius(r["high-P-rate-constant"]);
      rx.k0 = read_arrhenius(r["low-P-rate-constant"]);
      if (r.has("Troe")) {
        const auto& t = r["Troe"];
        rx.troe = true;
        rx.troe_alpha = t["A"].number();
        rx.troe_T3 = t["T3"].number();
        rx.troe_T1 = t["T1"].number();
        rx.troe_has_T2 = t.has("T2");
        if (rx.troe_has_T2) rx.troe_T2 = t["T2"].number();
        if (!(rx.troe_T3 > 0.0) || !(rx.troe_T1 > 0.0)) throw std::runtime_error("Troe T3 and T1 must be positive");
      } else if (r.has("SRI")) {
        const auto& t = r["SRI"];
        rx.sri = true;
        rx.sri_a = t["A"].number();
        rx.sri_b = t["B"].number();
        rx.sri_c = t["C"].number();
        rx.sri_d = t.has("D") ? t["D"].number() : 1.0;
        rx.sri_e = t.has("E") ? t["E"].number() : 0.0;
        if (!(rx.sri_c > 0.0) || !(rx.sri_d > 0.0)) throw std::runtime_error("SRI C and D must be positive");
      }
    } else if (rx.kind == RxKind::Plog) {
      for (auto& e : r["rate-constants"].arr) {
        const double P = e["P"].number();
        if (!(P > 0.0) || !std::isfinite(P)) throw std::runtime_error("P-log pressures must be positive");
        rx.plog.emplace_back(std::log(P), read_arrhenius(e));
      }
      if (rx.plog.empty()) throw std::runtime_error("P-log reaction without rate constants");
      std::sort(rx.plog.begin(), rx.plog.end(),
                [](const std::pair<double, Arrhenius>& x, const std::pair<double, Arrhenius>& y) { return x.first < y.first; });
      for (size_t i = 1; i < rx.plog.size(); ++i)
        if (!(rx.plog[i].first > rx.plog[i - 1].first)) throw std::runtime_error("P-log pressures must be distinct");
      rx.k = rx.plog.front().second;
    } else {
      rx.k = read_arrhenius(r["rate-constant"]);
    }
    if (rx.kind == RxKind::Plog) {
      rx.default_eff = 1.0;   // p = R T sum_i C_i: the rate depends on every concentration once
    } else if (rx.kind != RxKind::Elementary) {
      if (r.has("default-efficiency")) rx.default_eff = r["default-efficiency"].number();
      if (r.has("efficiencies")) {
        for (auto& kv : r["efficiencies"].obj) {
          auto it = idx.find(kv.first);
          if (it == idx.end()) throw std::runtime_error("unknown species '" + kv.first + "' in efficiencies");
          double a = kv.second.number();
          if (a != rx.default_eff) rx.eff.emplace_back(it->second, a);
        }
      }
    }
    m.reactions.push_back(rx);
  }
  return m;
}

}  // namespace chem
