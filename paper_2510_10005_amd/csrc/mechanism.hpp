// Host-side mechanism model: what the code generator needs to emit a mechanism's kernels.
#pragma once

#include <map>
#include <string>
#include <vector>

namespace chem {

constexpr double kR = 8314.462618;  // J/(kmol K)

enum class RxKind { Elementary, ThirdBody, Falloff, Plog };

struct Arrhenius {
  double lnA = 0.0;   // ln of the prefactor (SI-kmol)
  double b = 0.0;
  double theta = 0.0; // Ea / R [K]
};

struct Reaction {
  RxKind kind = RxKind::Elementary;
  bool reversible = true;
  std::vector<std::pair<int, int>> reactants;  // (species, integer coefficient nu^f)
  std::vector<std::pair<int, int>> products;   // (species, integer coefficient nu^r)
  Arrhenius k;        // elementary/third-body rate, or the high-pressure limit of a falloff
  Arrhenius k0;       // falloff low-pressure limit
  bool troe = false;
  double troe_alpha = 0.0, troe_T3 = 0.0, troe_T1 = 0.0, troe_T2 = 0.0;
  bool troe_has_T2 = false;
  std::vector<std::pair<double, Arrhenius>> plog;  // P-log: (ln p_i, rate) sorted by pressure; k = the first
  bool sri = false;   // SRI broadening F = d [a exp(-b/T) + exp(-T/c)]^X T^e
  double sri_a = 0.0, sri_b = 0.0, sri_c = 1.0, sri_d = 1.0, sri_e = 0.0;
  double default_eff = 1.0;
  std::vector<std::pair<int, double>> eff;      // species with alpha != default
  std::string equation;
};

struct Species {
  std::string name;
  double W = 0.0;                  // kg/kmol
  double T_mid = 1000.0;
  double lo[7] = {0}, hi[7] = {0};  // NASA-7 coefficients
  bool poly = false;                // single-range cp/R = sum_k cp[k] T^k with integration constants
  std::vector<double> cp;           // h0 (h/RT = (h0 + sum cp_k T^(k+1)/(k+1)) / T) and s0
  double h0 = 0.0, s0 = 0.0;
  bool inert = false;
};

struct Mechanism {
  std::vector<Species> species;
  std::vector<Reaction> reactions;
  std::vector<std::string> elements;
  double p_ref = 101325.0;
  int ns() const { return static_cast<int>(species.size()); }
  int nr() const { return static_cast<int>(reactions.size()); }
  int n() const { return ns() + 1; }
  // net stoichiometric coefficient nu_ij = nu^r - nu^f
  std::map<int, int> net(int j) const;
};

// Parse and validate; throws std::runtime_error with a readable message on failure.
Mechanism parse_mechanism(const std::string& json_text);

// Generated HIP source for the mechanism (everything the kernels need, constants folded).
// dense_limit: state sizes up to this use register-resident Jacobian/LU storage.
// full_system (register-resident mechanisms only): every species in the integrators' solved system
std::string generate_source(const Mechanism& m, int dense_limit, bool full_system = false);

}  // namespace chem
