"""Seeded synthetic reaction mechanisms in a Cantera-like JSON layout.

The paper's workloads use real mechanisms (H2 sub-models, GRI-3.0-sized,
FFCM-2-sized; Section 5, Table 3).  None is available here and none is
reproduced; instead this module draws mechanisms of the same size and
structure from a fixed seed:

* species are random formulas over a given element set (at most
  ``max_atoms`` atoms), plus reference diatomics and an inert collider;
* thermo data are NASA-7 two-range polynomials (split at 1000 K, fitted on
  [300, 1000] and [1000, 5000] K so that extrapolation up to 6000 K stays
  sane during heat release) fitted by least squares to a smooth heat-capacity model (translation + rotation +
  Einstein vibrational modes), with formation enthalpies from a simple
  bond-energy model and standard entropies growing with atom count;
* reactions are element-balanced, reversible, with at most three species
  per side, written in their exothermic direction (by the generator's own
  formation-enthalpy table); a chosen number are third-body and Troe
  falloff reactions of the form A + B (+M) <=> AB (+M);
* rate parameters are drawn as ln A ~ U[20, 35], b ~ U[-1.5, 2],
  Ea/R ~ U[0, 25000] K, with ln A read in (cm, mol, s) units at a 1000 K
  reference for the T^b factor and stored converted to SI-kmol (taken
  literally in SI-kmol with T in K, the draws are up to ~1e10 times faster
  than gas-kinetic collision rates); falloff low-pressure limits are
  independent draws of the same distributions; third-body efficiencies
  are U[0.5, 5] on three random species; Troe alpha ~ U[0.4, 0.9] and
  T***, T*, T** ~ log-U[50, 1e4] K.

The stoichiometric matrix is required to have full rank modulo the linear
invariants (element totals and inert species), so that element totals
are the only conserved linear combinations.

Nothing here evaluates rates, source terms or integrators.  The only
thermodynamic arithmetic is the construction of the NASA-7 data
themselves (least-squares fit of cp/R and the two integration constants
that pin h and s at 298.15 K and make them continuous at 1000 K).
"""

from __future__ import annotations

import itertools
import json
import math
from dataclasses import dataclass, field

import numpy as np

R_UNIVERSAL = 8314.462618  # J/(kmol K); the file stores Ea in J/kmol

ATOMIC_WEIGHT = {"H": 1.008, "C": 12.011, "N": 14.007, "O": 15.999, "Ar": 39.948}
# gas-phase atom formation enthalpies at 298 K [kJ/mol] (the bond model's anchor)
ATOM_ENTHALPY = {"H": 218.0, "O": 249.2, "N": 472.7, "C": 716.7, "Ar": 0.0}
REFERENCE_DIATOMICS = {"H2": {"H": 2}, "O2": {"O": 2}, "N2": {"N": 2}}

T_LOW, T_MID, T_HIGH = 300.0, 1000.0, 5000.0
T_298 = 298.15


@dataclass(frozen=True)
class MechConfig:
    name: str
    seed: int
    elements: tuple
    n_species: int
    n_reactions: int
    n_third_body: int
    n_falloff: int
    max_atoms: int
    inert: tuple          # inert collider species (appear in no reaction)
    reference: tuple      # reference diatomics forced into the species list
    isomers: bool = False
    broadening: str = "troe"   # falloff broadening: "troe" or "sri"
    n_plog: int = 0            # elementary reactions rewritten as P-log tables (the first ones drawn)


MECH_CONFIGS = {
    # 10 species from {H, O, N} with <= 4 atoms, N2-like inert; 27 reactions, 4 third-body
    "h2like_10_27": MechConfig("h2like_10_27", 1000, ("H", "O", "N"), 10, 27, 4, 0, 4,
                               ("N2",), ("H2", "O2")),
    # 53 species from {C, H, O, N, Ar}; 325 reactions: 29 Troe falloff, 40 third-body
    "ch4like_53_325": MechConfig("ch4like_53_325", 1002, ("C", "H", "O", "N", "Ar"), 53, 325, 40, 29, 6,
                                 ("Ar",), ("H2", "O2", "N2"), isomers=True),
    # 150 species, 1000 reactions: 60 Troe falloff, 120 third-body
    "large_150_1000": MechConfig("large_150_1000", 1004, ("C", "H", "O", "N", "Ar"), 150, 1000, 120, 60, 10,
                                 ("Ar",), ("H2", "O2", "N2"), isomers=True),
    # tiny mechanisms for unit tests
    "tiny_5_6": MechConfig("tiny_5_6", 1010, ("H", "O"), 5, 6, 1, 1, 3, (), ("H2", "O2")),
    "tiny_8_14": MechConfig("tiny_8_14", 1011, ("H", "O", "N"), 8, 14, 2, 2, 4, ("N2",), ("H2", "O2")),
    # 12 species from {H, O, N}; 30 reactions: 6 falloff with SRI broadening, 4 third-body
    "sri_12_30": MechConfig("sri_12_30", 1012, ("H", "O", "N"), 12, 30, 4, 6, 4, ("N2",), ("H2", "O2"),
                            broadening="sri"),
    # 12 species from {H, O, N}; 30 reactions: 8 P-log (3 pressures), 4 third-body, 2 Troe falloff
    "plog_12_30": MechConfig("plog_12_30", 1013, ("H", "O", "N"), 12, 30, 4, 2, 4, ("N2",), ("H2", "O2"),
                             n_plog=8),
    # 30 species from {C, H, O, N} (the one-wavefront-per-cell form, n = 31); 90 reactions: 10 P-log,
    # 6 falloff with SRI broadening, 8 third-body
    "mix_30_90": MechConfig("mix_30_90", 1014, ("C", "H", "O", "N"), 30, 90, 8, 6, 5, ("N2",), ("H2", "O2"),
                            broadening="sri", n_plog=10),
    # 14 species from {C, H, O, N}, N2-like inert (13 active: the Rosenbrock kernels' packed upper
    # factor needs 91 doubles per lane of LDS); 40 reactions: 4 third-body, 3 Troe falloff
    "mid_14_40": MechConfig("mid_14_40", 1015, ("C", "H", "O", "N"), 14, 40, 4, 3, 5, ("N2",), ("H2", "O2"),
                            isomers=True),
}

PLOG_PRESSURES = (1.0e4, 1.0e5, 1.0e6)   # Pa: the table straddles the workloads' ~1 atm


# --------------------------------------------------------------------------- species

def _formula_name(comp):
    order = ["C", "H", "O", "N", "Ar"]
    s = ""
    for el in order:
        c = comp.get(el, 0)
        if c == 1:
            s += el
        elif c > 1:
            s += f"{el}{c}"
    return s


def _all_formulas(elements, max_atoms):
    els = [e for e in elements if e != "Ar"]
    out = []
    for counts in itertools.product(range(max_atoms + 1), repeat=len(els)):
        tot = sum(counts)
        if 1 <= tot <= max_atoms:
            out.append({e: c for e, c in zip(els, counts) if c > 0})
    return out


def _heat_capacity_model(rng, n_atoms, linear):
    """Return (rot, thetas): cp/R(T) = 2.5 + rot + sum_m E(theta_m / T)."""
    if n_atoms == 1:
        return 0.0, np.zeros(0)
    rot = 1.0 if linear else 1.5
    n_modes = 3 * n_atoms - (5 if linear else 6)
    thetas = np.exp(rng.uniform(math.log(500.0), math.log(5000.0), size=n_modes))
    return rot, thetas


def _cp_model(T, rot, thetas):
    T = np.asarray(T, dtype=float)
    cp = 2.5 + rot + np.zeros_like(T)
    for th in thetas:
        x = th / T
        ex = np.exp(-x)  # x^2 e^x/(e^x-1)^2 == x^2 e^-x/(1-e^-x)^2
        cp = cp + x * x * ex / (1.0 - ex) ** 2
    return cp


def _fit_nasa7(rot, thetas, dh_f_kJmol, s298_JmolK):
    """Least-squares NASA-7 fit of cp/R on [300,1000] and [1000,5000] with cp continuous at 1000 K.

    Returns (low[7], high[7]) coefficient lists.
    """
    tl = np.linspace(T_LOW, T_MID, 71)
    th = np.linspace(T_MID, T_HIGH, 201)
    fl = _cp_model(tl, rot, thetas)
    fh = _cp_model(th, rot, thetas)
    # fit in tau = T/1000 for conditioning
    Al = np.vander(tl / 1000.0, 5, increasing=True)
    Ah = np.vander(th / 1000.0, 5, increasing=True)
    m = np.ones(5)  # tau = 1 at T_mid
    K = np.zeros((11, 11))
    K[:5, :5] = 2 * Al.T @ Al
    K[5:10, 5:10] = 2 * Ah.T @ Ah
    K[10, :5] = m
    K[10, 5:10] = -m
    K[:5, 10] = m
    K[5:10, 10] = -m
    rhs = np.concatenate([2 * Al.T @ fl, 2 * Ah.T @ fh, [0.0]])
    sol = np.linalg.solve(K, rhs)
    scale = 1000.0 ** np.arange(5)
    lo = sol[:5] / scale
    hi = sol[5:10] / scale

    def h_poly(a, T):  # H/R without the constant
        return a[0] * T + a[1] * T**2 / 2 + a[2] * T**3 / 3 + a[3] * T**4 / 4 + a[4] * T**5 / 5

    def s_poly(a, T):  # S/R without the constant
        return a[0] * math.log(T) + a[1] * T + a[2] * T**2 / 2 + a[3] * T**3 / 3 + a[4] * T**4 / 4

    H298_R = dh_f_kJmol * 1.0e6 / R_UNIVERSAL
    S298_R = s298_JmolK * 1.0e3 / R_UNIVERSAL
    a6_lo = H298_R - h_poly(lo, T_298)
    a7_lo = S298_R - s_poly(lo, T_298)
    a6_hi = a6_lo + h_poly(lo, T_MID) - h_poly(hi, T_MID)
    a7_hi = a7_lo + s_poly(lo, T_MID) - s_poly(hi, T_MID)
    low = [float(v) for v in lo] + [float(a6_lo), float(a7_lo)]
    high = [float(v) for v in hi] + [float(a6_hi), float(a7_hi)]
    return low, high


def _cp_poly_ok(low, high, rot, thetas):
    """Reject fits that misbehave when extrapolated (cp must stay near the model on [200, 6000] K)."""
    for a, grid in ((low, np.linspace(200.0, T_MID, 60)), (high, np.linspace(T_MID, 6000.0, 200))):
        cp = sum(a[k] * grid**k for k in range(5))
        model = _cp_model(grid, rot, thetas)
        if np.any(cp < 0.5 * model) or np.any(cp > 2.0 * model):
            return False
    return True


@dataclass
class _Species:
    name: str
    comp: dict
    n_atoms: int
    dh_f: float      # kJ/mol at 298 K
    s298: float      # J/mol/K
    low: list = field(default_factory=list)
    high: list = field(default_factory=list)
    inert: bool = False

    @property
    def weight(self):
        return sum(ATOMIC_WEIGHT[e] * c for e, c in self.comp.items())


def _make_species(rng, name, comp, reference=False, inert=False):
    n_atoms = sum(comp.values())
    linear = n_atoms <= 2 or rng.uniform() < 0.2
    if reference:
        dh = 0.0
    elif n_atoms == 1:
        el = next(iter(comp))
        dh = ATOM_ENTHALPY[el]
    else:
        atoms = sum(ATOM_ENTHALPY[e] * c for e, c in comp.items())
        dh = atoms - (n_atoms - 1) * rng.uniform(300.0, 500.0)
    s298 = (110.0 + 35.0 * (n_atoms - 1)) * rng.uniform(0.9, 1.1)
    if comp == {"Ar": 1}:
        s298 = 154.8 * rng.uniform(0.98, 1.02)
    for _ in range(200):
        rot, thetas = _heat_capacity_model(rng, n_atoms, linear)
        low, high = _fit_nasa7(rot, thetas, dh, s298)
        if _cp_poly_ok(low, high, rot, thetas):
            break
    else:  # pragma: no cover - the model is smooth; 200 draws never all fail
        raise RuntimeError(f"could not fit NASA-7 data for {name}")
    return _Species(name, dict(comp), n_atoms, float(dh), float(s298), low, high, inert)


def _draw_species(rng, cfg: MechConfig):
    species = []
    names = set()

    def add(comp, reference=False, inert=False):
        base = _formula_name(comp) if comp != {"Ar": 1} else "Ar"
        name, k = base, 1
        while name in names:
            k += 1
            name = f"{base}-{k}"
        names.add(name)
        species.append(_make_species(rng, name, comp, reference, inert))

    for nm in cfg.reference:
        add(REFERENCE_DIATOMICS[nm], reference=True)
    for nm in cfg.inert:
        comp = {"Ar": 1} if nm == "Ar" else REFERENCE_DIATOMICS[nm]
        add(comp, reference=(nm in REFERENCE_DIATOMICS), inert=True)
    formulas = _all_formulas(cfg.elements, cfg.max_atoms)
    taken = {tuple(sorted(REFERENCE_DIATOMICS[n].items())) for n in cfg.reference + cfg.inert if n != "Ar"}
    pool = [f for f in formulas if tuple(sorted(f.items())) not in taken]
    n_more = cfg.n_species - len(species)
    if cfg.isomers:
        # atoms and small radicals first (every chemistry has them), the rest drawn with replacement
        small = [f for f in pool if sum(f.values()) <= 2]
        idx = rng.permutation(len(small))[: max(0, min(len(small), n_more // 4))]
        chosen = [small[i] for i in idx]
        while len(chosen) < n_more:
            f = pool[int(rng.integers(len(pool)))]
            if sum(f.values()) == 1 and f in chosen:
                continue  # atoms have no isomers
            chosen.append(f)
    else:
        idx = rng.permutation(len(pool))[:n_more]
        chosen = [pool[i] for i in idx]
    for comp in chosen:
        add(comp)
    return species


# --------------------------------------------------------------------------- reactions

def _composition_vector(species, elements):
    return np.array([[sp.comp.get(e, 0) for e in elements] for sp in species], dtype=np.int64)


def _multisets(indices, max_size):
    out = []
    for size in range(1, max_size + 1):
        out.extend(itertools.combinations_with_replacement(indices, size))
    return out


def _stoich_dict(ms):
    d = {}
    for i in ms:
        d[i] = d.get(i, 0) + 1
    return d


def _invariant_rank(species, elements):
    E = _composition_vector(species, elements).T.astype(float)
    rows = [E]
    for i, sp in enumerate(species):
        if sp.inert:
            e = np.zeros((1, len(species)))
            e[0, i] = 1.0
            rows.append(e)
    return int(np.linalg.matrix_rank(np.vstack(rows)))


def _draw_reactions(rng, species, cfg: MechConfig):
    elements = list(cfg.elements)
    comp = _composition_vector(species, elements)
    reactive = [i for i, sp in enumerate(species) if not sp.inert]
    by_comp = {}
    for ms in _multisets(reactive, 3):
        key = tuple(comp[list(ms)].sum(axis=0))
        by_comp.setdefault(key, []).append(ms)
    ns = len(species)
    target_rank = ns - _invariant_rank(species, elements)

    chosen = []      # list of (reactants multiset, products multiset, kind)
    seen = set()

    def key_of(a, b):
        return (tuple(sorted(a)), tuple(sorted(b)))

    def try_add(a, b, kind):
        if set(a) & set(b):
            return False
        k1, k2 = key_of(a, b), key_of(b, a)
        if k1 in seen or k2 in seen:
            return False
        seen.add(k1)
        chosen.append((a, b, kind))
        return True

    def nu_matrix(rs):
        N = np.zeros((ns, len(rs)))
        for j, (a, b, _) in enumerate(rs):
            for i in a:
                N[i, j] -= 1
            for i in b:
                N[i, j] += 1
        return N

    # pressure-dependent reactions: A + B (+M) <=> AB (+M)
    pairs = []
    for ab in reactive:
        if species[ab].n_atoms < 2:
            continue
        for ms in by_comp.get(tuple(comp[ab]), []):
            if len(ms) == 2 and ab not in ms:
                pairs.append((ms, (ab,)))
    n_pd = cfg.n_third_body + cfg.n_falloff
    if len(pairs) < n_pd:
        raise RuntimeError("not enough recombination candidates")
    order = rng.permutation(len(pairs))
    kinds = ["falloff"] * cfg.n_falloff + ["three-body"] * cfg.n_third_body
    k = 0
    for idx in order:
        if k == len(kinds):
            break
        a, b = pairs[idx]
        if try_add(a, b, kinds[k]):
            k += 1

    def random_reaction():
        size = int(rng.choice([1, 2, 3], p=[0.15, 0.75, 0.10]))
        a = tuple(sorted(int(x) for x in rng.choice(reactive, size=size, replace=True)))
        cands = [b for b in by_comp.get(tuple(comp[list(a)].sum(axis=0)), []) if not (set(a) & set(b))]
        if not cands:
            return None
        return a, cands[int(rng.integers(len(cands)))]

    # elementary reactions: first grow the rank, then fill at random
    rank = np.linalg.matrix_rank(nu_matrix(chosen)) if chosen else 0
    attempts = 0
    while rank < target_rank and len(chosen) < cfg.n_reactions:
        attempts += 1
        if attempts > 20000:
            raise RuntimeError("could not reach full stoichiometric rank")
        r = random_reaction()
        if r is None:
            continue
        trial = chosen + [(r[0], r[1], "elementary")]
        new_rank = np.linalg.matrix_rank(nu_matrix(trial))
        if new_rank > rank and try_add(r[0], r[1], "elementary"):
            rank = new_rank
    attempts = 0
    while len(chosen) < cfg.n_reactions:
        attempts += 1
        if attempts > 20000:
            raise RuntimeError("not enough distinct balanced reactions")
        r = random_reaction()
        if r is not None:
            try_add(r[0], r[1], "elementary")
    if np.linalg.matrix_rank(nu_matrix(chosen)) != target_rank:
        raise RuntimeError("stoichiometric rank deficit")
    order = rng.permutation(len(chosen))
    return [chosen[i] for i in order], target_rank


T_REF_RATE = 1000.0


def _arrhenius(rng, order):
    """Draw (ln A, b, Ea/R) and return SI-kmol {A, b, Ea} for a rate of the given molecular order.

    ln A ~ U[20, 35] is read in the conventional (cm, mol, s) units in which real mechanisms
    quote prefactors, with b multiplying ln(T / 1000 K); the stored A is the equivalent
    prefactor of A T^b exp(-Ea/RT) in (m, kmol, s).
    """
    lnA_ref = rng.uniform(20.0, 35.0)
    b = rng.uniform(-1.5, 2.0)
    theta = rng.uniform(0.0, 25000.0)
    lnA = lnA_ref - b * math.log(T_REF_RATE) + (order - 1) * math.log(1.0e-3)
    return {"A": float(math.exp(lnA)), "b": float(b), "Ea": float(theta * R_UNIVERSAL)}


def generate_mechanism(name: str) -> dict:
    """Draw the mechanism ``name`` (a key of MECH_CONFIGS) and return it as a JSON-ready dict."""
    cfg = MECH_CONFIGS[name]
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    for _attempt in range(50):
        species = _draw_species(rng, cfg)
        try:
            reactions, rank = _draw_reactions(rng, species, cfg)
            break
        except RuntimeError:
            continue
    else:  # pragma: no cover
        raise RuntimeError(f"could not draw mechanism {name}")
    names = [sp.name for sp in species]
    rx_out = []
    n_plog_left = cfg.n_plog
    for a, b, kind in reactions:
        dH = sum(species[i].dh_f for i in b) - sum(species[i].dh_f for i in a)
        if dH > 0.0:  # write every reaction in its exothermic direction
            a, b = b, a
        reac = {names[i]: c for i, c in _stoich_dict(a).items()}
        prod = {names[i]: c for i, c in _stoich_dict(b).items()}

        def side(d):
            return " + ".join(f"{c} {s}" if c > 1 else s for s, c in d.items())

        rx = {"reactants": reac, "products": prod, "reversible": True}
        if kind == "elementary" and n_plog_left > 0:
            n_plog_left -= 1
            rx["type"] = "pressure-dependent-Arrhenius"
            rx["equation"] = f"{side(reac)} <=> {side(prod)}"
            base = _arrhenius(rng, sum(reac.values()))
            rx["rate-constants"] = []
            for P in PLOG_PRESSURES:
                db = float(rng.uniform(-0.3, 0.3))     # A compensated so that k(1000 K) moves by e^U[-1.5, 1.5]
                rx["rate-constants"].append(
                    {"P": P, "A": base["A"] * math.exp(float(rng.uniform(-1.5, 1.5)) - db * math.log(T_REF_RATE)),
                     "b": base["b"] + db, "Ea": base["Ea"] * float(rng.uniform(0.9, 1.1))})
        elif kind == "elementary":
            rx["type"] = "elementary"
            rx["equation"] = f"{side(reac)} <=> {side(prod)}"
            rx["rate-constant"] = _arrhenius(rng, sum(reac.values()))
        else:
            eff_idx = rng.choice(len(species), size=3, replace=False)
            eff = {names[int(i)]: float(rng.uniform(0.5, 5.0)) for i in eff_idx}
            rx["efficiencies"] = eff
            if kind == "three-body":
                rx["type"] = "three-body"
                rx["equation"] = f"{side(reac)} + M <=> {side(prod)} + M"
                rx["rate-constant"] = _arrhenius(rng, sum(reac.values()) + 1)
            else:
                rx["type"] = "falloff"
                rx["equation"] = f"{side(reac)} (+M) <=> {side(prod)} (+M)"
                rx["high-P-rate-constant"] = _arrhenius(rng, sum(reac.values()))
                rx["low-P-rate-constant"] = _arrhenius(rng, sum(reac.values()) + 1)
                lo, hi = math.log(50.0), math.log(1.0e4)
                if cfg.broadening == "sri":
                    rx["SRI"] = {"A": float(rng.uniform(0.3, 2.0)),
                                 "B": float(math.exp(rng.uniform(math.log(50.0), math.log(1.0e3)))),
                                 "C": float(math.exp(rng.uniform(math.log(200.0), math.log(3.0e3)))),
                                 "D": float(rng.uniform(0.8, 1.2)),
                                 "E": float(rng.uniform(-0.3, 0.3))}
                else:
                    rx["Troe"] = {"A": float(rng.uniform(0.4, 0.9)),
                                  "T3": float(math.exp(rng.uniform(lo, hi))),
                                  "T1": float(math.exp(rng.uniform(lo, hi))),
                                  "T2": float(math.exp(rng.uniform(lo, hi)))}
        rx_out.append(rx)
    return {
        "description": f"synthetic mechanism {name}: {len(species)} species, {len(rx_out)} reactions",
        "generator": {"config": name, "seed": cfg.seed, "stoichiometric-rank": rank},
        "units": {"length": "m", "quantity": "kmol", "activation-energy": "J/kmol",
                  "pressure": "Pa", "temperature": "K"},
        "reference-pressure": 101325.0,
        "elements": [{"symbol": e, "atomic-weight": ATOMIC_WEIGHT[e]} for e in cfg.elements],
        "species": [
            {"name": sp.name, "composition": sp.comp, "molecular-weight": sp.weight,
             "inert": sp.inert,
             "thermo": {"model": "NASA7", "temperature-ranges": [T_LOW, T_MID, T_HIGH],
                        "data": [sp.low, sp.high]},
             "note": {"dh_f298_kJ_per_mol": sp.dh_f, "s298_J_per_mol_K": sp.s298}}
            for sp in species
        ],
        "reactions": rx_out,
    }


def write_mechanism(mech: dict, path: str) -> str:
    """Write a mechanism dict as JSON with round-trip (17 significant digit) floats."""
    with open(path, "w") as f:
        json.dump(mech, f, indent=1)
    return path


def mechanism_file(name: str, directory: str | None = None) -> str:
    """Path of the JSON file for mechanism ``name``, drawing and writing it on first use.

    Files go to ``directory``, else $CHEM_MECH_DIR, else ``_build/mechanisms`` at the
    repository root.  The draw is deterministic, so a cached file is always the same.
    """
    import os
    if directory is None:
        directory = os.environ.get("CHEM_MECH_DIR") or os.path.join(
            os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "_build", "mechanisms")
    os.makedirs(directory, exist_ok=True)
    path = os.path.join(directory, f"{name}.json")
    if not os.path.exists(path):
        tmp = f"{path}.tmp{os.getpid()}"
        write_mechanism(generate_mechanism(name), tmp)
        os.replace(tmp, path)
    return path
