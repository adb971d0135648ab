"""Seeded synthetic cell states: temperature, pressure and mass fractions.

Every batch is returned as plain arrays (T[n_cells], p[n_cells],
Y[n_cells, n_species]); each side of the comparison turns them into its
own state vector with its own code.  Mass fractions are Dirichlet draws;
temperatures are uniform; the pressure is the initial pressure of the
constant-pressure cells.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass(frozen=True)
class StateConfig:
    name: str
    mech: str
    seed: int
    n_cells: int
    T_range: tuple
    alpha: float
    p: float = 101325.0


STATE_CONFIGS = {
    # 1024 cells, T0 ~ U[1000, 1500] K, Y ~ Dirichlet(1)
    "be_small": StateConfig("be_small", "h2like_10_27", 2000, 1024, (1000.0, 1500.0), 1.0),
    # 1,048,576 cells, T0 ~ U[900, 2400] K, Y ~ Dirichlet(0.5)
    "ros2_1m": StateConfig("ros2_1m", "h2like_10_27", 2001, 1 << 20, (900.0, 2400.0), 0.5),
    # 262,144 cells, T0 ~ U[800, 2600] K, Y ~ Dirichlet(0.5)
    "ros2_methane": StateConfig("ros2_methane", "ch4like_53_325", 2002, 1 << 18, (800.0, 2600.0), 0.5),
    # 16,384 cells on the 53-species mechanism (adjoint workload)
    "adjoint_methane": StateConfig("adjoint_methane", "ch4like_53_325", 2003, 1 << 14, (800.0, 2600.0), 0.5),
    # 65,536 cells on the 150-species mechanism
    "ros2_large": StateConfig("ros2_large", "large_150_1000", 2004, 1 << 16, (900.0, 2400.0), 0.5),
}


def sample_states(n_species: int, n_cells: int, seed: int, T_range=(1000.0, 1500.0), alpha=1.0,
                  p=101325.0, first: int = 0):
    """Draw ``n_cells`` states; ``first`` skips that many cells of the same stream (for subsets).

    Returns (T, p, Y) with T, p of shape [n_cells] and Y of shape [n_cells, n_species].
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    total = first + n_cells
    T = rng.uniform(T_range[0], T_range[1], size=total)
    Y = rng.dirichlet(np.full(n_species, float(alpha)), size=total)
    T, Y = T[first:], Y[first:]
    return T.astype(np.float64), np.full(n_cells, float(p)), Y.astype(np.float64)


def sample_config(name: str, n_species: int, n_cells: int | None = None):
    """States of one named workload, or ``n_cells`` states with its distribution and seed.

    All temperatures are drawn before the compositions, so a smaller set is not the first cells of
    the full one (take a prefix of the full set for that)."""
    c = STATE_CONFIGS[name]
    n = c.n_cells if n_cells is None else n_cells
    return sample_states(n_species, n, c.seed, c.T_range, c.alpha, c.p)


def paper_sampler(n_species: int, n_cells: int, seed: int):
    """Accuracy-test states following the paper's random-state recipe (Section 5.1):
    T = 1000 + 1500 r K, p = (0.1 + 9.9 r) atm, composition fractions r_i renormalised
    (drawn here as mass fractions)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T = 1000.0 + 1500.0 * rng.uniform(size=n_cells)
    p = (0.1 + 9.9 * rng.uniform(size=n_cells)) * 101325.0
    r = rng.uniform(size=(n_cells, n_species))
    Y = r / r.sum(axis=1, keepdims=True)
    return T, p, Y


def oracle_subset(n_total: int, n_subset: int = 16384, seed: int = 5000):
    """Sorted indices of the seeded cell subset on which the CPU oracle is timed and checked."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.sort(rng.choice(n_total, size=min(n_subset, n_total), replace=False))


def loss_weights(n_cells: int, n_species: int, seed: int = 3000):
    """w ~ N(0, 1) per (cell, species) for the scalar loss of the adjoint workload."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size=(n_cells, n_species))
