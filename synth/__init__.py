"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only draws inputs: mechanism files (species, NASA-7 thermo
data, reactions with their rate parameters) and batches of cell states
(T, p, mass fractions).  It evaluates no rate, no source term, no
Jacobian and no integrator step; those live separately in ``oracle/``
(CPU reference) and in the HIP library, which share no code.
"""

from .mechgen import generate_mechanism, write_mechanism, mechanism_file, MECH_CONFIGS  # noqa: F401
from .states import sample_states, STATE_CONFIGS  # noqa: F401
