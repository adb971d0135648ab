"""CPU FP64 oracle for the per-cell chemistry hot path -- TEST INFRASTRUCTURE ONLY.

This package is a plain, slow, NumPy (float64) restatement of what the
paper computes for every cell: NASA-7 thermodynamics (Section 2.1,
Table 1), rates of progress and net production rates (Section 2.2,
eqs. for q_j, K_j, the Arrhenius, third-body and Troe forms), the
temperature source under constant volume (Section 3, eq.
temperature_source) or constant pressure (Appendix B), the analytic
source Jacobian (Section 3.2), backward Euler with Newton (Section 3.2),
the SDIRK schemes (two and five stages, Appendix A.1/A.2), YASS (Appendix
A.4) with an LU or Jacobi-preconditioned GMRES solve (Section 3.4), the
CFD coupling (temperature from the energy density by Newton, Section 2.1; the
linearised species source of the detonation case) and the
two-stage Rosenbrock scheme (Appendix A.3), plus forward and
reverse sensitivities of the backward-Euler map and the discrete adjoint
of the Rosenbrock map along its accepted step sequence.

It exists to check the HIP library, never to stand in for it: only the
test suite, the smoke check and the CPU-baseline leg of the benchmark may
import it.  It shares no code with the HIP path; the only common input is
the mechanism file and the seeded states from ``synth``.

Parity status: every function here is pinned by tests against
independent facts (closed forms, complex-step derivatives, invariants,
equilibrium, convergence order, finite differences) except the adaptive
step-size controller constants of the Rosenbrock integrator, which the
paper does not give ("parity unpinned" for those constants: only the
resulting solution's convergence to the fixed-step reference is pinned).
"""

from .mechanism import Mechanism, load_mechanism  # noqa: F401
from .thermo import nasa7_molar, thermo_mass_specific  # noqa: F401
from .kinetics import (  # noqa: F401
    CONST_P, CONST_V, CONST_P_REACTOR, rates_of_progress, source_terms, jacobian, jacobian_complex_step,
    dsource_dlnA, source_sum_scale,
)
from .integrate import (  # noqa: F401
    CELL_OK, CELL_NEWTON_FAIL, CELL_DT_UNDERFLOW, CELL_MAX_STEPS, CELL_NONFINITE, CELL_T_RANGE,
    LINSOLVE_LU, LINSOLVE_GMRES, IntegratorOptions, state_from_TPY, mass_fractions, integrate_be, integrate_ros2,
    integrate_sdirk2, integrate_sdirk4, integrate_yass,
)
from .linsolve import gmres  # noqa: F401
from .coupling import T_from_energy, energy_density, openfoam_source  # noqa: F401
from .sensitivity import be_tangent, be_adjoint, ros2_replay, ros2_adjoint, ros2_adjoint_cell  # noqa: F401
