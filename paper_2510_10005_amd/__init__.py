"""MI355X-native per-cell chemistry: generated HIP kernels for thermo, source terms, analytic
Jacobians and implicit integrators behind a C ABI (include/chem.h), with a thin Python layer."""

from ._binding import (  # noqa: F401
    CHEM_BE, CHEM_ROS2, CHEM_SDIRK2, CHEM_SDIRK4, CHEM_YASS, CHEM_LINSOLVE_LU, CHEM_LINSOLVE_GMRES,
    CHEM_PRECOND_NONE, CHEM_PRECOND_JACOBI, CHEM_PRECOND_GAUSS_SEIDEL, CHEM_CONST_P, CHEM_CONST_V, CHEM_CONST_P_REACTOR, CHEM_PERSISTENT, CHEM_PLAIN, CHEM_FLAG_CHECK_CELLS,
    ChemError, IntegratorOptions, Mechanism, Tape, default_options, load, precompile,
)
