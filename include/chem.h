/*
 * chem.h -- C ABI of the per-cell chemistry library (libchem.so) for AMD Instinct MI355X (gfx950).
 *
 * The library evaluates, for every CFD cell independently, the chemical state y = (T, C_1..C_ns)
 * of the ChemGen paper (arXiv 2510.10005, Section 3, eq. extracted_problem): NASA-7 species
 * thermodynamics (Section 2.1, Table 1), the source term S(y) = (omega_T, omega_1..omega_ns) with
 * Arrhenius, third-body and Troe/SRI/Lindemann falloff rates and reverse rates from equilibrium
 * constants (Section 2.2), its analytic Jacobian (Section 3.2), and the implicit integration of
 * dy/dt = S(y) over one operator-split step (backward Euler with Newton, Section 3.2; two-stage
 * Rosenbrock, Appendix A.3), plus the discrete adjoints of both integrations.
 *
 * Conventions shared by every call:
 *  - Units are SI with kmol: T [K], C [kmol/m^3], p [Pa], time [s].
 *  - Arrays named y, dydt, jac, T, p, Y, cp, h, s, g are DEVICE pointers to FP64 data laid out
 *    structure-of-arrays with leading dimension ld >= n_cells: component k of cell c lives at
 *    [k * ld + c].  State index 0 is T, index 1 + i is species i.  The Jacobian uses component
 *    (i * n + j) for dS_i/dy_j with n = ns + 1.
 *  - lnA (nullable) is a DEVICE array of nr FP64 values: ln of each reaction's (high-pressure)
 *    Arrhenius prefactor in SI-kmol units.  For a falloff reaction the low-pressure prefactor
 *    moves with it, so lnA_j scales k_f and k_r of reaction j alike.  NULL means the file's values.
 *  - stream is a hipStream_t (NULL = the default stream).  Work is enqueued asynchronously on it;
 *    argument errors are reported synchronously before anything is enqueued.
 *  - The caller owns every array passed in.  The library owns mechanisms, compiled kernels,
 *    tapes and its internal workspaces.  Calls on one mechanism from several host threads must
 *    use distinct streams; workspace-using calls (chem_integrate, chem_integrate_adjoint)
 *    serialise internally per mechanism.
 *  - Functions return chem_err; no C++ exception crosses the ABI.  chem_last_error_message()
 *    gives a human-readable detail of the last failure on the calling thread.
 */
#ifndef CHEM_H
#define CHEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct chem_mech chem_mech;   /* loaded mechanism + compiled kernels; immutable after load */
typedef struct chem_tape chem_tape;   /* adjoint tape: checkpoints and step records of one forward run */

typedef enum {
  CHEM_OK = 0,
  CHEM_EINVAL = 1,       /* bad argument (null pointer, ld < n_cells, unknown option value ...) */
  CHEM_ENOMEM = 2,       /* host or device allocation failed */
  CHEM_EPARSE = 3,       /* mechanism file unreadable or malformed */
  CHEM_EDEVICE = 4,      /* HIP runtime error (no device, launch failure ...) */
  CHEM_ECOMPILE = 5,     /* generated kernel source failed to compile */
  CHEM_ECELLS = 6,       /* only with CHEM_FLAG_CHECK_CELLS: at least one cell status != OK */
  CHEM_EUNSUPPORTED = 7  /* valid request this build does not implement */
} chem_err;

/* per-cell status written by chem_integrate (int32 per cell) */
enum {
  CHEM_CELL_OK = 0,
  CHEM_CELL_NEWTON_FAIL = 1,   /* backward Euler: Newton failed even after the deepest halving */
  CHEM_CELL_DT_UNDERFLOW = 2,  /* Rosenbrock: step size fell below h_min after a rejection */
  CHEM_CELL_MAX_STEPS = 3,     /* attempt budget exhausted */
  CHEM_CELL_NONFINITE = 4,     /* non-finite input state */
  CHEM_CELL_T_RANGE = 5        /* input temperature <= 0 */
};

enum { CHEM_BE = 0, CHEM_ROS2 = 1, CHEM_SDIRK2 = 2, CHEM_SDIRK4 = 3, CHEM_YASS = 4 };
enum { CHEM_LINSOLVE_LU = 0, CHEM_LINSOLVE_GMRES = 1 };
enum { CHEM_PRECOND_NONE = 0, CHEM_PRECOND_JACOBI = 1, CHEM_PRECOND_GAUSS_SEIDEL = 2 };
enum { CHEM_CONST_P = 0, CHEM_CONST_V = 1, CHEM_CONST_P_REACTOR = 2 };
enum { CHEM_PERSISTENT = 0, CHEM_PLAIN = 1 };
enum { CHEM_FLAG_CHECK_CELLS = 1 };  /* synchronise and return CHEM_ECELLS if a cell failed */

/*
 * Integrator options.  Fill with chem_default_options() and override fields.
 *  method   CHEM_BE: n_steps fixed steps of dt/n_steps (n_steps 0 means 1), each solved by full Newton
 *                    (G = I/h - J(y_k) re-evaluated every iteration, Section 3.2); a step whose
 *                    Newton iteration fails is split in two halves recursively down to
 *                    halving_max_depth (the step-halving of YASS, Appendix A.4).
 *           CHEM_ROS2: two-stage Rosenbrock of Appendix A.3 from t = 0 to dt; adaptive step size
 *                    (embedded first-order solution, weighted RMS error, rtol/atol on T [K] and
 *                    on mass fractions) unless n_steps > 0, which gives fixed steps dt/n_steps.
 *           CHEM_SDIRK2: two-stage SDIRK of Appendix A.1 (gamma = 1 - sqrt(2)/2), n_steps fixed steps
 *                    of dt/n_steps (0 means 1); each stage Gamma = S(b + gamma h Gamma) is solved by
 *                    full Newton, (I - gamma h J) delta = -(Gamma - S), from the guess S(y_n), with
 *                    the state change gamma h delta in the Newton test below.  A failed step sets
 *                    CHEM_CELL_NEWTON_FAIL (no halving).  Persistent form only, n <= 24 only, no
 *                    adjoint tape; counters: completed steps, 0, Newton iterations.
 *           CHEM_SDIRK4: the five-stage, fourth-order, stiffly accurate SDIRK of Appendix A.2
 *                    (a_ii = 4/15; the tableau's 7-digit values as printed, a_52 = b_2).  Stage p
 *                    solves Gamma_p = S(y_n + h sum_{j<p} a_pj Gamma_j + a_pp h Gamma_p) by Newton
 *                    as for CHEM_SDIRK2; y_{n+1} = y_n + h sum_p b_p Gamma_p.  Same restrictions,
 *                    failure status and counters as CHEM_SDIRK2.
 *           CHEM_YASS: YASS of Appendix A.4 over n_steps fixed steps of dt/n_steps (0 means 1).  Each
 *                    substep of size h solves the linearised backward-Euler step
 *                    (I - h J(y)) dy = h S(y) once, with LU (linear_solver CHEM_LINSOLVE_LU) or
 *                    restarted GMRES (CHEM_LINSOLVE_GMRES, Section 3.4; left preconditioning by
 *                    M = diag(I - hJ) with CHEM_PRECOND_JACOBI, by M = its lower triangle with
 *                    the diagonal (forward substitution) with CHEM_PRECOND_GAUSS_SEIDEL, or
 *                    none; stop when the Euclidean
 *                    norm of the preconditioned residual is <= krylov_rtol |M^-1 b|, or after
 *                    krylov_max_iter iterations; restart length krylov_dim, 0 = system size).
 *                    The substep is accepted when dy is finite, T stays > 0 and
 *                    max(|dT|/T, max_i |dY_i|) <= yass_alpha (dY: mass fractions); else it is
 *                    halved, and a cell whose halved substep would be below h_min stops with
 *                    CHEM_CELL_DT_UNDERFLOW.  A halved substep is kept until the fixed step is
 *                    covered; every fixed step starts from dt/n_steps.  max_steps bounds the
 *                    attempts (CHEM_CELL_MAX_STEPS).  Persistent form only, n <= 24 only, no
 *                    adjoint tape; counters: accepted substeps, rejected attempts, Krylov
 *                    iterations (0 with LU).
 *  energy   CHEM_CONST_P: omega_T = -sum H_i omega_i / sum C_i Cp_i (Appendix B)
 *           CHEM_CONST_V: omega_T = -sum U_i omega_i / sum C_i Cv_i (Section 3)
 *           CHEM_CONST_P_REACTOR: the constant-pressure reactor with its density change (the
 *           omega_T of CHEM_CONST_P, species sources omega_i - C_i g; see chem_source_terms).
 *           Every method and form; adjoint tapes for backward Euler only (CHEM_EUNSUPPORTED for a
 *           Rosenbrock tape).  Its expansion changes
 *           every concentration, so for n <= 24 the integrators run a second build of the
 *           mechanism whose solved system holds every species (the regular one holds the species
 *           that take part in no reaction fixed); it is generated, compiled (or taken from the
 *           kernel cache, where chem_precompile puts it) and loaded on the first such call.
 *           chem_integrate_noalloc refuses the mode until that has happened.
 *  form     CHEM_PERSISTENT: one persistent kernel, cells pulled from a work queue lane by lane.
 *           CHEM_PLAIN: one kernel launch per substep (BE: per full step) over all cells.
 *  Newton convergence: max_i |delta_i| / sc_i <= 1 with sc_T = newton_rtol T + newton_atol_T and,
 *  for species, sc = (newton_atol_Y + newton_rtol |Y_i|) rho / W_i; divergence: the scaled
 *  norm grows from the third iteration on.
 *  probe_attempts  (CHEM_ROS2 + CHEM_PERSISTENT) > 0: the split step runs as a probe launch in
 *           which each cell takes at most probe_attempts attempts, then a resume launch that
 *           continues the unfinished cells, those with the most predicted remaining work first
 *           (their first attempts' rate extrapolated), so that long cells do not start last.
 *           The step sequence of every cell, and so every result, is the same as with 0 (one
 *           launch).  Ignored for other methods and forms, and when n_cells >= 2^31.
 */
typedef struct {
  int method;
  int energy;
  int form;
  int flags;
  double dt;
  int n_steps;
  int max_steps;
  double rtol;
  double atol;
  double h_min;
  int newton_max;
  int halving_max_depth;
  double newton_rtol;
  double newton_atol_T;
  double newton_atol_Y;
  int probe_attempts;
  int reserved_;  /* padding; keep 0 */
  double yass_alpha;    /* CHEM_YASS: bound on the substep's change (see method) */
  int linear_solver;    /* CHEM_YASS: CHEM_LINSOLVE_LU or CHEM_LINSOLVE_GMRES */
  int krylov_dim;       /* GMRES restart length, 0 = the size of the solved system */
  double krylov_rtol;   /* GMRES stop: preconditioned residual <= krylov_rtol |M^-1 b| */
  int krylov_max_iter;  /* GMRES iterations per solve, over all restarts */
  int krylov_precond;   /* CHEM_PRECOND_JACOBI, CHEM_PRECOND_GAUSS_SEIDEL or CHEM_PRECOND_NONE */
} chem_integrator_opts;

/* Defaults: BE, const-p, persistent, dt 1e-7, n_steps 0, max_steps 100000, rtol 1e-6, atol 1e-10,
 * h_min 1e-20, newton_max 10, halving_max_depth 8, newton_rtol 1e-10, newton_atol_T 1e-8 K,
 * newton_atol_Y 1e-14, probe_attempts 48, yass_alpha 0.1, linear_solver LU, krylov_dim 0,
 * krylov_rtol 1e-12, krylov_max_iter 100, krylov_precond Jacobi. */
void chem_default_options(chem_integrator_opts* opts);

/* Human-readable name of an error code (static string, never NULL). */
const char* chem_error_string(chem_err err);
/* Detail of the last error raised on the calling thread (static thread-local buffer). */
const char* chem_last_error_message(void);

/*
 * Load a mechanism file (Cantera-like JSON: species with NASA-7 data, or with the single-range
 * model {"model": "polynomial-cp", "cp-R": [a_0..a_np], "h0", "s0"} of Section 2.1 -- cp/R =
 * sum a_k T^k, h/RT = sum a_k T^k/(k+1) + h0/T, s/R = a_0 ln T + sum_(k>=1) a_k T^k/k + s0; n <= 24
 * only; reactions of type
 * elementary, three-body, falloff with Troe, SRI (Section 2.2) or Lindemann broadening, or
 * pressure-dependent-Arrhenius (P-log: {P [Pa], A, b, Ea} sets at distinct pressures, ln k linear
 * in ln p between them with p = R T sum C, the end sets outside); A, b, Ea in SI-kmol with
 * Ea in J/kmol -- the units of the paper's worked example, Section 4.3), validate it, generate
 * HIP source specialised to it (the code-generation step of Section 4.3) and compile it for the
 * current device's architecture with hipRTC.  Compiled code objects are cached in cache_dir (or
 * $CHEM_KERNEL_CACHE, else a per-user temp directory) keyed by a hash of the generated source
 * and the compiler options.  The current HIP device at load time is the one the mechanism runs on.
 * State size n = species + 1 selects the kernel form: n <= 24 one cell per GPU lane with the
 * Jacobian and its LU in registers (every method, form and adjoint); 24 < n <= 160 the block form,
 * one cell per 256-thread workgroup with the species, reactions and matrix rows spread over the
 * threads (constants in generated tables) and the iteration matrix factored by a pivoted LU whose
 * updates run on the FP64 matrix cores (Section 3.4, direct solver).  In the block form
 * chem_integrate and chem_autotune serve CHEM_BE and CHEM_ROS2 in the persistent form, with
 * backward-Euler adjoint tapes (the plain form, the other methods and Rosenbrock tapes return
 * CHEM_EUNSUPPORTED); its Jacobian API kernel runs
 * one cell per 64-lane wavefront for n <= 64.  n > 160 is rejected with CHEM_EUNSUPPORTED.
 * On success *out owns the mechanism; release it with chem_free_mechanism.
 */
chem_err chem_load_mechanism(const char* path, const char* cache_dir, chem_mech** out);
void chem_free_mechanism(chem_mech* mech);

/* Generate and compile the kernels of a mechanism file for gfx950 into cache_dir without needing
 * a GPU (the ahead-of-time step of the build).  A mechanism whose state exceeds the register-
 * resident limit (n > 24) is compiled as four programs (API kernels, Rosenbrock, backward Euler,
 * adjoint) on concurrent threads.  Writes the code-object path(s) to path_out, separated by ';'
 * (truncated to path_cap - 1 characters). */
chem_err chem_precompile(const char* path, const char* cache_dir, char* path_out, size_t path_cap);

/* Sizes: species, reactions, elements, state length n = ns + 1. */
chem_err chem_mechanism_info(const chem_mech* mech, int* n_species, int* n_reactions, int* n_elements,
                             int* n_state);
/* HOST copies: molecular weights [ns] (kg/kmol) and the file's ln A [nr]. */
chem_err chem_molecular_weights(const chem_mech* mech, double* W_host);
chem_err chem_default_lnA(const chem_mech* mech, double* lnA_host);

/*
 * Species thermodynamics at temperatures T [ld] (Table 1, mass-specific): cp [J/kg/K], h [J/kg],
 * s0 [J/kg/K] at p_ref, g0 = h - T s0 [J/kg]; each output [ns][ld].  Any output may be NULL.
 */
chem_err chem_thermo(const chem_mech* mech, int64_t n_cells, int64_t ld, const double* T,
                     double* cp, double* h, double* s, double* g, void* stream);

/* Temperature from the energy density (Section 2.1, eqs. temperature-nonlinear,
 * netwons-method-temperature): n_iter Newton iterations (the paper uses 5) of
 *   T_k = T_{k-1} + (e - e(C, T_{k-1})) / e_T(C, T_{k-1})
 * with e = rho u = sum_i C_i U_i(T) and e_T = rho c_v = sum_i C_i Cv_i for energy CHEM_CONST_V, or
 * e = rho h = sum_i C_i H_i(T) and e_T = rho c_p = sum_i C_i Cp_i for CHEM_CONST_P (molar U, H,
 * Cv, Cp from the NASA-7 fits; Cv = Cp - R).  (The printed update subtracts the quotient; the
 * Newton equation printed just before it fixes the sign used here.)
 * C[ns][ld] (kmol/m^3; e.g. the species rows of a state array y + ld), e[ld] (J/m^3) and T0[ld]
 * (K, the initial guess) in; T[ld] out (T may alias T0).  n_iter >= 1.  No per-cell checks: a
 * non-positive or non-finite result propagates.  CHEM_CONST_P_REACTOR is the enthalpy form of
 * CHEM_CONST_P.  CHEM_EINVAL for null pointers or a bad mode. */
chem_err chem_T_from_energy(const chem_mech* mech, int64_t n_cells, int64_t ld, const double* C, const double* e,
                            const double* T0, int energy, int n_iter, double* T, void* stream);

/* Linearised species production term of the CFD coupling (the detonation case's eq. openfom_RR):
 * R[ns][ld] = W_i (C_i^{n+1} - C_i^n) / dt  [kg/(m^3 s)] from the states y_n and y_np1
 * ([n][ld] each: T, C) before and after a chemistry step of length dt > 0. */
chem_err chem_cfd_source(const chem_mech* mech, int64_t n_cells, int64_t ld, const double* y_n, const double* y_np1,
                         double dt, double* R, void* stream);

/* Source term S(y) (eq. extracted_problem): dydt[n][ld] from y[n][ld].
 * energy CHEM_CONST_P / CHEM_CONST_V: (omega_T, omega_1..omega_ns) as in Section 3 and Appendix B
 * (dC_i/dt = omega_i: the density is held, so p = R T sum C drifts).
 * energy CHEM_CONST_P_REACTOR: the homogeneous reactor at fixed pressure.  C_i = rho Y_i / W_i with
 * dY_i/dt = W_i omega_i / rho and rho = p Wbar / (R T) gives d ln rho / dt = -g,
 *   g = sum_i omega_i / sum_i C_i + omega_T / T,   dC_i/dt = omega_i - C_i g,
 * and omega_T as for CHEM_CONST_P; R T sum C and sum C_i H_i / rho stay constant along it. */
chem_err chem_source_terms(const chem_mech* mech, int64_t n_cells, int64_t ld, const double* y,
                           const double* lnA, int energy, double* dydt, void* stream);

/* Analytic Jacobian dS/dy (eq. derivative_matrices_temp_evol): jac[n*n][ld], row-major i*n+j.
 * For CHEM_CONST_P_REACTOR the species rows are J_ik - delta_ik g - C_i dg/dy_k (J: the
 * CHEM_CONST_P Jacobian; dg/dy_k from the column sums of its species rows and its T row). */
chem_err chem_jacobian(const chem_mech* mech, int64_t n_cells, int64_t ld, const double* y,
                       const double* lnA, int energy, double* jac, void* stream);

/* Initial-state map: y = (T, C) with rho = p Wbar/(R T), C_i = rho Y_i / W_i.
 * T[ld], p[ld], Y[ns][ld] in; y[n][ld] out. */
chem_err chem_state_from_TPY(const chem_mech* mech, int64_t n_cells, int64_t ld, const double* T,
                             const double* p, const double* Y, double* y, void* stream);
/* Mass fractions Y_i = W_i C_i / sum_k W_k C_k: Y[ns][ld] from y[n][ld]. */
chem_err chem_mass_fractions(const chem_mech* mech, int64_t n_cells, int64_t ld, const double* y,
                             double* Y, void* stream);
/* Pull-backs (vector-Jacobian products) of the two maps above, for gradients:
 *  chem_state_from_TPY_vjp: given dL/dy [n][ld] at the map's output, writes dL/dT [ld] and
 *                           dL/dY [ns][ld] (unconstrained partials; Y is not renormalised).
 *  chem_mass_fractions_vjp: given dL/dY [ns][ld] and dL/dT_direct [ld] (nullable), writes
 *                           dL/dy [n][ld] at y. */
chem_err chem_state_from_TPY_vjp(const chem_mech* mech, int64_t n_cells, int64_t ld, const double* T,
                                 const double* p, const double* Y, const double* dL_dy, double* dL_dT,
                                 double* dL_dY, void* stream);
chem_err chem_mass_fractions_vjp(const chem_mech* mech, int64_t n_cells, int64_t ld, const double* y,
                                 const double* dL_dY, const double* dL_dT, double* dL_dy, void* stream);

/*
 * Integrate every cell over one split step: y[n][ld] is read and overwritten with the final
 * state.  status [ld] (required) receives a CHEM_CELL_* code; counters (nullable) [3][ld]
 * receives accepted substeps (BE: completed full steps), rejected attempts and Newton
 * iterations.  A failed cell keeps its last accepted state.  tape (nullable) records what
 * chem_integrate_adjoint needs; it must have been created for >= n_cells cells and for this
 * method (chem_tape_create: CHEM_BE; chem_tape_create_ros2: CHEM_ROS2 in the persistent form),
 * and the same options must be used by the adjoint call.
 */
chem_err chem_integrate(const chem_mech* mech, int64_t n_cells, int64_t ld, double* y,
                        const double* lnA, const chem_integrator_opts* opts, chem_tape* tape,
                        int32_t* status, int32_t* counters, void* stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): chem_integrate without a tape, persistent form only, with
 * every library workspace (work-queue counter, probe/resume schedule, parked cells' state and
 * order, and the counters when counters is NULL) taken from a device array of 48 MiB + 4352 B
 * that the library holds per GPU until the process ends; it calls no hipMalloc, hipFree or other
 * allocating routine.  Limits: n_cells <= 2^20 and, with counters NULL, ld <= 2^20
 * (CHEM_EINVAL otherwise); CHEM_FLAG_CHECK_CELLS is refused.  The array is shared by every
 * mechanism and stream on a GPU and keeps the last call's contents (what must start at zero is
 * cleared by each call): calls that overlap in time on one GPU race, so the caller must order
 * them (one stream, or events).  Same arguments, results and per-cell statuses as chem_integrate.
 */
chem_err chem_integrate_noalloc(const chem_mech* mech, int64_t n_cells, int64_t ld, double* y, const double* lnA,
                                const chem_integrator_opts* opts, int32_t* status, int32_t* counters, void* stream);

/* Tape for the backward-Euler discrete adjoint (every n <= 160): the state is checkpointed every
 * checkpoint_every steps; the backward pass recomputes each segment from its checkpoint.  In the
 * block form (n > 24) the backward pass maps cells statically to workgroups, one cell at a time. */
chem_err chem_tape_create(const chem_mech* mech, int64_t n_cells, int checkpoint_every, chem_tape** out);

/* Tape for the discrete adjoint of the two-stage Rosenbrock method (Appendix A.3), n <= 24 only
 * (CHEM_EUNSUPPORTED otherwise).  chem_integrate with method CHEM_ROS2, the persistent form and
 * this tape records the initial states and the step size of every accepted step (8 B per step
 * and cell), on the device, allocated by that call; chem_integrate_adjoint rebuilds a checkpoint
 * every checkpoint_every accepted steps (8 n B per checkpoint and cell, in the tape) by replaying
 * the recorded steps.  A cell that needs more than max_steps accepted steps stops with
 * CHEM_CELL_MAX_STEPS.  The step-size controller is not differentiated: the adjoint is that of the
 * recorded step sequence. */
chem_err chem_tape_create_ros2(const chem_mech* mech, int64_t n_cells, int max_steps, int checkpoint_every,
                               chem_tape** out);
void chem_tape_free(chem_tape* tape);

/*
 * Discrete adjoint of the recorded integration.  Given dL/dy_N [n][ld] at the final state, writes
 * dL/dy_0 [n][ld] and dL/dlnA [nr] (summed over cells, deterministic order).  Cells whose forward
 * status was not CHEM_CELL_OK get dL/dy_0 = 0 and add nothing to dL/dlnA.  Uses the same lnA as
 * the forward run.
 * Backward Euler: every accepted (sub)step y -> y' with step h contributes
 *   (I/h - J(y'))^T mu = lambda',  lambda = mu / h,  dL/dlnA_j += q_j(y') (sum_i nu_ij mu_i + mu_T dwT_j)
 * where dwT_j is d omega_T / d lnA_j per unit q_j.
 * Rosenbrock: every recorded step y -> y + m1 g1 + m2 g2 with G = I/(gamma h) - J(y) and
 * y* = y + alpha g1 contributes (lambda = dL/dy' on entry, dL/dy on exit)
 *   G^T u2 = m2 lambda,  G^T u1 = m1 lambda + alpha J(y*)^T u2 + (beta/h) u2,
 *   lambda <- lambda + J(y)^T u1 + J(y*)^T u2 + (J'(y)[g1])^T u1 + (J'(y)[g2])^T u2,
 *   dL/dlnA += u1^T (dS/dlnA(y) + (dS/dlnA)'(y)[g1]) + u2^T (dS/dlnA(y*) + (dS/dlnA)'(y)[g2])
 * (F'(y)[v]: derivative along v, evaluated with dual numbers).
 */
chem_err chem_integrate_adjoint(const chem_mech* mech, chem_tape* tape, const double* lnA,
                                const double* dL_dyN, double* dL_dy0, double* dL_dlnA, void* stream);

/*
 * Kernel launch configuration of chem_integrate for a method/form: threads per block and blocks
 * of the persistent grid (0 = library default).  chem_autotune times the candidates on the given
 * cells (which it leaves unchanged) and keeps the fastest; chem_get_launch reports the current one.
 * For CHEM_BE and CHEM_ROS2 of mechanisms with 24 < n <= 64 (block form, factors in LDS) the
 * candidates also span the LU strategy of the per-cell direct solve (Section 3.4).
 */
chem_err chem_set_launch(chem_mech* mech, int method, int form, int block, int grid);
chem_err chem_get_launch(const chem_mech* mech, int method, int form, int* block, int* grid);
chem_err chem_autotune(chem_mech* mech, int64_t n_cells, int64_t ld, const double* y, const double* lnA,
                       const chem_integrator_opts* opts, void* stream);

/*
 * LU strategy of the persistent integration kernel of a method (the direct solve of Section 3.4,
 * partial pivoting in both): 0 (default) = the panel of four columns factored in registers by
 * one wavefront with a DPP wave maximum and one barrier per panel, triangular solves by one
 * wavefront in registers; 1 = the panel factored in LDS with a 64-bit key maximum and the pivot
 * rows staged in LDS (several barriers per panel), solves blocked by 16 steps.  Both update the
 * trailing matrix with FP64 matrix-core products.  Strategy 1 exists for CHEM_BE and CHEM_ROS2 of
 * mechanisms with 24 < n <= 64; elsewhere chem_set_lu_strategy(…, 1) returns CHEM_EUNSUPPORTED
 * (and mechanisms with n > 64 always use the LDS-panel LU).  A run that records an adjoint tape
 * uses strategy 0, as the adjoint's replays do.  Results of the two strategies agree to rounding.
 * Errors: CHEM_EINVAL for a null mechanism/pointer, an unknown method or a strategy other than
 * 0 or 1.
 */
chem_err chem_set_lu_strategy(chem_mech* mech, int method, int strategy);
chem_err chem_get_lu_strategy(const chem_mech* mech, int method, int* strategy);

#ifdef __cplusplus
}
#endif
#endif /* CHEM_H */
