// Runs kernels of the generated block-form source (one cell per 256-thread workgroup) on the fiber
// emulation (fiber.hpp).
// Usage:
//   block_driver be|ros2|ros2p n ld dt n_steps in.bin out.bin [grid] [lu_strategy]
//     (ros2p: probe/resume schedule; lu_strategy 1: the LDS-panel kernels, be and ros2 only)
//     in.bin: state [NY][ld] then ln A [NR]; out.bin: state, status [ld], counters [3][ld]
//   block_driver adj n ld dt n_steps K in.bin out.bin [grid] [energy]   (backward Euler with a tape, then its adjoint)
//     in.bin: state [NY][ld], ln A [NR], dL/dy_N [NY][ld]; out.bin: state, status [ld], dL/dy0 [NY][ld],
//     dL/dlnA [NR] (workgroup partials summed in workgroup order)
//   block_driver src|jac n ld in.bin out.bin          (API kernels of mechanisms with n > 64)
//     in.bin: state [NY][ld] then ln A [NR]; out.bin: sources [NY][ld] then (jac) [n][NY][NY]
//   block_driver lu in.bin out.bin [lu_strategy]
//     in.bin: A [NY][NY] row-major, b [NY], lam [NY]; out.bin: x = A^-1 b [NY], mu = A^-T lam [NY], then
//     the factors [NY][NY], the pivot row of each step [NY] and the reciprocal pivots [NY]
#include "fiber.hpp"
#include <vector>
#define BK_OCC   // no GPU occupancy attribute in the host build
#include "src.hip"

static bool read_all(const char* path, std::vector<double>& v) {
  FILE* f = fopen(path, "rb");
  if (!f) return false;
  const bool ok = fread(v.data(), 8, v.size(), f) == v.size();
  fclose(f);
  return ok;
}

// standalone factor + solves with LU strategy LUS: G = 0 I - (-A) = A
template <int LUS>
static void lu_kernel(const double* A, const double* b, const double* lam, double* x, double* mu, double* ws,
                      double* dump) {
  BkShared& sh = bk_shared();
  const int t = threadIdx.x;
  double* F = bk_fptr(sh, ws);
  for (int e = t; e < NY * NY; e += BK_T) F[(e / NY) * BK_FLD + e % NY] = -A[e];
  if (t < BK_NP) {
    sh.v0[t] = t < NY ? b[t] : 0.0;
    sh.v2[t] = t < NY ? lam[t] : 0.0;
  }
  __syncthreads();
  bk_factor<LUS>(sh, F, 0.0);
  bk_fsolve<LUS>(sh, F, sh.v0, sh.v1);
  bk_fsolve_T<LUS>(sh, F, sh.v2, sh.v3);
  if (t < NY) {
    x[t] = sh.v1[t];
    mu[t] = sh.v3[t];
  }
  // factors (row-major NY x NY), pivot row of each step, reciprocal pivots
  if (dump) {
    for (int e = t; e < NY * NY; e += BK_T) dump[e] = F[(e / NY) * BK_FLD + e % NY];
    if (t < NY) {
      dump[NY * NY + t] = sh.prow[t];
      dump[NY * NY + NY + t] = sh.dinv[t];
    }
  }
}

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  // every workgroup starts with its LDS full of 0xFF bytes (NaN doubles, -1 integers)
  emu::g_block_start = [] { std::memset(&bk_shared(), 0xFF, sizeof(BkShared)); };
  const char* which = argv[1];
  if (!strcmp(which, "lu")) {
    std::vector<double> in((size_t)NY * NY + 2 * NY), out(2 * NY + NY * NY + 2 * NY, 0.0), ws((size_t)BK_NP * BK_NP, 0.0);
    if (!read_all(argv[2], in)) return 4;
    const double* A = in.data();
    const int lus = argc > 4 ? atoi(argv[4]) : 0;
    emu::run_grid(1, [&] {
      if (lus == 0)
        lu_kernel<0>(A, A + NY * NY, A + NY * NY + NY, out.data(), out.data() + NY, ws.data(), out.data() + 2 * NY);
      else
        lu_kernel<1>(A, A + NY * NY, A + NY * NY + NY, out.data(), out.data() + NY, ws.data(), out.data() + 2 * NY);
    }, BK_T);
    FILE* f = fopen(argv[3], "wb");
    fwrite(out.data(), 8, out.size(), f);
    fclose(f);
    return 0;
  }
  const long long n = atoll(argv[2]), ld = atoll(argv[3]);
  if (!strcmp(which, "src") || !strcmp(which, "jac")) {
#if CHEM_WAVE_API
    return 5;
#else
    std::vector<double> in((size_t)NY * ld + NR), S((size_t)NY * ld, 0.0), J;
    if (!read_all(argv[4], in)) return 4;
    const double* y = in.data();
    const double* lnA = in.data() + (size_t)NY * ld;
    const int energy = argc > 6 ? atoi(argv[6]) : 0;
    emu::run_grid((unsigned)n, [&] { chem_k_source(n, ld, y, lnA, energy, S.data()); }, BK_T);
    if (!strcmp(which, "jac")) {
      J.assign((size_t)n * NY * NY, 0.0);
      emu::run_grid((unsigned)n, [&] { chem_k_jacobian(n, ld, y, lnA, energy, J.data(), 0); }, BK_T);
    }
    FILE* f = fopen(argv[5], "wb");
    fwrite(S.data(), 8, S.size(), f);
    fwrite(J.data(), 8, J.size(), f);
    fclose(f);
    return 0;
#endif
  }
  if (!strcmp(which, "adj")) {
#if CHEM_IN_GROUP(3)
    if (argc < 9) return 2;
    const double dt = atof(argv[4]);
    const int n_steps = atoi(argv[5]), K = atoi(argv[6]);
    const unsigned grid = argc > 9 ? (unsigned)atoi(argv[9]) : 2u;
    std::vector<double> in((size_t)2 * NY * ld + NR);
    if (!read_all(argv[7], in)) return 4;
    std::vector<double> y(in.begin(), in.begin() + (size_t)NY * ld);
    std::vector<double> lnA(in.begin() + (size_t)NY * ld, in.begin() + (size_t)NY * ld + NR);
    std::vector<double> lamN(in.begin() + (size_t)NY * ld + NR, in.end());
    std::vector<double> ws((size_t)grid * BK_NP * BK_NP, 0.0), ckpt((size_t)(n_steps / K + 1) * NY * ld, 0.0);
    std::vector<double> seg((size_t)grid * K * NY, 0.0), gpart((size_t)grid * NR, 0.0), lam0((size_t)NY * ld, 0.0);
    std::vector<unsigned short> nsub((size_t)n_steps * ld, 0);
    std::vector<int> status(ld, -7), counters(3 * ld, 0);
    unsigned long long queue = 0;
    ChemOpts o{};
    o.dt = dt; o.rtol = 1e-6; o.atol = 1e-10; o.h_min = 1e-20; o.newton_rtol = 1e-10; o.newton_atol_T = 1e-8;
    o.newton_atol_Y = 1e-14; o.n_steps = n_steps; o.max_steps = 100000; o.newton_max = 10;
    o.halving_max_depth = 8; o.energy = argc > 10 ? atoi(argv[10]) : 0; o.ckpt_every = K;
    emu::run_grid(grid, [&] {
      chem_k_be_persistent(n, ld, y.data(), lnA.data(), o, status.data(), counters.data(), &queue, ws.data(), 0,
                           ckpt.data(), nsub.data());
    }, BK_T);
    emu::run_grid(grid, [&] {
      chem_k_be_adjoint(n, ld, lnA.data(), o, status.data(), ckpt.data(), nsub.data(), lamN.data(), lam0.data(),
                        gpart.data(), seg.data(), grid, ws.data(), grid, nullptr);
    }, BK_T);
    std::vector<double> g(NR, 0.0);
    for (unsigned b = 0; b < grid; ++b)
      for (int j = 0; j < NR; ++j) g[j] += gpart[(size_t)b * NR + j];
    FILE* f = fopen(argv[8], "wb");
    fwrite(y.data(), 8, y.size(), f);
    fwrite(status.data(), 4, ld, f);
    fwrite(lam0.data(), 8, lam0.size(), f);
    fwrite(g.data(), 8, g.size(), f);
    fclose(f);
    return 0;
#else
    return 5;
#endif
  }
  if (argc < 8) return 2;
  const double dt = atof(argv[4]);
  const int n_steps = atoi(argv[5]);
  const unsigned grid = argc > 8 ? (unsigned)atoi(argv[8]) : 2u;
  const int lus = argc > 9 ? atoi(argv[9]) : 0;   // LU strategy (1: the LDS-panel kernels)
#if !BK_LDS_F
  if (lus != 0) return 6;
#endif
  std::vector<double> in((size_t)NY * ld + NR);
  if (!read_all(argv[6], in)) return 4;
  std::vector<double> y(in.begin(), in.begin() + (size_t)NY * ld), lnA(in.begin() + (size_t)NY * ld, in.end());
  std::vector<double> ws((size_t)grid * BK_NP * BK_NP, 0.0);
  std::vector<int> status(ld, -7), counters(3 * ld, 0);
  unsigned long long queue = 0;
  ChemOpts o{};
  o.dt = dt; o.rtol = 1e-6; o.atol = 1e-10; o.h_min = 1e-20; o.newton_rtol = 1e-10; o.newton_atol_T = 1e-8;
  o.newton_atol_Y = 1e-14; o.n_steps = n_steps; o.max_steps = 100000; o.newton_max = 10;
  o.halving_max_depth = 8; o.energy = argc > 10 ? atoi(argv[10]) : 0; o.ckpt_every = 1;
  long long coll;
  if (!strcmp(which, "be"))
    coll = emu::run_grid(grid, [&] {
      if (lus == 0)
        chem_k_be_persistent(n, ld, y.data(), lnA.data(), o, status.data(), counters.data(), &queue, ws.data(), 0,
                             nullptr, nullptr);
#if BK_LDS_F
      else
        chem_k_be_persistent_lup(n, ld, y.data(), lnA.data(), o, status.data(), counters.data(), &queue, ws.data(),
                                 0, nullptr, nullptr);
#endif
    }, BK_T);
  else if (!strcmp(which, "ros2"))
    coll = emu::run_grid(grid, [&] {
      if (lus == 0)
        chem_k_ros2_persistent(n, ld, y.data(), lnA.data(), o, status.data(), counters.data(), &queue, ws.data(), 0,
                               0, nullptr, nullptr, nullptr);
#if BK_LDS_F
      else
        chem_k_ros2_persistent_lup(n, ld, y.data(), lnA.data(), o, status.data(), counters.data(), &queue,
                                   ws.data(), 0, 0, nullptr, nullptr, nullptr);
#endif
    }, BK_T);
  else {
    // "ros2p": the library's Rosenbrock sequence with a probe budget of 48 attempts: probe launch,
    // bin scan, scatter of the parked cells, resume launch in that order
    const int budget = 48;
    std::vector<double> wst(4 * (size_t)n, 0.0);
    std::vector<int> order(n, 0);
    std::vector<unsigned int> sched(2 + 2 * CHEM_SCHED_BINS, 0u);
    coll = emu::run_grid(grid, [&] {
      chem_k_ros2_persistent(n, ld, y.data(), lnA.data(), o, status.data(), counters.data(), &queue, ws.data(), 0,
                             budget, wst.data(), nullptr, sched.data());
    }, BK_T);
    emu::run_grid(1, [&] { chem_k_sched_scan(sched.data()); }, CHEM_SCHED_BINS);
    emu::run_grid((unsigned)((n + 255) / 256), [&] {
      chem_k_sched_scatter(n, status.data(), wst.data(), sched.data(), order.data());
    }, 256);
    queue = 0;
    coll += emu::run_grid(grid, [&] {
      chem_k_ros2_persistent(n, ld, y.data(), lnA.data(), o, status.data(), counters.data(), &queue, ws.data(), 0, 0,
                             wst.data(), order.data(), sched.data());
    }, BK_T);
  }
  fprintf(stderr, "collectives %lld\n", coll);
  FILE* f = fopen(argv[7], "wb");
  fwrite(y.data(), 8, y.size(), f);
  fwrite(status.data(), 4, ld, f);
  fwrite(counters.data(), 4, 3 * ld, f);
  fclose(f);
  return 0;
}
