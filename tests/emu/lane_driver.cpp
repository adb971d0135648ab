// Runs the register-resident form's Rosenbrock recording kernel and its discrete adjoint kernel
// (generated source, one cell per lane) on the fiber emulation (fiber.hpp), the whole sequence the
// library issues for a tape: initial states to checkpoint 0, recording forward run, adjoint sweep.
// The kernels run with one-lane workgroups (a partial wave): on the GPU a wave's lanes leave the
// per-cell loops at different times and the ballots inside run on the lanes still active, which
// the fiber emulation (all lanes of a wave at every collective) cannot follow; with one lane per
// wave every collective is uniform.  One workgroup pulls every cell from the queue.
// Usage:
//   lane_driver ros2adj n ld dt K in.bin out.bin [probe]
//     probe > 0: the recording run as the library issues it with a probe budget: probe launch (each
//     cell at most `probe` attempts), bin scan, scatter of the parked cells, resume launch
//     in.bin: state [NY][ld], ln A [NR], dL/dy_N [NY][ld]
//     out.bin: final state [NY][ld], status [ld], accepted steps [ld], dL/dy0 [NY][ld], dL/dlnA [NR]
// The test includes the generated source with two textual changes: the dynamic LDS declaration
// becomes a static array, and the cross-lane reduction of the ln A partials (64 lanes per wave)
// becomes a per-lane sum into the block's partials.
#include "fiber.hpp"
#include <cstdlib>
#include <vector>
#include "src.hip"

static bool read_all(FILE* f, double* p, size_t n) { return fread(p, 8, n, f) == n; }

int main(int argc, char** argv) {
  if (argc < 8 || strcmp(argv[1], "ros2adj") != 0) return 2;
  const long long n = atoll(argv[2]), ld = atoll(argv[3]);
  const double dt = atof(argv[4]);
  const int K = atoi(argv[5]);
  const int block = 1;
  if (n <= 0 || ld < n || K < 1) return 2;
  std::vector<double> y((size_t)NY * ld), lnA(NR), lamN((size_t)NY * ld);
  FILE* fi = fopen(argv[6], "rb");
  if (!fi || !read_all(fi, y.data(), y.size()) || !read_all(fi, lnA.data(), lnA.size()) ||
      !read_all(fi, lamN.data(), lamN.size()))
    return 4;
  fclose(fi);
  const int max_steps = 100000;
  ChemOpts o{};
  o.dt = dt; o.rtol = 1e-6; o.atol = 1e-10; o.h_min = 1e-20; o.newton_rtol = 1e-10; o.newton_atol_T = 1e-8;
  o.newton_atol_Y = 1e-14; o.n_steps = 0; o.max_steps = max_steps; o.newton_max = 10;
  o.halving_max_depth = 8; o.energy = 0; o.ckpt_every = K;
  // forward run with the tape: step sizes [cap][ld], accepted counts [ld]; checkpoint 0 = y0
  const int cap = 4096;
  std::vector<double> hs((size_t)cap * ld, 0.0);
  std::vector<int> status(ld, -7), counters(3 * ld, 0), tacc(ld, 0);
  std::vector<double> ck((size_t)(cap / K + 2) * NY * ld, 0.0);
  std::copy(y.begin(), y.end(), ck.begin());
  unsigned long long queue = 0;
  const int budget = argc > 8 ? atoi(argv[8]) : 0;
  std::vector<double> wst(4 * (size_t)n, 0.0);
  std::vector<int> order(n, 0);
  std::vector<unsigned int> sched(2 + 2 * CHEM_SCHED_BINS, 0u);
  emu::run_grid(1, [&] {
    chem_k_ros2_persistent_rec(n, ld, y.data(), lnA.data(), o, status.data(), counters.data(), &queue, nullptr, 0,
                               budget, budget > 0 ? wst.data() : nullptr, nullptr, budget > 0 ? sched.data() : nullptr,
                               hs.data(), tacc.data(), cap);
  }, block);
  if (budget > 0) {
    emu::run_grid(1, [&] { chem_k_sched_scan(sched.data()); }, CHEM_SCHED_BINS);
    emu::run_grid((unsigned)((n + 255) / 256), [&] {
      chem_k_sched_scatter(n, status.data(), wst.data(), sched.data(), order.data());
    }, 256);
    queue = 0;
    emu::run_grid(1, [&] {
      chem_k_ros2_persistent_rec(n, ld, y.data(), lnA.data(), o, status.data(), counters.data(), &queue, nullptr, 0,
                                 0, wst.data(), order.data(), sched.data(), hs.data(), tacc.data(), cap);
    }, block);
  }
  // adjoint: one block, cells strided over its lanes; segment records [K][SEG_W][seg_ld]
  const long long seg_ld = block;
  std::vector<double> seg((size_t)K * (4 * NY + NY * NY) * seg_ld, 0.0), dLdy0((size_t)NY * ld, 0.0),
      gpart(NR, 0.0);
  emu::run_grid(1, [&] {
    chem_k_ros2_adjoint(n, ld, lnA.data(), o, status.data(), tacc.data(), hs.data(), ck.data(), lamN.data(),
                        dLdy0.data(), gpart.data(), seg.data(), seg_ld);
  }, block);
  FILE* fo = fopen(argv[7], "wb");
  fwrite(y.data(), 8, y.size(), fo);
  fwrite(status.data(), 4, ld, fo);
  fwrite(tacc.data(), 4, ld, fo);
  fwrite(dLdy0.data(), 8, dLdy0.size(), fo);
  fwrite(gpart.data(), 8, gpart.size(), fo);
  fclose(fo);
  return 0;
}
