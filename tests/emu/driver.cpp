// Runs one persistent integration kernel of the generated one-wavefront-per-cell source on the
// fiber emulation of a 64-lane wavefront (fiber.hpp).
// Usage: driver be|ros2 n ld dt n_steps in.bin out.bin [grid]
//   in.bin: state [NY][ld] then ln A [NR] (float64); out.bin: state, status [ld], counters [3][ld].
//   grid: workgroups launched (they run one after another and share the work queue).
#include "fiber.hpp"
#include <vector>
#include "src.hip"
int main(int argc, char** argv) {
  if (argc < 8) return 2;
  const char* which = argv[1];
  const long long n = atoll(argv[2]), ld = atoll(argv[3]);
  const double dt = atof(argv[4]);
  const int n_steps = atoi(argv[5]);
  const unsigned grid = argc > 8 ? (unsigned)atoi(argv[8]) : 2u;
  FILE* f = fopen(argv[6], "rb");
  if (!f) return 3;
  std::vector<double> y((size_t)NY * ld), lnA(NR);
  if (fread(y.data(), 8, y.size(), f) != y.size() || fread(lnA.data(), 8, NR, f) != (size_t)NR) return 4;
  fclose(f);
  std::vector<int> status(ld, -7), counters(3 * ld, 0);
  unsigned long long queue = 0;
  ChemOpts o{};
  o.dt = dt; o.rtol = 1e-6; o.atol = 1e-10; o.h_min = 1e-20; o.newton_rtol = 1e-10; o.newton_atol_T = 1e-8;
  o.newton_atol_Y = 1e-14; o.n_steps = n_steps; o.max_steps = 100000; o.newton_max = 10;
  o.halving_max_depth = 8; o.energy = 0; o.ckpt_every = 1;
  long long coll;
  if (!strcmp(which, "be"))
    coll = emu::run_grid(grid, [&] {
      chem_k_be_persistent(n, ld, y.data(), lnA.data(), o, status.data(), counters.data(), &queue, nullptr, 0,
                           nullptr, nullptr);
    });
  else
    coll = emu::run_grid(grid, [&] {
      chem_k_ros2_persistent(n, ld, y.data(), lnA.data(), o, status.data(), counters.data(), &queue, nullptr, 0, 0,
                             nullptr, nullptr, nullptr);
    });
  fprintf(stderr, "collectives %lld\n", coll);
  f = fopen(argv[7], "wb");
  fwrite(y.data(), 8, y.size(), f);
  fwrite(status.data(), 4, ld, f);
  fwrite(counters.data(), 4, 3 * ld, f);
  fclose(f);
  return 0;
}
