// Host build of the generated per-lane mechanism functions (prelude + mechanism block of the
// register-resident form) to check mech_vjp against the oracle on the CPU: for each case reads
// y, u, d [NY] and writes J(y)^T u, the lnA contraction, and the value and dual parts of the
// same quantities at the dual state y + eps d.
#include <cmath>
#include <cstdio>
#include <vector>
using std::exp; using std::log; using std::fma; using std::fabs; using std::sqrt; using std::fmax; using std::fmin;
#define __device__
#define __forceinline__ inline
#define __noinline__
#define __restrict__
#include "mech_block.hip"

struct Acc {
  double a[NR];
  double& operator[](int j) { return a[j]; }
};

int main(int argc, char** argv) {
  if (argc < 4) return 2;
  const int energy = std::atoi(argv[1]);
  FILE* fi = std::fopen(argv[2], "rb");
  FILE* fo = std::fopen(argv[3], "wb");
  if (!fi || !fo) return 3;
  int ncase = 0;
  if (std::fread(&ncase, sizeof(int), 1, fi) != 1) return 4;
  std::vector<double> lnA(NR);
  if (std::fread(lnA.data(), sizeof(double), NR, fi) != (size_t)NR) return 4;
  for (int c = 0; c < ncase; ++c) {
    double y[NY], u[NY], d[NY];
    if (std::fread(y, sizeof(double), NY, fi) != (size_t)NY || std::fread(u, sizeof(double), NY, fi) != (size_t)NY ||
        std::fread(d, sizeof(double), NY, fi) != (size_t)NY)
      return 4;
    double v[NY];
    Acc g{};
    mech_vjp<double>(y, lnA.data(), energy, u, v, g, 0);
    ChemDual yd[NY], vd[NY];
    for (int k = 0; k < NY; ++k) yd[k] = ChemDual(y[k], d[k]);
    Acc g1{}, g2{};
    mech_vjp<ChemDual>(yd, lnA.data(), energy, u, vd, g1, 1);
    mech_vjp<ChemDual>(yd, lnA.data(), energy, u, vd, g2, 2);
    double vv[NY], vdd[NY];
    for (int k = 0; k < NY; ++k) {
      vv[k] = vd[k].v;
      vdd[k] = vd[k].d;
    }
    std::fwrite(v, sizeof(double), NY, fo);
    std::fwrite(g.a, sizeof(double), NR, fo);
    std::fwrite(vv, sizeof(double), NY, fo);
    std::fwrite(vdd, sizeof(double), NY, fo);
    std::fwrite(g1.a, sizeof(double), NR, fo);
    std::fwrite(g2.a, sizeof(double), NR, fo);
  }
  std::fclose(fo);
  return 0;
}
