// Host-side check of the library's one-time setup (ordinates, coarse ordinates, ConvFEM stencils),
// built with g++ and the address / undefined-behaviour sanitizers by tests/test_host_sanitizers.py.
// Prints every value so that the test can compare them with the oracle.
#include <cstdio>

#include "../../paper_2301_09991_amd/csrc/internal.h"

int main() {
  for (int na : {1, 2, 4}) {
    for (int faces : {8, 4}) {
      const ctf::Quadrature q = ctf::build_quadrature(na, faces);
      const ctf::Quadrature c = ctf::coarsen_quadrature(q);
      for (const ctf::Quadrature* x : {&q, &c}) {
        std::printf("Q %d %d %d %zu\n", na, faces, x == &q ? 0 : 1, x->w.size());
        for (size_t n = 0; n < x->w.size(); ++n)
          std::printf("%.17g %.17g %.17g\n", x->mu[n], x->nu[n], x->w[n]);
      }
    }
  }
  for (int p = 1; p <= ctf::kMaxP; ++p) {
    double m[2 * ctf::kMaxP + 1], d[2 * ctf::kMaxP + 1], k[2 * ctf::kMaxP + 1];
    ctf::convfem_stencils(p, m, d, k);
    std::printf("S %d\n", p);
    for (int t = 0; t < 2 * p + 1; ++t) std::printf("%.17g %.17g %.17g\n", m[t], d[t], k[t]);
  }
  return 0;
}
