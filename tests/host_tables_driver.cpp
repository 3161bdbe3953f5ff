// Host-only driver for the sanitizer test: exercises the real-Gaunt table, the channel list
// and the Gauss rules of host_tables.cpp, and checks a few exact properties.
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "wefq_host.h"

int main() {
  int bad = 0;
  for (int L = 0; L <= 8; ++L) {
    std::vector<wefq::Channel> ch = wefq::enumerate_channels(L);
    std::vector<wefq::CooRow> rows = wefq::build_coo(L);
    for (const wefq::CooRow& r : rows) {
      const int NQ = (L + 1) * (L + 1);
      if (r.q1 < 0 || r.q1 >= NQ || r.q2 < 0 || r.q2 >= NQ || r.q3 < 0 || r.q3 >= NQ) ++bad;
      if (r.c < 0 || r.c >= (int)ch.size()) ++bad;
      if (!std::isfinite(r.g)) ++bad;
    }
    if (L == 4 && rows.size() != 1158) ++bad;          // Table 6 count at L = 4
  }
  // real Gaunt symmetry in its three arguments
  for (int l1 = 0; l1 <= 3; ++l1)
    for (int l2 = 0; l2 <= 3; ++l2)
      for (int l3 = 0; l3 <= 3; ++l3)
        for (int m1 = -l1; m1 <= l1; ++m1)
          for (int m2 = -l2; m2 <= l2; ++m2)
            for (int m3 = -l3; m3 <= l3; ++m3) {
              const double a = wefq::real_gaunt(l1, m1, l2, m2, l3, m3);
              const double b = wefq::real_gaunt(l3, m3, l1, m1, l2, m2);
              if (std::fabs(a - b) > 1e-13) ++bad;
            }
  // Gauss-Legendre weights sum to 2; Gauss-Laguerre (alpha = 0) weights sum to 1
  for (int n = 1; n <= 40; ++n) {
    std::vector<double> x, w;
    wefq::gauss_rule(0, n, 0.0, x, w);
    double s = 0.0;
    for (double v : w) s += v;
    if (std::fabs(s - 2.0) > 1e-12) ++bad;
    wefq::gauss_rule(1, n, 0.0, x, w);
    s = 0.0;
    for (double v : w) s += v;
    if (std::fabs(s - 1.0) > 1e-12) ++bad;
  }
  // launch chunking: the launches of a batch cover every cell once and each holds at most
  // 2^32 - 1 threads, for the tile shapes of the apply kernels and the naive FP64 kernel
  const int64_t big = (int64_t)1 << 36;
  for (int64_t tb : {16, 8, 4, 2, 64})
    for (int64_t block : {256, 512})
      for (int64_t per : {1, 4, 1229})
        for (int64_t B : {(int64_t)1, (int64_t)12345, big, big + 7}) {
          const int64_t mc = wefq::max_cells_per_launch(tb, block, per);
          if (mc <= 0) { ++bad; continue; }
          int64_t covered = 0;
          for (int64_t c0 = 0; c0 < B; c0 += mc) {
            const int64_t nc = B - c0 < mc ? B - c0 : mc;
            const int64_t threads = (nc + tb - 1) / tb * per * block;
            if (threads > wefq::max_launch_threads()) ++bad;
            covered += nc;
          }
          if (covered != B) ++bad;
        }
  std::printf("host tables: %d failures\n", bad);
  return bad != 0;
}
