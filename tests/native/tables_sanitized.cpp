// Host-only driver for the basis-table builder (tables.cpp), built with g++ under
// AddressSanitizer and UndefinedBehaviorSanitizer by tests/test_host_sanitizers.py: every shape
// at P = 1..16 with Q = P + 1 and Q = P + 2 (the range the builder accepts), every table read in
// full, the 1-D rules at Q = 1..17, and the rejected inputs.  Any out-of-bounds access or
// undefined operation aborts the run; the exit status says whether the tables are finite.
#include <cmath>
#include <cstdio>
#include <vector>

#include "nir_internal.h"

int main() {
  using namespace nir;
  int bad = 0;
  double sum = 0.0;
  for (int shape = kHex; shape <= kPyr; ++shape)
    for (int P = 1; P <= 16; ++P)
      for (int Q = P + 1; Q <= P + 2 && Q <= 17; ++Q) {
        HostTables t;
        if (!build_tables(shape, P, Q, t)) {
          std::printf("build_tables(%d, %d, %d) failed\n", shape, P, Q);
          ++bad;
          continue;
        }
        for (int id = 0; id < NIR_TAB_COUNT; ++id) {
          int64_t count = -1;
          bool is_int = false;
          const void* p = host_table(t, id, &count, &is_int);
          if (!p || count < 0) continue;
          for (int64_t i = 0; i < count; ++i) {
            const double v = is_int ? double(static_cast<const int32_t*>(p)[i]) : static_cast<const double*>(p)[i];
            if (!std::isfinite(v)) {
              std::printf("non-finite entry: shape %d P %d Q %d table %d index %lld\n", shape, P, Q, id,
                          static_cast<long long>(i));
              ++bad;
              break;
            }
            sum += v;
          }
        }
      }
  for (int rule = 0; rule <= 1; ++rule)
    for (int alpha = 0; alpha <= 2; ++alpha)
      for (int Q = 1; Q <= 17; ++Q) {
        std::vector<double> z(Q), w(Q);
        if (!quadrature_1d(rule, alpha, Q, z.data(), w.data())) continue;
        for (int i = 0; i < Q; ++i) sum += z[i] + w[i];
      }
  HostTables t;
  if (build_tables(kHex, 0, 2, t) || build_tables(kPyr + 1, 3, 4, t) || build_tables(kTet, 3, 18, t)) ++bad;
  std::printf("tables checked: %d failures (checksum %.6e)\n", bad, sum);
  return bad == 0 ? 0 : 1;
}
