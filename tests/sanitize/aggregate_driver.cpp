// Drives rn_aggregate_host on generated strength graphs and malformed input,
// for a build with AddressSanitizer and UndefinedBehaviorSanitizer
// (tests/test_sanitizers.py).  Exit status 0 when every case behaves.
#include <cstdio>
#include <vector>

#include "rnamg.h"

int main() {
  for (int nx : {1, 2, 9, 40}) {
    const int nn = nx * nx;
    std::vector<int32_t> Sp(nn + 1), Sj;
    for (int I = 0; I < nn; ++I) {
      const int x = I % nx, y = I / nx;
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx)
          if (x + dx >= 0 && x + dx < nx && y + dy >= 0 && y + dy < nx) Sj.push_back(I + dy * nx + dx);
      Sp[I + 1] = (int32_t)Sj.size();
    }
    std::vector<int32_t> agg(nn), roots(nn);
    int32_t na = 0;
    if (rn_aggregate_host(nn, Sp.data(), Sj.data(), agg.data(), roots.data(), &na) != RN_OK) return 1;
    for (int I = 0; I < nn; ++I)
      if (agg[I] < 0 || agg[I] >= na) return 2;
    for (int a = 0; a < na; ++a)
      if (agg[roots[a]] != a) return 3;
  }
  // malformed graphs are refused without reading out of bounds
  std::vector<int32_t> Sp = {0, 2, 1}, Sj = {0, 5}, agg(2), roots(2);
  int32_t na = 0;
  if (rn_aggregate_host(2, Sp.data(), Sj.data(), agg.data(), roots.data(), &na) != RN_EINVAL) return 4;
  Sp = {0, 1, 2};
  Sj = {0, 7};
  if (rn_aggregate_host(2, Sp.data(), Sj.data(), agg.data(), roots.data(), &na) != RN_EINVAL) return 5;
  if (rn_aggregate_host(0, nullptr, nullptr, nullptr, nullptr, &na) != RN_OK || na != 0) return 6;
  std::printf("aggregate driver ok\n");
  return 0;
}
