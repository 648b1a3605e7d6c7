// The thread-pool part of libqtn's host code (exact costs of many cut sets,
// qtn_cost_exact with several threads) under ThreadSanitizer: a standalone
// program, so that the sanitizer runtime is the executable's own.  Exits 0
// when the results of 1 and 4 threads agree.
#include <cstdint>
#include <cstdio>
#include <vector>

#include "qtn.h"

int main() {
  // 40 vertices of degree 3: a ring plus the 20 diameters
  const uint32_t n = 40, p = 2, k = 4, sets = 64;
  std::vector<uint32_t> edges;
  for (uint32_t i = 0; i < n; ++i) {
    edges.push_back(i);
    edges.push_back((i + 1) % n);
  }
  for (uint32_t i = 0; i < n / 2; ++i) {
    edges.push_back(i);
    edges.push_back(i + n / 2);
  }
  const qtn_graph g{n, (uint32_t)edges.size() / 2, edges.data()};
  // distinct variables per set from a linear congruential sequence
  const uint32_t nvars = n * p;
  std::vector<uint32_t> cut;
  uint64_t x = 12345;
  for (uint32_t s = 0; s < sets; ++s) {
    std::vector<uint32_t> row;
    while (row.size() < k) {
      x = x * 6364136223846793005ull + 1442695040888963407ull;
      const uint32_t v = (uint32_t)(x >> 33) % nvars;
      bool dup = false;
      for (uint32_t u : row) dup |= u == v;
      if (!dup) row.push_back(v);
    }
    cut.insert(cut.end(), row.begin(), row.end());
  }
  std::vector<int32_t> w1(sets), w4(sets);
  std::vector<double> c1(sets), c4(sets);
  if (qtn_cost_exact(&g, p, cut.data(), sets, k, w1.data(), c1.data(), 1) != QTN_OK) return 2;
  if (qtn_cost_exact(&g, p, cut.data(), sets, k, w4.data(), c4.data(), 4) != QTN_OK) return 3;
  for (uint32_t s = 0; s < sets; ++s)
    if (w1[s] != w4[s] || c1[s] != c4[s]) return 4;
  std::printf("done\n");
  return 0;
}
