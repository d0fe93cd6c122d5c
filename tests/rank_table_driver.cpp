// Test driver for RankTable::build_from_edges (no GPU): for each weight
// matrix given, in order, one table is built from the matrix (build) and
// one from the finite edges of its lower triangle sorted by weight
// (build_from_edges, kept across the matrices, so that every build after
// the first of a size resets only what the previous one wrote). The two
// must agree entry for entry (ranks, rank -> weight table, neighbour
// bitmaps, the sparse flag). diameter_edge on ranks alone (no weights
// attached) is also checked against diameter_edge on the weights for
// random simplices of dimensions 1-3.
//
//   rank_table_driver <matrix file>...
//
// Each file holds n (int32) and the n x n weights as float bits (uint32,
// kInf = 0xFFFFFFFF beyond the threshold and on the diagonal). Prints "ok" and
// exits 0, or prints the first difference and exits 1.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <random>
#include <vector>

#include "reduce.h"

using namespace vrph;

static std::vector<uint64_t> binomials(int n, int kmax) {
  std::vector<uint64_t> B((size_t)(kmax + 1) * (n + 1), 0);
  for (int k = 0; k <= kmax; ++k)
    for (int v = 0; v <= n; ++v) {
      if (k > v) continue;
      unsigned __int128 c = 1;
      for (int i = 0; i < k; ++i) c = c * (unsigned)(v - i) / (unsigned)(i + 1);
      B[(size_t)k * (n + 1) + v] = (uint64_t)c;
    }
  return B;
}

int main(int argc, char** argv) {
  RankTable inc;  // built from edge lists, across all files
  std::mt19937_64 rng(7);
  for (int f = 1; f < argc; ++f) {
    FILE* fp = fopen(argv[f], "rb");
    if (!fp) return 2;
    int32_t n = 0;
    if (fread(&n, 4, 1, fp) != 1) return 2;
    std::vector<uint32_t> W((size_t)n * n);
    if (fread(W.data(), 4, W.size(), fp) != W.size()) return 2;
    fclose(fp);
    RankTable ref;
    ref.build(n, W.data());
    std::vector<Column> e;
    for (int a = 1; a < n; ++a)
      for (int b = 0; b < a; ++b)
        if (W[(size_t)a * n + b] != kInf)
          e.push_back(Column{W[(size_t)a * n + b], 0u, ((uint64_t)a << 32) | (uint32_t)b});
    std::stable_sort(e.begin(), e.end(), [](const Column& x, const Column& y) { return x.key_hi < y.key_hi; });
    inc.build_from_edges(n, e.data(), e.size());
    if (inc.Wr != ref.Wr) { printf("file %d: Wr differs\n", f); return 1; }
    if (inc.bits != ref.bits) { printf("file %d: bits differ\n", f); return 1; }
    if (inc.nbw != ref.nbw || inc.nb != ref.nb) { printf("file %d: neighbour bitmaps differ\n", f); return 1; }
    if (inc.sparse != ref.sparse) { printf("file %d: sparse flag differs\n", f); return 1; }
    // diameter edges from ranks alone
    std::vector<uint64_t> B = binomials(n, 5);
    HostComplex Hw, Hr;
    Hw.n = Hr.n = n;
    Hw.binom = Hr.binom = B.data();
    Hw.kmax = Hr.kmax = 5;
    Hw.W = W.data();
    ref.attach(Hw);
    inc.attach(Hr);  // Hr.W stays null
    for (int d = 1; d <= 3 && d < n; ++d) {
      const uint64_t cnt = B[(size_t)(d + 1) * (n + 1) + n];
      for (int t = 0; t < 2000; ++t) {
        const uint64_t c = rng() % cnt;
        int32_t u1 = -1, w1 = -1, u2 = -1, w2 = -1;
        diameter_edge(Hw, c, d, &u1, &w1);
        diameter_edge(Hr, c, d, &u2, &w2);
        if (u1 != u2 || w1 != w2) {
          printf("file %d: diameter edge of simplex %llu (dim %d) differs\n", f, (unsigned long long)c, d);
          return 1;
        }
      }
    }
  }
  printf("ok\n");
  return 0;
}
