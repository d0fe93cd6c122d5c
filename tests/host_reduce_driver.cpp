// Test driver for the host reduction (reduce_dimension) on its own, without a
// GPU: the stages before it are done here on the host in the plainest way,
// and every pair of dimensions 1..max_dim is printed, so that a test can
// compare runs on different thread counts with each other and with the oracle.
//
//   host_reduce_driver <matrix file> <max_dim> <tau> <threads> <always_wide>
//
// The matrix file holds n (int32) and the n x n float32 distance matrix; tau
// is the effective threshold (the threshold already lowered to the
// enclosing radius). Output: one line "dim birth death birth_bits death_bits"
// per pair (death 2^64-1 and death_bits 2^32-1 for an essential class),
// apparent pairs after the reduced ones of each dimension.
//
// Stages: the weights W (float bits, kInf above tau and on the diagonal);
// H0 by Kruskal over the edges in filtration order, whose tree edges are the
// cleared columns of dimension 1; then per dimension d, every d-simplex of
// the complex that is not cleared is a column, an apparent pair (Def. 5.3.4:
// its oldest cofacet t has the same diameter and s is the youngest facet of
// t) or left for the reduction, in coboundary order (diameter descending,
// then index ascending). The deaths of dimension d (apparent cofacets and
// reduced pivots) are the cleared columns of dimension d + 1 (Alg. 17).
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <set>
#include <vector>

#include "reduce.h"

using namespace vrph;

int main(int argc, char** argv) {
  if (argc != 6) {
    fprintf(stderr, "usage: %s matrix max_dim tau threads always_wide\n", argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t n = 0;
  if (fread(&n, 4, 1, f) != 1 || n < 1 || n > 4096) return 2;
  std::vector<float> D((size_t)n * n);
  if (fread(D.data(), 4, D.size(), f) != D.size()) return 2;
  fclose(f);
  const int max_dim = atoi(argv[2]);
  const float tau = (float)atof(argv[3]);
  const int threads = atoi(argv[4]);
  const bool wide = atoi(argv[5]) != 0;
  if (max_dim < 1 || max_dim > 4) return 2;

  std::vector<uint32_t> W((size_t)n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      float x = D[(size_t)i * n + j];
      if (x == 0.0f) x = 0.0f;  // -0 as +0
      uint32_t b;
      memcpy(&b, &x, 4);
      W[(size_t)i * n + j] = (i != j && x <= tau) ? b : kInf;
    }
  const int kmax = max_dim + 2;
  std::vector<uint64_t> B((size_t)(kmax + 1) * (n + 1), 0);
  for (int k = 0; k <= kmax; ++k)
    for (int v = 0; v <= n; ++v) {
      if (k > v) continue;
      unsigned __int128 c = 1;
      for (int i = 0; i < k; ++i) c = c * (unsigned)(v - i) / (unsigned)(i + 1);
      B[(size_t)k * (n + 1) + v] = (uint64_t)c;
    }
  HostComplex H;
  H.n = n;
  H.W = W.data();
  H.binom = B.data();
  H.kmax = kmax;
  RankTable ranks;
  ranks.build(n, W.data());
  ranks.attach(H);
  auto w = [&](int a, int b) { return W[(size_t)a * n + b]; };

  // H0: Kruskal; the tree edges are cleared in dimension 1
  std::set<uint64_t> cleared;
  {
    std::vector<std::pair<uint64_t, uint64_t>> E;  // (weight, -index), index
    for (int a = 1; a < n; ++a)
      for (int b = 0; b < a; ++b)
        if (w(a, b) != kInf) {
          const uint64_t idx = H.C(a, 2) + (uint64_t)b;
          E.push_back({((uint64_t)w(a, b) << 32) | (0xFFFFFFFFull - idx), idx});
        }
    std::sort(E.begin(), E.end());
    std::vector<int> parent(n);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int x) {
      while (parent[x] != x) x = parent[x] = parent[parent[x]];
      return x;
    };
    for (auto& e : E) {
      int v[2];
      decode_simplex(H, e.second, 1, v);
      const int ra = find(v[0]), rb = find(v[1]);
      if (ra != rb) {
        parent[std::min(ra, rb)] = std::max(ra, rb);
        cleared.insert(e.second);
      }
    }
  }

  for (int d = 1; d <= max_dim; ++d) {
    std::vector<Column> cols;
    std::vector<PairRec> app;
    std::set<uint64_t> next_cleared;
    int v[8];
    for (uint64_t c = 0; c < H.C(n, d + 1); ++c) {
      decode_simplex(H, c, d, v);  // v[d] > ... > v[0]
      uint32_t dm = 0;
      for (int i = 1; i <= d; ++i)
        for (int j = 0; j < i; ++j) dm = std::max(dm, w(v[i], v[j]));
      if (dm == kInf || cleared.count(c)) continue;
      // oldest cofacet with the same diameter: the largest such x
      int x = -1;
      for (int y = n - 1; y >= 0 && x < 0; --y) {
        bool in = false;
        uint32_t m = 0;
        for (int i = 0; i <= d; ++i) {
          in |= v[i] == y;
          m = std::max(m, y == v[i] ? 0u : w(v[i], y));
        }
        if (!in && m <= dm) x = y;
      }
      bool apparent = x >= 0;
      // s is the youngest facet of t = s + {x}: no facet t - {u} with u > x
      // (a smaller index) keeps the diameter
      for (int u = 0; u <= d && apparent; ++u) {
        if (v[u] < x) continue;
        uint32_t m = 0;
        for (int i = 0; i <= d; ++i) {
          if (i == u) continue;
          m = std::max(m, w(v[i], x));
          for (int j = 0; j < i; ++j)
            if (j != u) m = std::max(m, w(v[i], v[j]));
        }
        if (m == dm) apparent = false;
      }
      if (apparent) {
        int t[9];
        int k = 0;
        for (int i = 0; i <= d; ++i) t[k++] = v[i];
        t[k++] = x;
        std::sort(t, t + k);
        uint64_t tidx = 0;
        for (int i = 0; i < k; ++i) tidx += H.C(t[i], i + 1);
        app.push_back(PairRec{c, tidx, dm, dm});
        next_cleared.insert(tidx);
      } else {
        cols.push_back(Column{~dm, 0u, c});
      }
    }
    std::sort(cols.begin(), cols.end(), [](const Column& a, const Column& b) {
      return a.key_hi != b.key_hi ? a.key_hi < b.key_hi : a.cidx < b.cidx;
    });
    std::vector<PairRec> pairs;
    std::vector<uint64_t> deaths;
    ReduceStats rs;
    reduce_dimension(H, d, cols.data(), (int64_t)cols.size(), threads, pairs, deaths, rs, wide);
    for (uint64_t t : deaths) next_cleared.insert(t);
    for (const PairRec& p : pairs)
      printf("%d %llu %llu %u %u\n", d, (unsigned long long)p.birth, (unsigned long long)p.death,
             p.bdiam, p.ddiam);
    for (const PairRec& p : app)
      printf("%d %llu %llu %u %u\n", d, (unsigned long long)p.birth, (unsigned long long)p.death,
             p.bdiam, p.ddiam);
    cleared.swap(next_cleared);
  }
  return 0;
}
