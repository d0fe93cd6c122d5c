// Test driver for the host part of the explicit-matrix path
// (reduce_explicit_columns) without a GPU: the scan's outputs are computed
// here from their definitions (leftmost 1 of every row; a column whose
// lowest 1 is its row's leftmost 1 is fixed; with clearing, the column its
// row names is zero; a column holding some row's leftmost 1 is a
// destroyer), then, with compression, the matrix is compressed
// (compress_explicit), the unstable columns are reduced on the given number
// of threads and every low(R_j) is printed, one per line; the compression's
// additions and removed entries go to stderr.
//
//   explicit_reduce_driver <matrix file> <threads> <always_wide> <clearing> [compression]
//
// The matrix file holds n (int64), then n + 1 column offsets and the rows
// (int64 each).
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "reduce.h"

int main(int argc, char** argv) {
  if (argc != 5 && argc != 6) {
    fprintf(stderr, "usage: %s matrix threads always_wide clearing [compression]\n", argv[0]);
    return 2;
  }
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t n = 0;
  if (fread(&n, 8, 1, f) != 1 || n < 0) return 2;
  std::vector<int64_t> ptr((size_t)n + 1);
  if (fread(ptr.data(), 8, ptr.size(), f) != ptr.size()) return 2;
  std::vector<int64_t> rows((size_t)ptr[(size_t)n]);
  if (!rows.empty() && fread(rows.data(), 8, rows.size(), f) != rows.size()) return 2;
  fclose(f);
  const int threads = atoi(argv[2]);
  const bool wide = atoi(argv[3]) != 0, clearing = atoi(argv[4]) != 0;
  const bool compression = argc == 6 && atoi(argv[5]) != 0;

  std::vector<int64_t> left((size_t)n, n);
  for (int64_t j = 0; j < n; ++j)
    for (int64_t q = ptr[(size_t)j]; q < ptr[(size_t)j + 1]; ++q)
      if (left[(size_t)rows[(size_t)q]] > j) left[(size_t)rows[(size_t)q]] = j;
  std::vector<int32_t> lookup((size_t)n, -1);
  std::vector<char> stable((size_t)n, 0);
  for (int64_t j = 0; j < n; ++j) {
    if (ptr[(size_t)j] == ptr[(size_t)j + 1]) {
      stable[(size_t)j] = 1;
      continue;
    }
    const int64_t r = rows[(size_t)ptr[(size_t)j + 1] - 1];
    if (left[(size_t)r] == j) {
      lookup[(size_t)r] = (int32_t)j;
      stable[(size_t)j] = 1;
      if (clearing) stable[(size_t)r] = 1;
    }
  }
  std::vector<int64_t> unstable;
  for (int64_t j = 0; j < n; ++j)
    if (!stable[(size_t)j]) unstable.push_back(j);
  const int64_t* rptr = ptr.data();
  const int64_t* rrows = rows.data();
  std::vector<int64_t> cptr, crows;
  if (compression) {
    std::vector<uint8_t> destroyer((size_t)n, 0);
    for (int64_t r = 0; r < n; ++r)
      if (left[(size_t)r] < n) destroyer[(size_t)left[(size_t)r]] = 1;
    int64_t cadds = 0, dropped = 0;
    if (!vrph::compress_explicit(n, ptr.data(), rows.data(), lookup.data(), destroyer.data(),
                                 unstable.data(), (int64_t)unstable.size(), threads, cptr, crows,
                                 &cadds, &dropped))
      return 4;
    fprintf(stderr, "compression additions %lld removed %lld\n", (long long)cadds,
            (long long)dropped);
    rptr = cptr.data();
    rrows = crows.data();
  }
  std::vector<int64_t> low((size_t)n);
  int64_t adds = 0;
  if (!vrph::reduce_explicit_columns(n, rptr, rrows, lookup.data(), unstable.data(),
                                     (int64_t)unstable.size(), threads, low.data(), &adds, wide))
    return 3;
  fprintf(stderr, "additions %lld\n", (long long)adds);
  for (int64_t j = 0; j < n; ++j) printf("%lld\n", (long long)low[(size_t)j]);
  return 0;
}
