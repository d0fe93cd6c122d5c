/* Test driver for the C oracle on its own, built with the address and
 * undefined-behaviour sanitizers by tests/test_sanitizers.py: every mode of
 * orc_barcode (with and without clearing) on one distance matrix must give
 * the same pairs, and the other entry points must run clean on it.
 *
 *   oracle_driver <matrix file> <max_dim> <threshold>
 *
 * The matrix file holds n (int32) and the n x n float32 distance matrix.
 * Prints the number of pairs and exits 0 if everything agrees. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "vr_oracle.h"

static int same(const orc_result* a, const orc_result* b) {
  const int64_t n = orc_result_count(a);
  if (n != orc_result_count(b)) return 0;
  return n == 0 || memcmp(orc_result_pairs(a), orc_result_pairs(b), (size_t)n * sizeof(orc_pair)) == 0;
}

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  FILE* f = fopen(argv[1], "rb");
  if (!f) return 2;
  int32_t n = 0;
  if (fread(&n, 4, 1, f) != 1 || n < 1 || n > 200) return 2;
  float* D = malloc((size_t)n * n * sizeof(float));
  if (!D || fread(D, 4, (size_t)n * n, f) != (size_t)n * n) return 2;
  fclose(f);
  const int max_dim = atoi(argv[2]);
  const float thr = (float)atof(argv[3]);

  orc_result* ref = NULL;
  if (orc_barcode(D, n, max_dim, thr, ORC_M1_BOUNDARY, 0, &ref) != 0) return 3;
  const int modes[3] = {ORC_M1_COBOUNDARY, ORC_M2_STREAMED, ORC_M3_REDUCTION_MATRIX};
  for (int k = 0; k < 3; ++k)
    for (uint32_t fl = 0; fl <= ORC_FLAG_NO_CLEARING; fl += ORC_FLAG_NO_CLEARING) {
      orc_result* r = NULL;
      if (orc_barcode(D, n, max_dim, thr, modes[k], fl, &r) != 0) return 3;
      if (!same(ref, r)) {
        fprintf(stderr, "mode %d flags %u differs\n", modes[k], fl);
        return 1;
      }
      orc_result_free(r);
    }

  /* H0, apparent pairs, diameter edges and the gradient on the same input */
  orc_pair* h0 = malloc((size_t)2 * n * sizeof(orc_pair));
  int64_t nh0 = 0;
  if (!h0 || orc_h0_kruskal(D, n, thr, 0, h0, 2 * n, &nh0) != 0) return 3;
  uint64_t* s = malloc(200000 * sizeof(uint64_t));
  uint64_t* t = malloc(200000 * sizeof(uint64_t));
  int64_t na = 0;
  if (!s || !t || orc_apparent_pairs(D, n, 1, thr, 0, s, t, 200000, &na) != 0) return 3;
  for (int64_t i = 0; i < na && i < 50; ++i) {
    uint64_t tt = 0;
    if (orc_is_apparent(D, n, 1, s[i], thr, 0, &tt) != 1 || tt != t[i]) return 1;
    int32_t u = 0, v = 0;
    if (orc_diameter_edge(D, n, 2, t[i], &u, &v) != 0) return 3;
  }
  const int64_t np = orc_result_count(ref);
  float* gb = calloc((size_t)np + 1, sizeof(float));
  float* gd = calloc((size_t)np + 1, sizeof(float));
  double* gX = malloc((size_t)n * 3 * sizeof(double));
  float* X = malloc((size_t)n * 3 * sizeof(float));
  for (int i = 0; i < 3 * n; ++i) X[i] = (float)((i * 37) % 101) / 101.0f;
  float* D2 = malloc((size_t)n * n * sizeof(float));
  if (!gb || !gd || !gX || !X || !D2 || orc_pdist(X, n, 3, D2) != 0) return 3;
  for (int64_t i = 0; i < np; ++i) gd[i] = 1.0f;
  if (orc_gradient(X, n, 3, D2, orc_result_pairs(ref), np, gb, gd, gX) != 0) return 3;

  printf("%lld pairs\n", (long long)np);
  orc_result_free(ref);
  free(D);
  free(D2);
  free(X);
  free(gX);
  free(gb);
  free(gd);
  free(s);
  free(t);
  free(h0);
  return 0;
}
