/*
 * vr_oracle.h — plain, slow CPU reference for Vietoris–Rips persistence pairs.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the product path (the HIP library and
 * its Python binding) may include, link or call this code. Only the tests, the
 * smoke check and the CPU-baseline leg of the benchmark use it, to check the
 * GPU path against a definition a reader can verify by eye against the paper
 * (Zhang, "Computing and Learning on Combinatorial Data", Ch. 3-5).
 *
 * What it computes (the plain definition, Alg. 11 with Alg. 2):
 *   Let S be the simplex-wise refinement (Sec. 5.1.4: diameter ascending, then
 *   dimension ascending, then combinatorial index descending) of the
 *   Vietoris–Rips complex Rips_tau(D) (Eq. 5.3, diam <= tau) restricted to
 *   simplices of dimension <= max_dim + 1. The persistence pairs are the
 *   pivots (low(j), j) of the standard reduction of the Z/2 boundary matrix of
 *   S (Alg. 2). Pivots do not depend on the reduction variant (Sec. 4.2), so
 *   all four modes must agree:
 *     ORC_M1_BOUNDARY   explicit boundary matrix, Alg. 2.
 *     ORC_M1_COBOUNDARY explicit anti-transposed (coboundary) matrix per
 *                       dimension (Def. 4.3.4, Prop. 4.3.5), Alg. 2, clearing
 *                       (Lemma 4.2.2) with the previous dimension's pairs.
 *     ORC_M2_STREAMED   the same coboundary matrix, each column generated only
 *                       when it is reduced, oblivious reduction (Alg. 12,
 *                       equivalent by Lemma 5.2.10). Memory = pivots only.
 *     ORC_M3_REDUCTION_MATRIX
 *                       the same coboundary matrix, streamed, reduced with the
 *                       reduction-matrix technique (Sec. 5.2.9): column j adds
 *                       R_k = D_k + sum_{i in V_k} D_i, so its low only moves
 *                       up; V_j is kept. The working column is a binary heap
 *                       in which equal row keys cancel in pairs.
 *
 * Readings where the paper is silent:
 *   - tau_eff = min(tau, R), R = min_i max_j D_ij the enclosing radius
 *     (Sec. 5.2.12, Prop. 5.2.13), unless ORC_FLAG_NO_ENCLOSING is given.
 *   - the threshold is inclusive (Eq. 5.3).
 *   - vertex v has combinatorial index v; a larger index is older (Sec. 5.1.4).
 *   - essential classes: dimension <= max_dim simplices whose reduced column
 *     is zero and which are not the death of a lower-dimensional pair; they are
 *     reported with death index UINT64_MAX and death diameter +inf.
 *   - distances (orc_pdist): D_ij = float32( sqrt_f64( sum_k (x_ik - x_jk)^2 ) )
 *     with the differences, squares and the left-to-right sum in IEEE binary64,
 *     a correctly rounded square root, and one final round-to-nearest to float32.
 *
 * Errors are returned as negative status codes; nothing aborts.
 */
#ifndef VR_ORACLE_H
#define VR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EOVERFLOW (-3)

#define ORC_FLAG_NO_ENCLOSING 1u /* use tau as given, no enclosing-radius cut */
#define ORC_FLAG_NO_CLEARING 2u  /* coboundary modes: reduce cleared columns too */

enum { ORC_M1_BOUNDARY = 0, ORC_M1_COBOUNDARY = 1, ORC_M2_STREAMED = 2, ORC_M3_REDUCTION_MATRIX = 3 };

/* One persistence pair. birth/death are combinatorial indices (Eq. 5.6) of the
 * birth simplex (dimension dim) and death simplex (dimension dim+1). */
typedef struct {
  int32_t dim;
  int32_t essential; /* 1: death == UINT64_MAX, death_diam == +inf */
  uint64_t birth;
  uint64_t death;
  float birth_diam;
  float death_diam;
} orc_pair;

typedef struct orc_result orc_result;

/* Pairwise distances of n points in R^m (row-major X), reading above. */
int orc_pdist(const float* X, int64_t n, int32_t m, float* D);

/* R = min_i max_j D_ij (Sec. 5.2.12). */
float orc_enclosing_radius(const float* D, int64_t n);

/* C(v, k) by the Pascal recurrence in 128-bit integers; UINT64_MAX if it does
 * not fit in 64 bits or the arguments are out of range. */
uint64_t orc_binomial(int64_t v, int32_t k);

/* Persistence pairs of dimensions 0..max_dim (see top of file), in canonical
 * order: by dimension, then birth index, then death index. */
int orc_barcode(const float* D, int64_t n, int32_t max_dim, float threshold,
                int32_t mode, uint32_t flags, orc_result** out);
int64_t orc_result_count(const orc_result* r);
const orc_pair* orc_result_pairs(const orc_result* r);
/* Number of columns of each dimension's coboundary matrix that were reduced
 * (after threshold and clearing); zero for the boundary mode. */
int64_t orc_result_columns(const orc_result* r, int32_t dim);
void orc_result_free(orc_result* r);

/* Alg. 2 on an explicit Z/2 matrix given column-wise (col_ptr[ncols+1] into
 * rows[], each column's row indices in any order, repeated rows cancel).
 * low_out[j] = lowest nonzero row of the reduced column j, or -1. */
int orc_reduce_explicit(int32_t ncols, const int64_t* col_ptr,
                        const int64_t* rows, int64_t* low_out);

/* Apparent pairs of dimension dim straight from Def. 5.3.4 on the explicit
 * coboundary matrix: entry (t, s) is the lowest entry of column s and all
 * entries to its left in row t are zero. Columns are all dim-simplices with
 * diam <= tau_eff (no clearing; Prop. 5.3.9 says clearing does not change the
 * set). Output sorted by s. *count receives the number found; at most cap
 * pairs are written. */
int orc_apparent_pairs(const float* D, int64_t n, int32_t dim, float threshold,
                       uint32_t flags, uint64_t* s_out, uint64_t* t_out,
                       int64_t cap, int64_t* count);

/* Def. 5.3.4 for one column s (dimension dim): enumerate every cofacet with
 * diam <= tau_eff, take the oldest; enumerate its facets, take the youngest.
 * Returns 1 and sets *t if (s, t) is apparent, 0 if not, <0 on error. */
int orc_is_apparent(const float* D, int64_t n, int32_t dim, uint64_t s,
                    float threshold, uint32_t flags, uint64_t* t);

/* H0 by Kruskal's algorithm with union-find (Sec. 5.2.5): edges in
 * simplex-wise order, each component represented by its oldest vertex (the
 * largest index); a merge kills the younger representative. Writes the finite
 * pairs then one essential pair per component, canonical order. */
int orc_h0_kruskal(const float* D, int64_t n, float threshold, uint32_t flags,
                   orc_pair* out, int64_t cap, int64_t* count);

/* The edge (u > v) realising the diameter of simplex (dim, cidx): among the
 * longest edges, the one with the largest edge index. */
int orc_diameter_edge(const float* D, int64_t n, int32_t dim, uint64_t cidx,
                      int32_t* u, int32_t* v);

/* Gradient of a loss on (birth, death) values w.r.t. the points, in binary64:
 * each pair's birth (dim >= 1) and finite death value is the length of its
 * diameter edge (u, v); d|x_u - x_v| / dx_u = (x_u - x_v) / |x_u - x_v|.
 * gX (n*m doubles) is overwritten. */
int orc_gradient(const float* X, int64_t n, int32_t m, const float* D,
                 const orc_pair* pairs, int64_t npairs, const float* g_birth,
                 const float* g_death, double* gX);

#ifdef __cplusplus
}
#endif
#endif
