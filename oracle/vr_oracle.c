/*
 * vr_oracle.c — plain, slow CPU reference for Vietoris–Rips persistence pairs.
 *
 * TEST INFRASTRUCTURE ONLY (see vr_oracle.h): the product path never includes,
 * links or calls this file. It shares no code with the HIP library.
 *
 * Every function follows one passage of the paper (Zhang, "Computing and
 * Learning on Combinatorial Data"); the passage is named above the function.
 * There is deliberately no blocking, fusion or reordering beyond what the
 * cited definition or algorithm states. Build: gcc -std=c11 -O2
 * -ffp-contract=off (no fused multiply-add, so binary64 arithmetic is exactly
 * the IEEE operations written here).
 */
#include "vr_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------------ */
/* small containers                                                         */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint64_t cidx;
  float diam;
  int32_t dim;
} simplex;

typedef struct {
  simplex* a;
  int64_t len, cap;
} simplex_vec;

static int sv_push(simplex_vec* v, simplex s) {
  if (v->len == v->cap) {
    int64_t nc = v->cap ? 2 * v->cap : 64;
    simplex* na = (simplex*)realloc(v->a, (size_t)nc * sizeof(simplex));
    if (!na) return ORC_ENOMEM;
    v->a = na;
    v->cap = nc;
  }
  v->a[v->len++] = s;
  return ORC_OK;
}

typedef struct {
  orc_pair* a;
  int64_t len, cap;
} pair_vec;

static int pv_push(pair_vec* v, orc_pair p) {
  if (v->len == v->cap) {
    int64_t nc = v->cap ? 2 * v->cap : 64;
    orc_pair* na = (orc_pair*)realloc(v->a, (size_t)nc * sizeof(orc_pair));
    if (!na) return ORC_ENOMEM;
    v->a = na;
    v->cap = nc;
  }
  v->a[v->len++] = p;
  return ORC_OK;
}

/* A Z/2 column: a strictly increasing array of row keys. Addition of two
 * columns is the symmetric difference of the two sets. */
typedef struct {
  u128* a;
  int64_t len, cap;
} col;

static int col_reserve(col* c, int64_t n) {
  if (n <= c->cap) return ORC_OK;
  int64_t nc = c->cap ? c->cap : 16;
  while (nc < n) nc *= 2;
  u128* na = (u128*)realloc(c->a, (size_t)nc * sizeof(u128));
  if (!na) return ORC_ENOMEM;
  c->a = na;
  c->cap = nc;
  return ORC_OK;
}

/* dst <- dst + src over Z/2 (sorted symmetric difference), using tmp. */
static int col_add(col* dst, const col* src, col* tmp) {
  if (col_reserve(tmp, dst->len + src->len)) return ORC_ENOMEM;
  int64_t i = 0, j = 0, k = 0;
  while (i < dst->len && j < src->len) {
    if (dst->a[i] < src->a[j])
      tmp->a[k++] = dst->a[i++];
    else if (src->a[j] < dst->a[i])
      tmp->a[k++] = src->a[j++];
    else {
      i++;
      j++;
    } /* 1 + 1 = 0 */
  }
  while (i < dst->len) tmp->a[k++] = dst->a[i++];
  while (j < src->len) tmp->a[k++] = src->a[j++];
  tmp->len = k;
  col t = *dst;
  *dst = *tmp;
  *tmp = t;
  return ORC_OK;
}

static int cmp_u128(const void* x, const void* y) {
  u128 a = *(const u128*)x, b = *(const u128*)y;
  return (a > b) - (a < b);
}

/* u64 -> i64 map, open addressing with linear probing (key+1 stored so that
 * 0 marks an empty slot; keys are < 2^63 by the overflow check). */
typedef struct {
  uint64_t* k;
  int64_t* v;
  int64_t cap, len;
} map64;

static uint64_t mix64(uint64_t x) {
  x ^= x >> 33;
  x *= 0xff51afd7ed558ccdULL;
  x ^= x >> 33;
  x *= 0xc4ceb9fe1a85ec53ULL;
  x ^= x >> 33;
  return x;
}

static int map_init(map64* m, int64_t expect) {
  int64_t cap = 64;
  while (cap < 2 * expect + 16) cap *= 2;
  m->k = (uint64_t*)calloc((size_t)cap, sizeof(uint64_t));
  m->v = (int64_t*)malloc((size_t)cap * sizeof(int64_t));
  m->cap = cap;
  m->len = 0;
  return (m->k && m->v) ? ORC_OK : ORC_ENOMEM;
}

static void map_free(map64* m) {
  free(m->k);
  free(m->v);
  m->k = NULL;
  m->v = NULL;
}

static int map_grow(map64* m);

static int map_put(map64* m, uint64_t key, int64_t val) {
  if (2 * (m->len + 1) > m->cap && map_grow(m)) return ORC_ENOMEM;
  uint64_t mask = (uint64_t)m->cap - 1, h = mix64(key) & mask;
  while (m->k[h] != 0 && m->k[h] != key + 1) h = (h + 1) & mask;
  if (m->k[h] == 0) m->len++;
  m->k[h] = key + 1;
  m->v[h] = val;
  return ORC_OK;
}

static int map_get(const map64* m, uint64_t key, int64_t* val) {
  uint64_t mask = (uint64_t)m->cap - 1, h = mix64(key) & mask;
  while (m->k[h] != 0) {
    if (m->k[h] == key + 1) {
      *val = m->v[h];
      return 1;
    }
    h = (h + 1) & mask;
  }
  return 0;
}

static int map_grow(map64* m) {
  map64 nm;
  if (map_init(&nm, m->cap)) return ORC_ENOMEM;
  for (int64_t i = 0; i < m->cap; i++)
    if (m->k[i]) map_put(&nm, m->k[i] - 1, m->v[i]);
  map_free(m);
  *m = nm;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Binomial coefficients and the combinatorial number system (Eq. 5.6)      */
/* ------------------------------------------------------------------------ */

#define BINOM_SAT (((u128)1) << 64) /* "does not fit in 64 bits" */

/* Pascal's rule C(v,k) = C(v-1,k-1) + C(v-1,k), saturating at 2^64. */
static u128* binom_table(int64_t n, int32_t kmax) {
  u128* t = (u128*)calloc((size_t)(n + 1) * (size_t)(kmax + 1), sizeof(u128));
  if (!t) return NULL;
  for (int64_t v = 0; v <= n; v++) {
    t[v * (kmax + 1) + 0] = 1;
    for (int32_t k = 1; k <= kmax; k++) {
      u128 x = (v == 0) ? 0 : t[(v - 1) * (kmax + 1) + (k - 1)] + t[(v - 1) * (kmax + 1) + k];
      t[v * (kmax + 1) + k] = x > BINOM_SAT ? BINOM_SAT : x;
    }
  }
  return t;
}

uint64_t orc_binomial(int64_t v, int32_t k) {
  if (v < 0 || k < 0) return UINT64_MAX;
  if (k > v) return 0;
  u128* t = binom_table(v, k);
  if (!t) return UINT64_MAX;
  u128 x = t[v * (k + 1) + k];
  free(t);
  return x >= BINOM_SAT ? UINT64_MAX : (uint64_t)x;
}

typedef struct {
  const float* D;
  int64_t n;
  float tau;      /* tau_eff */
  int32_t kmax;   /* largest number of vertices of any simplex considered */
  u128* binom;    /* (n+1) x (kmax+1) */
} ctx;

static uint64_t C(const ctx* c, int64_t v, int32_t k) {
  if (k > v) return 0;
  return (uint64_t)c->binom[v * (c->kmax + 1) + k];
}

/* Eq. 5.6 with vertices a[0] < a[1] < ... < a[q]: cidx = sum_i C(a[i], i+1). */
static uint64_t cidx_of(const ctx* c, const int32_t* a, int32_t q) {
  uint64_t s = 0;
  for (int32_t i = 0; i <= q; i++) s += C(c, a[i], i + 1);
  return s;
}

/* Inverse of Eq. 5.6: for position i from the top down, the vertex is the
 * largest v with C(v, i+1) <= remaining index. */
static void decode(const ctx* c, uint64_t cidx, int32_t q, int32_t* a) {
  int64_t v = c->n - 1;
  for (int32_t i = q; i >= 0; i--) {
    while (C(c, v, i + 1) > cidx) v--;
    a[i] = (int32_t)v;
    cidx -= C(c, v, i + 1);
    v--;
  }
}

static float dist(const ctx* c, int32_t i, int32_t j) { return c->D[(int64_t)i * c->n + j]; }

/* diam(s) = largest pairwise distance (Eq. 5.3); 0 for a vertex. */
static float diam_of(const ctx* c, const int32_t* a, int32_t q) {
  float d = 0.0f;
  for (int32_t i = 0; i <= q; i++)
    for (int32_t j = 0; j < i; j++)
      if (dist(c, a[i], a[j]) > d) d = dist(c, a[i], a[j]);
  return d;
}

/* ------------------------------------------------------------------------ */
/* Distances, enclosing radius, validation                                  */
/* ------------------------------------------------------------------------ */

int orc_pdist(const float* X, int64_t n, int32_t m, float* D) {
  if (!X || !D || n < 0 || m < 1) return ORC_EINVAL;
  for (int64_t i = 0; i < n; i++) {
    D[i * n + i] = 0.0f;
    for (int64_t j = 0; j < i; j++) {
      double s = 0.0;
      for (int32_t k = 0; k < m; k++) {
        double d = (double)X[i * m + k] - (double)X[j * m + k];
        double sq = d * d;
        s = s + sq;
      }
      float r = (float)sqrt(s);
      D[i * n + j] = r;
      D[j * n + i] = r;
    }
  }
  return ORC_OK;
}

/* Sec. 5.2.12: R = min over x of max over y of d(x, y). */
float orc_enclosing_radius(const float* D, int64_t n) {
  float R = INFINITY;
  for (int64_t i = 0; i < n; i++) {
    float mx = 0.0f;
    for (int64_t j = 0; j < n; j++)
      if (D[i * n + j] > mx) mx = D[i * n + j];
    if (mx < R) R = mx;
  }
  return R;
}

/* Def. 5.1.1 without the triangle inequality (Sec. 5.6.6 allows inputs that
 * violate it): finite, non-negative, symmetric, zero diagonal. */
static int validate(const float* D, int64_t n) {
  if (!D || n < 1) return ORC_EINVAL;
  for (int64_t i = 0; i < n; i++) {
    if (D[i * n + i] != 0.0f) return ORC_EINVAL;
    for (int64_t j = 0; j < n; j++) {
      float x = D[i * n + j];
      if (!isfinite(x) || x < 0.0f || x != D[j * n + i]) return ORC_EINVAL;
    }
  }
  return ORC_OK;
}

static int make_ctx(ctx* c, const float* D, int64_t n, int32_t kmax, float threshold,
                    uint32_t flags) {
  int rc = validate(D, n);
  if (rc) return rc;
  if (isnan(threshold) || kmax < 1) return ORC_EINVAL;
  c->D = D;
  c->n = n;
  c->kmax = kmax;
  c->tau = threshold;
  if (!(flags & ORC_FLAG_NO_ENCLOSING)) {
    float R = orc_enclosing_radius(D, n);
    if (R < c->tau) c->tau = R;
  }
  c->binom = binom_table(n, kmax);
  if (!c->binom) return ORC_ENOMEM;
  /* every index used must stay below 2^63 */
  if (c->binom[n * (kmax + 1) + kmax] >= (((u128)1) << 63)) {
    free(c->binom);
    return ORC_EOVERFLOW;
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Enumeration of Rips_tau simplices (Eq. 5.3)                              */
/* ------------------------------------------------------------------------ */

/* Depth-first over increasing vertex lists: a list is a simplex of Rips_tau
 * iff all its pairwise distances are <= tau. Emits simplices with between
 * qmin+1 and qmax+1 vertices. */
static int enum_rec(const ctx* c, int32_t* a, int32_t len, float diam, int32_t qmin,
                    int32_t qmax, simplex_vec* out) {
  if (len >= 1 && len - 1 >= qmin) {
    simplex s = {cidx_of(c, a, len - 1), diam, len - 1};
    if (sv_push(out, s)) return ORC_ENOMEM;
  }
  if (len == qmax + 1) return ORC_OK;
  for (int32_t u = (len ? a[len - 1] + 1 : 0); u < c->n; u++) {
    float d = diam;
    int ok = 1;
    for (int32_t i = 0; i < len; i++) {
      float e = dist(c, u, a[i]);
      if (!(e <= c->tau)) {
        ok = 0;
        break;
      }
      if (e > d) d = e;
    }
    if (!ok) continue;
    a[len] = u;
    if (enum_rec(c, a, len + 1, d, qmin, qmax, out)) return ORC_ENOMEM;
  }
  return ORC_OK;
}

static int enumerate(const ctx* c, int32_t qmin, int32_t qmax, simplex_vec* out) {
  int32_t a[64];
  if (qmax >= 63) return ORC_EINVAL;
  return enum_rec(c, a, 0, 0.0f, qmin, qmax, out);
}

/* Sec. 5.1.4: the simplex-wise refinement orders by increasing diameter,
 * then increasing dimension, then decreasing combinatorial index. */
static int cmp_filtration(const void* x, const void* y) {
  const simplex* a = (const simplex*)x;
  const simplex* b = (const simplex*)y;
  if (a->diam != b->diam) return a->diam < b->diam ? -1 : 1;
  if (a->dim != b->dim) return a->dim < b->dim ? -1 : 1;
  if (a->cidx != b->cidx) return a->cidx > b->cidx ? -1 : 1;
  return 0;
}

/* Reverse of the above within one dimension: the column (and row) order of a
 * coboundary matrix (Sec. 5.2.1: decreasing diameter, increasing index). */
static int cmp_coboundary(const void* x, const void* y) { return -cmp_filtration(x, y); }

static uint32_t fbits(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  return u;
}

/* Row key of a simplex in a coboundary matrix: increasing key = increasing
 * row index = reverse filtration order (diameter descending, index
 * ascending). Diameters here are >= 0, whose IEEE bit patterns order like the
 * values, and +0.0 is the only zero produced. */
static u128 row_key(float diam, uint64_t cidx) {
  return ((u128)(0xFFFFFFFFu - fbits(diam)) << 64) | (u128)cidx;
}
static uint64_t key_cidx(u128 k) { return (uint64_t)k; }
static float key_diam(u128 k) {
  uint32_t b = 0xFFFFFFFFu - (uint32_t)(k >> 64);
  float f;
  memcpy(&f, &b, 4);
  return f;
}

/* ------------------------------------------------------------------------ */
/* Results                                                                  */
/* ------------------------------------------------------------------------ */

struct orc_result {
  pair_vec pairs;
  int64_t columns[64];
};

static int cmp_pair(const void* x, const void* y) {
  const orc_pair* a = (const orc_pair*)x;
  const orc_pair* b = (const orc_pair*)y;
  if (a->dim != b->dim) return a->dim < b->dim ? -1 : 1;
  if (a->birth != b->birth) return a->birth < b->birth ? -1 : 1;
  if (a->death != b->death) return a->death < b->death ? -1 : 1;
  return 0;
}

int64_t orc_result_count(const orc_result* r) { return r ? r->pairs.len : 0; }
const orc_pair* orc_result_pairs(const orc_result* r) { return r ? r->pairs.a : NULL; }
int64_t orc_result_columns(const orc_result* r, int32_t dim) {
  return (r && dim >= 0 && dim < 64) ? r->columns[dim] : 0;
}
void orc_result_free(orc_result* r) {
  if (!r) return;
  free(r->pairs.a);
  free(r);
}

static orc_pair make_pair(int32_t dim, uint64_t b, float bd, uint64_t d, float dd) {
  orc_pair p;
  p.dim = dim;
  p.essential = 0;
  p.birth = b;
  p.death = d;
  p.birth_diam = bd;
  p.death_diam = dd;
  return p;
}

static orc_pair make_essential(int32_t dim, uint64_t b, float bd) {
  orc_pair p = make_pair(dim, b, bd, UINT64_MAX, INFINITY);
  p.essential = 1;
  return p;
}

/* ------------------------------------------------------------------------ */
/* Mode M1-boundary: Alg. 11 with Alg. 2 on the full boundary matrix        */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint64_t cidx;
  int64_t findex;
} idx_entry;

static int cmp_idx_entry(const void* x, const void* y) {
  const idx_entry* a = (const idx_entry*)x;
  const idx_entry* b = (const idx_entry*)y;
  return (a->cidx > b->cidx) - (a->cidx < b->cidx);
}

static int64_t find_index(const idx_entry* t, int64_t len, uint64_t cidx) {
  int64_t lo = 0, hi = len - 1;
  while (lo <= hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (t[mid].cidx == cidx) return t[mid].findex;
    if (t[mid].cidx < cidx)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

static int barcode_boundary(const ctx* c, int32_t max_dim, orc_result* res) {
  int rc = ORC_OK;
  simplex_vec S = {0};
  int32_t K = max_dim + 1;
  if ((rc = enumerate(c, 0, K, &S))) goto done;
  /* Alg. 11: the simplex-wise refinement */
  qsort(S.a, (size_t)S.len, sizeof(simplex), cmp_filtration);
  int64_t N = S.len;

  /* per-dimension lookup cidx -> filtration index, to find facets */
  idx_entry** tab = (idx_entry**)calloc((size_t)K + 1, sizeof(idx_entry*));
  int64_t* tlen = (int64_t*)calloc((size_t)K + 1, sizeof(int64_t));
  col* R = (col*)calloc((size_t)(N ? N : 1), sizeof(col));
  int64_t* L = (int64_t*)malloc((size_t)(N ? N : 1) * sizeof(int64_t));
  char* is_low = (char*)calloc((size_t)(N ? N : 1), 1);
  col tmp = {0};
  if (!tab || !tlen || !R || !L || !is_low) {
    rc = ORC_ENOMEM;
    goto done2;
  }
  for (int32_t q = 0; q <= K; q++) {
    tab[q] = (idx_entry*)malloc((size_t)(N ? N : 1) * sizeof(idx_entry));
    if (!tab[q]) {
      rc = ORC_ENOMEM;
      goto done2;
    }
  }
  for (int64_t i = 0; i < N; i++) {
    int32_t q = S.a[i].dim;
    tab[q][tlen[q]].cidx = S.a[i].cidx;
    tab[q][tlen[q]].findex = i;
    tlen[q]++;
  }
  for (int32_t q = 0; q <= K; q++) qsort(tab[q], (size_t)tlen[q], sizeof(idx_entry), cmp_idx_entry);

  /* Alg. 11: R <- boundary matrix; column j lists the filtration indices of
   * the facets of simplex j (remove one vertex at a time) */
  for (int64_t j = 0; j < N; j++) {
    int32_t q = S.a[j].dim;
    if (q == 0) continue;
    int32_t a[64], f[64];
    decode(c, S.a[j].cidx, q, a);
    if (col_reserve(&R[j], q + 1)) {
      rc = ORC_ENOMEM;
      goto done2;
    }
    for (int32_t r = 0; r <= q; r++) {
      int32_t m = 0;
      for (int32_t i = 0; i <= q; i++)
        if (i != r) f[m++] = a[i];
      int64_t fi = find_index(tab[q - 1], tlen[q - 1], cidx_of(c, f, q - 1));
      if (fi < 0) {
        rc = ORC_EINVAL; /* a facet missing from the complex: impossible */
        goto done2;
      }
      R[j].a[R[j].len++] = (u128)fi;
    }
    qsort(R[j].a, (size_t)R[j].len, sizeof(u128), cmp_u128);
  }

  /* Alg. 2: left to right; while low(R[j]) is already a pivot row, add the
   * column that owns it. */
  for (int64_t i = 0; i < N; i++) L[i] = -1;
  for (int64_t j = 0; j < N; j++) {
    while (R[j].len > 0 && L[(int64_t)R[j].a[R[j].len - 1]] != -1) {
      int64_t k = L[(int64_t)R[j].a[R[j].len - 1]];
      if (col_add(&R[j], &R[k], &tmp)) {
        rc = ORC_ENOMEM;
        goto done2;
      }
    }
    if (R[j].len > 0) L[(int64_t)R[j].a[R[j].len - 1]] = j;
  }

  /* pivots (low(j), j) are the pairs (Alg. 11) */
  for (int64_t j = 0; j < N; j++) {
    if (R[j].len == 0) continue;
    int64_t lo = (int64_t)R[j].a[R[j].len - 1];
    is_low[lo] = 1;
    if (S.a[lo].dim > max_dim) continue;
    if (pv_push(&res->pairs, make_pair(S.a[lo].dim, S.a[lo].cidx, S.a[lo].diam, S.a[j].cidx,
                                       S.a[j].diam))) {
      rc = ORC_ENOMEM;
      goto done2;
    }
  }
  /* essential: zero column that is never a pivot row (Thm 3.2.20, (0, i)) */
  for (int64_t i = 0; i < N; i++) {
    if (R[i].len != 0 || is_low[i] || S.a[i].dim > max_dim) continue;
    if (pv_push(&res->pairs, make_essential(S.a[i].dim, S.a[i].cidx, S.a[i].diam))) {
      rc = ORC_ENOMEM;
      goto done2;
    }
  }

done2:
  if (tab)
    for (int32_t q = 0; q <= K; q++) free(tab[q]);
  free(tab);
  free(tlen);
  if (R)
    for (int64_t j = 0; j < N; j++) free(R[j].a);
  free(R);
  free(L);
  free(is_low);
  free(tmp.a);
done:
  free(S.a);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Coboundary columns (Sec. 5.2.1, Def. 4.3.4)                               */
/* ------------------------------------------------------------------------ */

/* All cofacets t = s + {v}, v not in s, with diam(t) <= tau, as row keys in
 * increasing order (the column of s in the coboundary matrix). */
static int coboundary(const ctx* c, const simplex* s, col* out) {
  int32_t a[64], b[65];
  int32_t q = s->dim;
  decode(c, s->cidx, q, a);
  out->len = 0;
  if (col_reserve(out, c->n)) return ORC_ENOMEM;
  for (int32_t v = 0; v < c->n; v++) {
    int in_s = 0;
    float d = s->diam;
    for (int32_t i = 0; i <= q; i++) {
      if (a[i] == v) in_s = 1;
      else if (dist(c, v, a[i]) > d)
        d = dist(c, v, a[i]);
    }
    if (in_s || !(d <= c->tau)) continue;
    /* vertices of t in increasing order */
    int32_t m = 0, placed = 0;
    for (int32_t i = 0; i <= q; i++) {
      if (!placed && v < a[i]) {
        b[m++] = v;
        placed = 1;
      }
      b[m++] = a[i];
    }
    if (!placed) b[m++] = v;
    out->a[out->len++] = row_key(d, cidx_of(c, b, q + 1));
  }
  qsort(out->a, (size_t)out->len, sizeof(u128), cmp_u128);
  return ORC_OK;
}

/* low of a coboundary column without building it: the largest row key, i.e.
 * the oldest cofacet. Returns 0 if the column is zero. */
static int coboundary_low(const ctx* c, const simplex* s, u128* low) {
  int32_t a[64], b[65];
  int32_t q = s->dim;
  int found = 0;
  decode(c, s->cidx, q, a);
  for (int32_t v = 0; v < c->n; v++) {
    int in_s = 0;
    float d = s->diam;
    for (int32_t i = 0; i <= q; i++) {
      if (a[i] == v) in_s = 1;
      else if (dist(c, v, a[i]) > d)
        d = dist(c, v, a[i]);
    }
    if (in_s || !(d <= c->tau)) continue;
    int32_t m = 0, placed = 0;
    for (int32_t i = 0; i <= q; i++) {
      if (!placed && v < a[i]) {
        b[m++] = v;
        placed = 1;
      }
      b[m++] = a[i];
    }
    if (!placed) b[m++] = v;
    u128 k = row_key(d, cidx_of(c, b, q + 1));
    if (!found || k > *low) *low = k;
    found = 1;
  }
  return found;
}

/* Columns of the dimension-q coboundary matrix: every q-simplex with
 * diam <= tau that is not cleared, in coboundary order. */
static int columns_of_dim(const ctx* c, int32_t q, const map64* deaths, int clearing,
                          simplex_vec* cols) {
  simplex_vec all = {0};
  int rc = enumerate(c, q, q, &all);
  if (rc) {
    free(all.a);
    return rc;
  }
  for (int64_t i = 0; i < all.len; i++) {
    int64_t dummy;
    if (clearing && deaths && map_get(deaths, all.a[i].cidx, &dummy)) continue; /* Lemma 4.2.2 */
    if (sv_push(cols, all.a[i])) {
      free(all.a);
      return ORC_ENOMEM;
    }
  }
  free(all.a);
  qsort(cols->a, (size_t)cols->len, sizeof(simplex), cmp_coboundary);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Modes M1-coboundary (Alg. 2) and M2-streamed (Alg. 12), per dimension     */
/* ------------------------------------------------------------------------ */

static int barcode_coboundary(const ctx* c, int32_t max_dim, int streamed, int clearing,
                              orc_result* res) {
  int rc = ORC_OK;
  map64 deaths_prev = {0}; /* deaths of dimension q-1 pairs */
  int have_prev = 0;
  for (int32_t q = 0; q <= max_dim; q++) {
    simplex_vec cols = {0};
    map64 lookup = {0};  /* row cidx -> column index (the pivot table L) */
    map64 deaths = {0};
    col* R = NULL;
    col work = {0}, tmp = {0}, other = {0};
    if ((rc = columns_of_dim(c, q, have_prev ? &deaths_prev : NULL, clearing, &cols))) goto next;
    res->columns[q] = cols.len;
    if ((rc = map_init(&lookup, cols.len)) || (rc = map_init(&deaths, cols.len))) goto next;

    if (!streamed) {
      /* M1: the whole matrix is built first (Def. 4.3.4), then Alg. 2. */
      R = (col*)calloc((size_t)(cols.len ? cols.len : 1), sizeof(col));
      if (!R) {
        rc = ORC_ENOMEM;
        goto next;
      }
      for (int64_t j = 0; j < cols.len; j++)
        if ((rc = coboundary(c, &cols.a[j], &R[j]))) goto next;
      for (int64_t j = 0; j < cols.len; j++) {
        int64_t k;
        while (R[j].len > 0 && map_get(&lookup, key_cidx(R[j].a[R[j].len - 1]), &k)) {
          if ((rc = col_add(&R[j], &R[k], &tmp))) goto next;
        }
        if (R[j].len > 0) {
          u128 lo = R[j].a[R[j].len - 1];
          if ((rc = map_put(&lookup, key_cidx(lo), j))) goto next;
          if ((rc = map_put(&deaths, key_cidx(lo), 1))) goto next;
          /* Prop. 4.3.5: pivot (row t, column s) is the pair (s, t) */
          if ((rc = pv_push(&res->pairs, make_pair(q, cols.a[j].cidx, cols.a[j].diam,
                                                   key_cidx(lo), key_diam(lo)))))
            goto next;
        }
      }
      for (int64_t j = 0; j < cols.len; j++) {
        int64_t dummy;
        if (R[j].len != 0) continue;
        if (have_prev && map_get(&deaths_prev, cols.a[j].cidx, &dummy)) continue;
        if ((rc = pv_push(&res->pairs, make_essential(q, cols.a[j].cidx, cols.a[j].diam))))
          goto next;
      }
    } else {
      /* M2: Alg. 12, the column is materialised only if its low is taken. */
      for (int64_t j = 0; j < cols.len; j++) {
        u128 lo;
        int64_t k;
        int nonzero = coboundary_low(c, &cols.a[j], &lo);
        if (nonzero && map_get(&lookup, key_cidx(lo), &k)) {
          if ((rc = coboundary(c, &cols.a[j], &work))) goto next;
          while (work.len > 0 && map_get(&lookup, key_cidx(work.a[work.len - 1]), &k)) {
            /* R[j] <- R[j] + D_lookup[low(R[j])]: the ORIGINAL column */
            if ((rc = coboundary(c, &cols.a[k], &other))) goto next;
            if ((rc = col_add(&work, &other, &tmp))) goto next;
          }
          nonzero = work.len > 0;
          if (nonzero) lo = work.a[work.len - 1];
        }
        if (nonzero) {
          if ((rc = map_put(&lookup, key_cidx(lo), j))) goto next;
          if ((rc = map_put(&deaths, key_cidx(lo), 1))) goto next;
          if ((rc = pv_push(&res->pairs, make_pair(q, cols.a[j].cidx, cols.a[j].diam,
                                                   key_cidx(lo), key_diam(lo)))))
            goto next;
        } else {
          int64_t dummy;
          if (have_prev && map_get(&deaths_prev, cols.a[j].cidx, &dummy)) continue;
          if ((rc = pv_push(&res->pairs, make_essential(q, cols.a[j].cidx, cols.a[j].diam))))
            goto next;
        }
      }
    }
  next:
    if (R)
      for (int64_t j = 0; j < cols.len; j++) free(R[j].a);
    free(R);
    free(work.a);
    free(tmp.a);
    free(other.a);
    free(cols.a);
    map_free(&lookup);
    if (have_prev) map_free(&deaths_prev);
    if (rc) {
      map_free(&deaths);
      return rc;
    }
    deaths_prev = deaths;
    have_prev = 1;
  }
  if (have_prev) map_free(&deaths_prev);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Mode M3: the reduction-matrix technique (Sec. 5.2.9), streamed             */
/* ------------------------------------------------------------------------ */

/* binary max-heap of row keys */
typedef struct {
  u128* a;
  int64_t len, cap;
} heap;

static int heap_push(heap* h, u128 k) {
  if (h->len == h->cap) {
    int64_t nc = h->cap ? 2 * h->cap : 256;
    u128* na = (u128*)realloc(h->a, (size_t)nc * sizeof(u128));
    if (!na) return ORC_ENOMEM;
    h->a = na;
    h->cap = nc;
  }
  int64_t i = h->len++;
  h->a[i] = k;
  while (i > 0 && h->a[(i - 1) / 2] < h->a[i]) {
    u128 t = h->a[i];
    h->a[i] = h->a[(i - 1) / 2];
    h->a[(i - 1) / 2] = t;
    i = (i - 1) / 2;
  }
  return ORC_OK;
}

static u128 heap_pop(heap* h) {
  u128 top = h->a[0];
  h->a[0] = h->a[--h->len];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < h->len && h->a[l] > h->a[m]) m = l;
    if (r < h->len && h->a[r] > h->a[m]) m = r;
    if (m == i) break;
    u128 t = h->a[i];
    h->a[i] = h->a[m];
    h->a[m] = t;
    i = m;
  }
  return top;
}

/* The low of the column the heap holds: the largest key that appears an odd
 * number of times (Z/2). Keys that cancel are removed; the low stays. */
static int heap_low(heap* h, u128* low) {
  while (h->len > 0) {
    u128 t = heap_pop(h);
    int count = 1;
    while (h->len > 0 && h->a[0] == t) {
      heap_pop(h);
      count++;
    }
    if (count & 1) {
      *low = t;
      return heap_push(h, t) == ORC_OK ? 1 : -1;
    }
  }
  return 0;
}

static int heap_add_coboundary(const ctx* c, const simplex* s, heap* h, col* scratch) {
  if (coboundary(c, s, scratch)) return ORC_ENOMEM;
  for (int64_t i = 0; i < scratch->len; i++)
    if (heap_push(h, scratch->a[i])) return ORC_ENOMEM;
  return ORC_OK;
}

typedef struct {
  int64_t* a;
  int64_t len, cap;
} i64vec;

static int iv_push(i64vec* v, int64_t x) {
  if (v->len == v->cap) {
    int64_t nc = v->cap ? 2 * v->cap : 8;
    int64_t* na = (int64_t*)realloc(v->a, (size_t)nc * sizeof(int64_t));
    if (!na) return ORC_ENOMEM;
    v->a = na;
    v->cap = nc;
  }
  v->a[v->len++] = x;
  return ORC_OK;
}

static int cmp_i64(const void* x, const void* y) {
  int64_t a = *(const int64_t*)x, b = *(const int64_t*)y;
  return (a > b) - (a < b);
}

static int barcode_reduction_matrix(const ctx* c, int32_t max_dim, int clearing, orc_result* res) {
  int rc = ORC_OK;
  map64 deaths_prev = {0};
  int have_prev = 0;
  for (int32_t q = 0; q <= max_dim; q++) {
    simplex_vec cols = {0};
    map64 lookup = {0}, deaths = {0};
    i64vec* V = NULL; /* V[j]: columns (indices into cols) added to column j */
    heap h = {0};
    col scratch = {0};
    i64vec vj = {0};
    if ((rc = columns_of_dim(c, q, have_prev ? &deaths_prev : NULL, clearing, &cols))) goto next;
    res->columns[q] = cols.len;
    V = (i64vec*)calloc((size_t)(cols.len ? cols.len : 1), sizeof(i64vec));
    if (!V || (rc = map_init(&lookup, cols.len)) || (rc = map_init(&deaths, cols.len))) {
      if (!rc) rc = ORC_ENOMEM;
      goto next;
    }
    for (int64_t j = 0; j < cols.len; j++) {
      u128 lo;
      int64_t k;
      int nonzero = coboundary_low(c, &cols.a[j], &lo);
      vj.len = 0;
      if (nonzero && map_get(&lookup, key_cidx(lo), &k)) {
        /* the column is needed: build it, then add reduced columns R_k */
        h.len = 0;
        if ((rc = heap_add_coboundary(c, &cols.a[j], &h, &scratch))) goto next;
        while (nonzero && map_get(&lookup, key_cidx(lo), &k)) {
          if ((rc = heap_add_coboundary(c, &cols.a[k], &h, &scratch))) goto next;
          if ((rc = iv_push(&vj, k))) goto next;
          for (int64_t i = 0; i < V[k].len; i++) {
            if ((rc = heap_add_coboundary(c, &cols.a[V[k].a[i]], &h, &scratch))) goto next;
            if ((rc = iv_push(&vj, V[k].a[i]))) goto next;
          }
          nonzero = heap_low(&h, &lo);
          if (nonzero < 0) {
            rc = ORC_ENOMEM;
            goto next;
          }
        }
        /* V_j over Z/2 */
        qsort(vj.a, (size_t)vj.len, sizeof(int64_t), cmp_i64);
        for (int64_t a = 0; a < vj.len;) {
          int64_t b = a;
          while (b < vj.len && vj.a[b] == vj.a[a]) b++;
          if (((b - a) & 1) && (rc = iv_push(&V[j], vj.a[a]))) goto next;
          a = b;
        }
      }
      if (nonzero) {
        if ((rc = map_put(&lookup, key_cidx(lo), j))) goto next;
        if ((rc = map_put(&deaths, key_cidx(lo), 1))) goto next;
        if ((rc = pv_push(&res->pairs, make_pair(q, cols.a[j].cidx, cols.a[j].diam,
                                                 key_cidx(lo), key_diam(lo)))))
          goto next;
      } else {
        int64_t dummy;
        if (have_prev && map_get(&deaths_prev, cols.a[j].cidx, &dummy)) continue;
        if ((rc = pv_push(&res->pairs, make_essential(q, cols.a[j].cidx, cols.a[j].diam))))
          goto next;
      }
    }
  next:
    if (V)
      for (int64_t j = 0; j < cols.len; j++) free(V[j].a);
    free(V);
    free(h.a);
    free(scratch.a);
    free(vj.a);
    free(cols.a);
    map_free(&lookup);
    if (have_prev) map_free(&deaths_prev);
    if (rc) {
      map_free(&deaths);
      return rc;
    }
    deaths_prev = deaths;
    have_prev = 1;
  }
  if (have_prev) map_free(&deaths_prev);
  return ORC_OK;
}

int orc_barcode(const float* D, int64_t n, int32_t max_dim, float threshold, int32_t mode,
                uint32_t flags, orc_result** out) {
  if (!out || max_dim < 0 || max_dim > 60) return ORC_EINVAL;
  *out = NULL;
  ctx c;
  int rc = make_ctx(&c, D, n, max_dim + 2, threshold, flags);
  if (rc) return rc;
  orc_result* res = (orc_result*)calloc(1, sizeof(orc_result));
  if (!res) {
    free(c.binom);
    return ORC_ENOMEM;
  }
  if (mode == ORC_M1_BOUNDARY)
    rc = barcode_boundary(&c, max_dim, res);
  else if (mode == ORC_M1_COBOUNDARY || mode == ORC_M2_STREAMED)
    rc = barcode_coboundary(&c, max_dim, mode == ORC_M2_STREAMED,
                            !(flags & ORC_FLAG_NO_CLEARING), res);
  else if (mode == ORC_M3_REDUCTION_MATRIX)
    rc = barcode_reduction_matrix(&c, max_dim, !(flags & ORC_FLAG_NO_CLEARING), res);
  else
    rc = ORC_EINVAL;
  free(c.binom);
  if (rc) {
    orc_result_free(res);
    return rc;
  }
  qsort(res->pairs.a, (size_t)res->pairs.len, sizeof(orc_pair), cmp_pair);
  *out = res;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Alg. 2 on an explicit matrix                                             */
/* ------------------------------------------------------------------------ */

int orc_reduce_explicit(int32_t ncols, const int64_t* col_ptr, const int64_t* rows,
                        int64_t* low_out) {
  if (ncols < 0 || !col_ptr || !low_out) return ORC_EINVAL;
  int rc = ORC_OK;
  col* R = (col*)calloc((size_t)(ncols ? ncols : 1), sizeof(col));
  col tmp = {0}, one = {0};
  map64 L = {0};
  if (!R || map_init(&L, ncols)) {
    free(R);
    map_free(&L);
    return ORC_ENOMEM;
  }
  for (int32_t j = 0; j < ncols; j++) {
    int64_t b = col_ptr[j], e = col_ptr[j + 1];
    if (e < b || b < 0) {
      rc = ORC_EINVAL;
      goto done;
    }
    /* column as a Z/2 set: add each listed row as a one-element column */
    for (int64_t p = b; p < e; p++) {
      if (rows[p] < 0) {
        rc = ORC_EINVAL;
        goto done;
      }
      if ((rc = col_reserve(&one, 1))) goto done;
      one.a[0] = (u128)rows[p];
      one.len = 1;
      if ((rc = col_add(&R[j], &one, &tmp))) goto done;
    }
  }
  for (int32_t j = 0; j < ncols; j++) {
    int64_t k;
    while (R[j].len > 0 && map_get(&L, (uint64_t)R[j].a[R[j].len - 1], &k))
      if ((rc = col_add(&R[j], &R[k], &tmp))) goto done;
    if (R[j].len > 0 && (rc = map_put(&L, (uint64_t)R[j].a[R[j].len - 1], j))) goto done;
  }
  for (int32_t j = 0; j < ncols; j++) low_out[j] = R[j].len ? (int64_t)R[j].a[R[j].len - 1] : -1;
done:
  for (int32_t j = 0; j < ncols; j++) free(R[j].a);
  free(R);
  free(tmp.a);
  free(one.a);
  map_free(&L);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Apparent pairs straight from Def. 5.3.4                                   */
/* ------------------------------------------------------------------------ */

typedef struct {
  uint64_t s, t;
} st_pair;

static int cmp_st(const void* x, const void* y) {
  const st_pair* a = (const st_pair*)x;
  const st_pair* b = (const st_pair*)y;
  return (a->s > b->s) - (a->s < b->s);
}

int orc_apparent_pairs(const float* D, int64_t n, int32_t dim, float threshold, uint32_t flags,
                       uint64_t* s_out, uint64_t* t_out, int64_t cap, int64_t* count) {
  if (dim < 0 || !count) return ORC_EINVAL;
  ctx c;
  int rc = make_ctx(&c, D, n, dim + 2, threshold, flags);
  if (rc) return rc;
  simplex_vec cols = {0};
  col* Cb = NULL;
  map64 leftmost = {0};
  st_pair* found = NULL;
  int64_t nf = 0;
  if ((rc = columns_of_dim(&c, dim, NULL, 0, &cols))) goto done;
  Cb = (col*)calloc((size_t)(cols.len ? cols.len : 1), sizeof(col));
  found = (st_pair*)malloc((size_t)(cols.len ? cols.len : 1) * sizeof(st_pair));
  if (!Cb || !found || map_init(&leftmost, 16 * cols.len)) {
    rc = ORC_ENOMEM;
    goto done;
  }
  /* the explicit matrix, columns in coboundary order */
  for (int64_t j = 0; j < cols.len; j++)
    if ((rc = coboundary(&c, &cols.a[j], &Cb[j]))) goto done;
  /* leftmost nonzero of every row */
  for (int64_t j = cols.len - 1; j >= 0; j--)
    for (int64_t p = 0; p < Cb[j].len; p++)
      if ((rc = map_put(&leftmost, key_cidx(Cb[j].a[p]), j))) goto done;
  /* (t, s) apparent: t = low(s) and s is the leftmost column of row t */
  for (int64_t j = 0; j < cols.len; j++) {
    int64_t lm;
    if (Cb[j].len == 0) continue;
    uint64_t t = key_cidx(Cb[j].a[Cb[j].len - 1]);
    if (map_get(&leftmost, t, &lm) && lm == j) {
      found[nf].s = cols.a[j].cidx;
      found[nf].t = t;
      nf++;
    }
  }
  qsort(found, (size_t)nf, sizeof(st_pair), cmp_st);
  for (int64_t i = 0; i < nf && i < cap; i++) {
    if (s_out) s_out[i] = found[i].s;
    if (t_out) t_out[i] = found[i].t;
  }
  *count = nf;
done:
  if (Cb)
    for (int64_t j = 0; j < cols.len; j++) free(Cb[j].a);
  free(Cb);
  free(found);
  free(cols.a);
  map_free(&leftmost);
  free(c.binom);
  return rc;
}

int orc_is_apparent(const float* D, int64_t n, int32_t dim, uint64_t s, float threshold,
                    uint32_t flags, uint64_t* t_out) {
  if (dim < 0) return ORC_EINVAL;
  ctx c;
  int rc = make_ctx(&c, D, n, dim + 2, threshold, flags);
  if (rc) return rc;
  int result = 0;
  int32_t a[64], b[65], f[65];
  if (s >= C(&c, c.n, dim + 1)) {
    free(c.binom);
    return ORC_EINVAL;
  }
  decode(&c, s, dim, a);
  simplex ss = {s, diam_of(&c, a, dim), dim};
  if (!(ss.diam <= c.tau)) {
    free(c.binom);
    return 0; /* not a column of the matrix */
  }
  /* oldest cofacet: smallest diameter, then largest index (Sec. 5.1.4) */
  u128 oldest;
  if (!coboundary_low(&c, &ss, &oldest)) {
    free(c.binom);
    return 0;
  }
  uint64_t t = key_cidx(oldest);
  float td = key_diam(oldest);
  decode(&c, t, dim + 1, b);
  /* youngest facet of t: largest diameter, then smallest index */
  int have = 0;
  float yd = 0.0f;
  uint64_t yc = 0;
  for (int32_t r = 0; r <= dim + 1; r++) {
    int32_t m = 0;
    for (int32_t i = 0; i <= dim + 1; i++)
      if (i != r) f[m++] = b[i];
    float fd = diam_of(&c, f, dim);
    uint64_t fc = cidx_of(&c, f, dim);
    if (!have || fd > yd || (fd == yd && fc < yc)) {
      yd = fd;
      yc = fc;
      have = 1;
    }
  }
  (void)td;
  if (yc == s) {
    result = 1;
    if (t_out) *t_out = t;
  }
  free(c.binom);
  return result;
}

/* ------------------------------------------------------------------------ */
/* H0 by Kruskal (Sec. 5.2.5)                                                */
/* ------------------------------------------------------------------------ */

typedef struct {
  float d;
  uint64_t cidx;
  int32_t u, v;
} edge;

static int cmp_edge(const void* x, const void* y) {
  const edge* a = (const edge*)x;
  const edge* b = (const edge*)y;
  if (a->d != b->d) return a->d < b->d ? -1 : 1;
  return (a->cidx < b->cidx) - (a->cidx > b->cidx); /* index descending */
}

static int32_t uf_find(int32_t* parent, int32_t x) {
  while (parent[x] != x) x = parent[x];
  return x;
}

int orc_h0_kruskal(const float* D, int64_t n, float threshold, uint32_t flags, orc_pair* out,
                   int64_t cap, int64_t* count) {
  if (!count) return ORC_EINVAL;
  ctx c;
  int rc = make_ctx(&c, D, n, 2, threshold, flags);
  if (rc) return rc;
  int64_t ne = 0;
  edge* E = (edge*)malloc((size_t)(n * (n - 1) / 2 + 1) * sizeof(edge));
  int32_t* parent = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  int32_t* rep = (int32_t*)malloc((size_t)n * sizeof(int32_t)); /* oldest vertex */
  pair_vec P = {0};
  if (!E || !parent || !rep) {
    rc = ORC_ENOMEM;
    goto done;
  }
  for (int32_t u = 1; u < n; u++)
    for (int32_t v = 0; v < u; v++)
      if (dist(&c, u, v) <= c.tau) {
        E[ne].d = dist(&c, u, v);
        E[ne].cidx = C(&c, u, 2) + (uint64_t)v;
        E[ne].u = u;
        E[ne].v = v;
        ne++;
      }
  qsort(E, (size_t)ne, sizeof(edge), cmp_edge);
  for (int32_t i = 0; i < n; i++) {
    parent[i] = i;
    rep[i] = i;
  }
  for (int64_t e = 0; e < ne; e++) {
    int32_t a = uf_find(parent, E[e].u), b = uf_find(parent, E[e].v);
    if (a == b) continue;
    /* elder rule: the component whose oldest vertex is younger dies */
    int32_t young = rep[a] < rep[b] ? a : b, old = young == a ? b : a;
    if ((rc = pv_push(&P, make_pair(0, (uint64_t)rep[young], 0.0f, E[e].cidx, E[e].d)))) goto done;
    parent[young] = old;
  }
  for (int32_t i = 0; i < n; i++)
    if (uf_find(parent, i) == i && (rc = pv_push(&P, make_essential(0, (uint64_t)rep[i], 0.0f))))
      goto done;
  qsort(P.a, (size_t)P.len, sizeof(orc_pair), cmp_pair);
  for (int64_t i = 0; i < P.len && i < cap; i++) out[i] = P.a[i];
  *count = P.len;
done:
  free(E);
  free(parent);
  free(rep);
  free(P.a);
  free(c.binom);
  return rc;
}

/* ------------------------------------------------------------------------ */
/* Diameter edges and the gradient                                          */
/* ------------------------------------------------------------------------ */

int orc_diameter_edge(const float* D, int64_t n, int32_t dim, uint64_t cidx, int32_t* u,
                      int32_t* v) {
  if (!D || n < 2 || dim < 1 || dim > 60 || !u || !v) return ORC_EINVAL;
  ctx c;
  c.D = D;
  c.n = n;
  c.kmax = dim + 1;
  c.binom = binom_table(n, dim + 1);
  if (!c.binom) return ORC_ENOMEM;
  if (cidx >= C(&c, n, dim + 1)) {
    free(c.binom);
    return ORC_EINVAL;
  }
  int32_t a[64];
  decode(&c, cidx, dim, a);
  float d = diam_of(&c, a, dim);
  uint64_t best = 0;
  int have = 0;
  for (int32_t i = 0; i <= dim; i++)
    for (int32_t j = 0; j < i; j++)
      if (dist(&c, a[i], a[j]) == d) {
        uint64_t e = C(&c, a[i], 2) + (uint64_t)a[j];
        if (!have || e > best) {
          best = e;
          *u = a[i];
          *v = a[j];
          have = 1;
        }
      }
  free(c.binom);
  return ORC_OK;
}

static void add_edge_grad(const float* X, int32_t m, int32_t u, int32_t v, double g, double* gX) {
  double nrm2 = 0.0;
  for (int32_t k = 0; k < m; k++) {
    double d = (double)X[(int64_t)u * m + k] - (double)X[(int64_t)v * m + k];
    nrm2 += d * d;
  }
  double nrm = sqrt(nrm2);
  if (nrm == 0.0) return; /* coincident points: no direction, no gradient */
  for (int32_t k = 0; k < m; k++) {
    double d = (double)X[(int64_t)u * m + k] - (double)X[(int64_t)v * m + k];
    gX[(int64_t)u * m + k] += g * d / nrm;
    gX[(int64_t)v * m + k] -= g * d / nrm;
  }
}

int orc_gradient(const float* X, int64_t n, int32_t m, const float* D, const orc_pair* pairs,
                 int64_t npairs, const float* g_birth, const float* g_death, double* gX) {
  if (!X || !D || !gX || n < 1 || m < 1 || (npairs > 0 && !pairs)) return ORC_EINVAL;
  memset(gX, 0, (size_t)n * (size_t)m * sizeof(double));
  for (int64_t p = 0; p < npairs; p++) {
    int32_t u, v;
    if (pairs[p].dim >= 1 && g_birth && g_birth[p] != 0.0f) {
      if (orc_diameter_edge(D, n, pairs[p].dim, pairs[p].birth, &u, &v)) return ORC_EINVAL;
      add_edge_grad(X, m, u, v, (double)g_birth[p], gX);
    }
    if (!pairs[p].essential && g_death && g_death[p] != 0.0f) {
      if (orc_diameter_edge(D, n, pairs[p].dim + 1, pairs[p].death, &u, &v)) return ORC_EINVAL;
      add_edge_grad(X, m, u, v, (double)g_death[p], gX);
    }
  }
  return ORC_OK;
}
