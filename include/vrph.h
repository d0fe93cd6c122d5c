/*
 * vrph.h — C ABI of the MI355X (gfx950) Vietoris–Rips persistence library.
 *
 * The problem (Zhang, "Computing and Learning on Combinatorial Data", Ch. 5):
 * a finite metric space given as a distance matrix D (Sec. 5.1, Def. 5.1.1)
 * or as points in R^m, a maximum dimension and a diameter threshold (Eq. 5.3)
 * go in; the persistence pairs of every dimension 0..max_dim of the
 * Vietoris–Rips filtration come out (Alg. 11 output, Sec. 5.2).
 *
 * Conventions used throughout:
 *  - Simplices are named by their combinatorial index (Eq. 5.6): vertices
 *    v_k > ... > v_0 map to sum_i C(v_i, i+1). A vertex v has index v.
 *  - The filtration order is the simplex-wise refinement of Sec. 5.1.4:
 *    diameter ascending, then dimension ascending, then index descending.
 *    A pair (birth, death) is a pivot of the reduced boundary matrix.
 *  - The threshold is inclusive (diam <= threshold). Unless
 *    VRPH_NO_ENCLOSING_RADIUS is given, the effective threshold is
 *    min(threshold, R) with R = min_i max_j D_ij the enclosing radius
 *    (Sec. 5.2.12); this never changes a pair of nonzero persistence
 *    (Prop. 5.2.13). threshold = +inf means the full Rips filtration.
 *  - Distances computed from points are
 *      D_ij = float32( sqrt( sum_k (x_ik - x_jk)^2 ) )
 *    with the differences, squares, left-to-right sum and a correctly rounded
 *    square root in IEEE binary64 and one final rounding to float32.
 *  - Pointer arguments named X, D, gX, edges, g_birth, g_death, X_packed are
 *    DEVICE pointers owned by the caller, read (or for gX accumulated into)
 *    in stream order on the given stream (NULL = the context's own stream).
 *    The call returns after the stream work it needs has completed.
 *  - Results (vrph_barcode) are owned by the library, live in host memory and
 *    are released with vrph_barcode_free.
 *  - Every entry point returns a vrph_status; nothing aborts or throws across
 *    the ABI. On failure no output object is produced and vrph_last_error()
 *    returns a thread-local description.
 *  - A context is not thread safe: use one per host thread.
 */
#ifndef VRPH_H
#define VRPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  VRPH_OK = 0,
  VRPH_EINVAL = -1,    /* bad argument or invalid distance matrix */
  VRPH_ENOMEM = -2,    /* device or host allocation failed */
  VRPH_EOVERFLOW = -3, /* C(n, max_dim + 2) >= 2^63: indices do not fit */
  VRPH_EDEVICE = -4,   /* a HIP call failed */
  VRPH_ESTATE = -5     /* call not valid in the object's current state, or a call
                          that waits for its stream made on a stream under capture */
} vrph_status;

/* flags */
#define VRPH_KEEP_ZERO_PERSISTENCE 1u /* report every pair, also birth == death */
#define VRPH_NO_ENCLOSING_RADIUS 2u   /* do not cut at the enclosing radius */
/* Autotune: the first call that meets a (dimension, size bucket) not yet
 * tuned times the enumeration + apparent-pairs kernel of that dimension over
 * its launch settings (workgroups per compute unit and, for dimension >= 2,
 * simplices per work unit), with HIP events, and keeps the fastest for the
 * context. If the environment variable VRPH_TUNING_FILE names a file,
 * tunings are read from it when the context is created and appended to it
 * when found (lines "arch dimension size_bucket variant unit_size
 * groups_per_cu", variant 0 for the global-memory kernel, 1 for the LDS one,
 * 2 for the dimension-1 kernel over neighbour lists, 3 for a batch plan,
 * see vrph_batch_plan). */
#define VRPH_AUTOTUNE 4u
/* Use the global-memory enumeration kernels even when the cloud is small
 * enough (n <= 200) for the kernels that read a 16-bit rank matrix from LDS.
 * Results are identical; this exists to compare and test the two. */
#define VRPH_NO_LDS 8u
/* Keep the cleared columns of every dimension >= 2 (Alg. 17: deaths and
 * apparent cofacets of the dimension below) in a hash set of their indices
 * instead of a bitmap over all C(n, d+1) indices. The library does this by
 * itself where a bitmap would exceed 8 GB (e.g. dimension 3 of 4096
 * points); the flag forces it, for testing. Results are identical. */
#define VRPH_HASHED_CLEARING 16u
/* Unknown flag bits are rejected with VRPH_EINVAL. */

/* vrph_boundary_pivots: no clearing step and no compression (for a matrix
 * that is not a boundary matrix, where Lemmas 4.2.3 and 4.2.4 do not hold) */
#define VRPH_BOUNDARY_NO_CLEARING 32u
/* vrph_boundary_pivots: no compression step (Sec. 4.3.3, Alg. 8-9) before
 * the host reduction; the pivots are the same (for comparing the two) */
#define VRPH_BOUNDARY_NO_COMPRESSION 64u
/* vrph_batch_plan: reduce the non-apparent columns of dimension 1 on host
 * threads instead of on the device (the results are the same; for comparing
 * the two) */
#define VRPH_HOST_REDUCTION 128u
/* vrph_batch_plan: reduce every cloud's dimension 1 on the device (unless its
 * tables overflow), instead of handing the clouds the cost model deems
 * heaviest to host threads that run beside the device reduction (the
 * results are the same; for comparing the two) */
#define VRPH_DEVICE_REDUCTION 512u
/* The paper's unfused order for dimensions 2 and 3 of a cloud of at most 200
 * points (the kernels that read the rank matrix from LDS): every column
 * that survives the threshold and clearing is written (Alg. 17), all of
 * them are sorted into coboundary order (Alg. 18), and the apparent-pairs
 * test (Lemma 5.3.6, Alg. 13) then runs over the sorted columns, instead of
 * the test fused into the enumeration with only the non-apparent columns
 * sorted. The results are the same; it exists to measure what the fusion
 * saves (stats.apparent_ms covers the three stages). Where it does not apply
 * (other dimensions, larger clouds, listed prefixes, hashed clearing sets,
 * or every pair reported) the fused path runs. It needs device memory for
 * three copies of 16 bytes per candidate of the dimension. */
#define VRPH_FULL_SORT 256u
#define VRPH_MAX_DIM 6 /* largest supported max_dim */

typedef struct vrph_ctx vrph_ctx;
typedef struct vrph_barcode vrph_barcode;
typedef struct vrph_batch vrph_batch;

/* One persistence pair; 48 bytes. birth/death are combinatorial indices of
 * the birth simplex (dimension dim) and death simplex (dimension dim+1).
 * Essential classes (never killed below the threshold) have essential = 1,
 * death = UINT64_MAX and death_diam = +inf. birth_edge / death_edge give the
 * vertices (u > v) of the edge realising the simplex's diameter: among the
 * longest edges, the one with the largest edge index. They are -1 for a
 * vertex birth and for an essential death. */
typedef struct {
  int32_t dim;
  int32_t essential;
  uint64_t birth;
  uint64_t death;
  float birth_diam;
  float death_diam;
  int32_t birth_edge[2];
  int32_t death_edge[2];
} vrph_pair;

/* Counts per dimension d (index d), in the terms of Ch. 5:
 *   candidates      simplices examined by the enumeration (all C(n, d+1)
 *                   indices; where at most half the vertex pairs are edges
 *                   and n > 200, dimensions 2 and 3 enumerate only vertex
 *                   sets over common neighbours, and this counts those)
 *   columns         columns of the coboundary matrix after the threshold and
 *                   clearing (Alg. 17)
 *   apparent        columns found apparent (Lemma 5.3.6)
 *   reduced         non-apparent columns reduced on the host (Sec. 5.5.1)
 *   additions       column additions made by that reduction
 *   pairs           pairs of dimension d, all of them (also zero persistence)
 *   cofacets        cofacets examined by the apparent-pairs scans
 *   facets          facets of a found cofacet whose diameter the second
 *                   condition of the apparent-pairs test computed
 *   emergent        non-apparent columns the host reduction paired at their
 *                   first pivot without any addition (the emergent-pair
 *                   shortcut of Sec. 5.2.11; apparent + emergent columns are
 *                   the columns that needed no reduction, Table 5.1)
 *   gpu_ms          device time of dimension d's kernels (HIP events)
 *   apparent_ms     device time of the enumeration + apparent-pairs kernel
 *                   of dimension d alone (HIP events on the call's stream)
 *   host_ms         host time of dimension d's reduction
 *   grid            workgroups launched by dimension d's enumeration kernel  */
typedef struct {
  int64_t candidates[VRPH_MAX_DIM + 1];
  int64_t columns[VRPH_MAX_DIM + 1];
  int64_t apparent[VRPH_MAX_DIM + 1];
  int64_t reduced[VRPH_MAX_DIM + 1];
  int64_t additions[VRPH_MAX_DIM + 1];
  int64_t pairs[VRPH_MAX_DIM + 1];
  int64_t cofacets[VRPH_MAX_DIM + 1];
  int64_t facets[VRPH_MAX_DIM + 1];
  int64_t emergent[VRPH_MAX_DIM + 1];
  double gpu_ms[VRPH_MAX_DIM + 1];
  double apparent_ms[VRPH_MAX_DIM + 1];
  double host_ms[VRPH_MAX_DIM + 1];
  int32_t grid[VRPH_MAX_DIM + 1];
  int32_t device_reduced; /* 1 if dimension 1 was reduced on the device (batches) */
  float tau_eff;       /* the threshold actually applied */
  int32_t max_dim;
  double total_ms;     /* host wall time of the whole call */
} vrph_stats;

/* Create a context on HIP device `device` (it becomes current for the calling
 * thread). The context owns a stream, device workspaces that grow on demand
 * and are reused across calls, and the binomial tables. */
vrph_status vrph_create(int device, vrph_ctx** out);
void vrph_destroy(vrph_ctx* ctx);

/* Thread-local text for the last non-OK status returned on this thread. */
const char* vrph_last_error(void);

/* Pairwise distances (Def. 5.1.1, formula above): X is n x m row-major
 * float32, D receives n x n float32 (symmetric, zero diagonal). */
vrph_status vrph_pdist(vrph_ctx* ctx, const float* X, int64_t n, int32_t m, float* D,
                       void* hip_stream);

/* Barcode of a distance matrix. D: n x n float32, finite, >= 0, symmetric,
 * zero diagonal (VRPH_EINVAL otherwise; the triangle inequality is not
 * required, Sec. 5.6.6). 1 <= n <= 16384 (the n x n weights take 4 n^2
 * bytes of device memory, 1 GiB at 16384), 0 <= max_dim <= VRPH_MAX_DIM,
 * threshold >= 0 or +inf. The host reduction receives the weights as the
 * n x n matrix, or, for a cloud of 512 points or more whose complex is
 * sparse (fewer than half of the vertex pairs within the threshold), as
 * its finite edges sorted by weight (16 bytes each); the environment
 * variable VRPH_DENSE_HOST_WEIGHTS, when set, keeps the matrix in every
 * case (the results are the same). */
vrph_status vrph_barcode_from_dist(vrph_ctx* ctx, const float* D, int64_t n, int32_t max_dim,
                                   float threshold, uint32_t flags, void* hip_stream,
                                   vrph_barcode** out);

/* Same from points: pdist, then the above. */
vrph_status vrph_barcode_from_points(vrph_ctx* ctx, const float* X, int64_t n, int32_t m,
                                     int32_t max_dim, float threshold, uint32_t flags,
                                     void* hip_stream, vrph_barcode** out);

/* Same from a sparse distance matrix (Sec. 5.3.12: the distances not given
 * are infinite, so no simplex with such an edge has a finite diameter; the
 * o3 run of Table 5.2 uses this input): nnz entries (row[k], col[k], val[k]),
 * each an unordered pair of distinct points 0 <= row, col < n given once, in
 * either orientation, with val finite and >= 0. Pairs that are not given are
 * not edges (an infinite distance): no simplex containing them is in the
 * filtration. row, col (int32) and val (float32) are DEVICE arrays of nnz
 * entries. The enclosing radius (unless VRPH_NO_ENCLOSING_RADIUS) is
 * min_i max_j D_ij with the missing entries infinite, i.e. it only cuts
 * where some point has all its n-1 distances given. VRPH_EINVAL for an
 * index out of range, a diagonal entry, a repeated pair, or a value that is
 * negative or not finite. 1 <= n <= 16384, 0 <= nnz <= n(n-1)/2. */
vrph_status vrph_barcode_from_sparse(vrph_ctx* ctx, int64_t n, int64_t nnz, const int32_t* row,
                                     const int32_t* col, const float* val, int32_t max_dim,
                                     float threshold, uint32_t flags, void* hip_stream,
                                     vrph_barcode** out);

/* Pairs of dimension dim (dim = -1: all dimensions), canonical order: by
 * dimension, then birth index, then death index. Without
 * VRPH_KEEP_ZERO_PERSISTENCE, pairs with birth_diam == death_diam are left
 * out, as in Ripser's output. */
int64_t vrph_barcode_count(const vrph_barcode* bc, int32_t dim);
const vrph_pair* vrph_barcode_pairs(const vrph_barcode* bc, int32_t dim);
const vrph_stats* vrph_barcode_stats(const vrph_barcode* bc);
void vrph_barcode_free(vrph_barcode* bc);

/* ---- batched point clouds -------------------------------------------------
 * A plan fixes the cloud sizes, the ambient dimension m, max_dim, threshold
 * and flags, and allocates every device buffer the batch needs up front.
 * Clouds are packed row-major one after another in X_packed
 * (sum(sizes) x m floats). vrph_batch_forward replays a captured HIP graph
 * over all clouds: distances, enclosing radii, H0, enumeration and the
 * apparent-pairs test and the sort of the non-apparent columns of dimension
 * 1. A second captured graph then reduces those columns (Sec.
 * 5.2.9-5.2.11), one workgroup per cloud, while host threads reduce the
 * clouds that a cost model (non-apparent columns x points, and a
 * host-to-device time ratio the batch updates from what each forward
 * measures) deems heaviest; the forward then copies the pairs back. A cloud
 * whose reduction outgrows its device tables is reduced on host threads
 * too. Under VRPH_DEVICE_REDUCTION every cloud is reduced on the device,
 * under VRPH_HOST_REDUCTION every cloud on host threads; the results do not
 * depend on where a cloud is reduced (stats.device_reduced tells which).
 * Each size must satisfy 2 <= size <= 4096 and every cloud uses the same
 * max_dim (<= 1). vrph_batch_plan accepts VRPH_KEEP_ZERO_PERSISTENCE,
 * VRPH_NO_ENCLOSING_RADIUS, VRPH_HOST_REDUCTION, VRPH_DEVICE_REDUCTION (not
 * both) and VRPH_AUTOTUNE: the first forward then runs the batch's device work
 * eagerly for a few launch settings (the device reduction's workgroup size,
 * 256, 512 or 1024 lanes per cloud; the dimension-1 edge kernel's
 * workgroups per compute unit), timed with HIP events with every cloud
 * reduced on the device, and captures the graphs with the fastest; the
 * choice is kept per (GPU architecture, size bucket of the largest cloud)
 * in the context and in VRPH_TUNING_FILE
 * (variant 3), and later plans of that bucket use it without tuning. Results
 * do not depend on the settings. It sizes every device buffer first and returns
 * VRPH_ENOMEM, allocating nothing, when they exceed the free device memory
 * or the byte count in the environment variable VRPH_WORKSPACE_CAP (if
 * set); a plan that fails frees whatever it had allocated. */
vrph_status vrph_batch_plan(vrph_ctx* ctx, const int64_t* sizes, int32_t count, int32_t m,
                            int32_t max_dim, float threshold, uint32_t flags, vrph_batch** out);
vrph_status vrph_batch_forward(vrph_batch* b, const float* X_packed, void* hip_stream);
/* Result of cloud i of the last forward; owned by the batch, valid until the
 * next forward or vrph_batch_destroy. Vertex and edge numbers are local to
 * the cloud. */
vrph_status vrph_batch_result(vrph_batch* b, int32_t cloud, const vrph_barcode** view);
void vrph_batch_destroy(vrph_batch* b);

/* ---- backward (gradient of a loss on birth and death values) ---------------
 * For pair p, edges[4p+0..1] is the diameter edge (u, v) of its birth simplex
 * and edges[4p+2..3] that of its death simplex, as global point numbers into
 * X (-1 = no edge: vertex birth or essential death). g_birth / g_death hold
 * dL/d(birth value) and dL/d(death value). Since the value is |x_u - x_v|,
 *   gX[u] += g (x_u - x_v) / |x_u - x_v|,  gX[v] -= the same,
 * with nothing added for coincident points. X and gX are n_total x m
 * (row-major); gX is accumulated into, with float32 atomics (summation order
 * is not fixed). Every edge entry must be -1 or in [0, n_total): otherwise
 * the call returns VRPH_EINVAL and gX is left unchanged (the entries are
 * checked on the device before anything is read or added). The pairs come
 * from vrph_barcode_pairs / vrph_batch_result (birth_edge, death_edge; batch
 * results are cloud-local and are offset by the cloud's first point). */
vrph_status vrph_backward(vrph_ctx* ctx, const float* X, int64_t n_total, int32_t m,
                          const int32_t* edges, int64_t npairs, const float* g_birth,
                          const float* g_death, float* gX, void* hip_stream);

/* Allocation-free backward, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight training or serving loops, harnesses
 * that forbid hipMalloc): the same arguments, result and errors as
 * vrph_backward, but its one word of device scratch (the edge-check flag) is
 * taken from a fixed 256-byte array that the library holds on every device
 * it runs on until the process ends, looked up when a context is created on
 * that device; no device or pinned memory is allocated by the call, whatever
 * npairs is. Every call on one GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other host threads, other contexts)
 * race with each other and must be serialised by the caller. VRPH_ESTATE if
 * the array of the context's device was not set up. */
vrph_status vrph_backward_noalloc(vrph_ctx* ctx, const float* X, int64_t n_total, int32_t m,
                                  const int32_t* edges, int64_t npairs, const float* g_birth,
                                  const float* g_death, float* gX, void* hip_stream);

/* ---- explicit boundary matrices (Sec. 4.3.2-4.3.3, Alg. 2-7) ---------------
 * The pivots low(R_j) of the Z/2 column reduction of Alg. 2 (R = D V, only
 * columns to the left added) of an explicit ncols x ncols matrix: the
 * boundary matrix of a filtration, cells in filtration order, so that the
 * rows of column j are faces of cell j and come before it. CSC, DEVICE
 * arrays: col_ptr (int64, ncols + 1 entries, col_ptr[0] = 0, non-decreasing)
 * and rows (int64, col_ptr[ncols] entries, strictly increasing within a
 * column, every row of column j in [0, j)).
 * The device scan (Alg. 3-6) finds the leftmost 1 of every row; a column
 * whose lowest 1 is the leftmost 1 of its row is a pivot no addition can
 * change (it is stable), zero columns are stable, and the column named by
 * such a pivot's row reduces to zero (clearing, Lemma 4.2.3, Alg. 7; left
 * out with VRPH_BOUNDARY_NO_CLEARING, which makes any strictly upper
 * triangular Z/2 matrix valid). With clearing, the host then compresses
 * the matrix (Sec. 4.3.3, Alg. 8-9): a row whose column holds some row's
 * leftmost 1 is zeroed (that column keeps a pivot, Lemma 4.2.5, so the row
 * never holds one, Lemma 4.2.4), and an entry at the row of a scan pivot of
 * a column to the left is removed by adding that (compressed) column,
 * without an addition when it is a single 1 (VRPH_BOUNDARY_NO_COMPRESSION
 * leaves this out). The host then reduces the other (unstable) columns in
 * order with Alg. 2, adding stable pivots' columns and reduced columns of
 * earlier unstable ones. Neither step changes a pivot.
 * low_out: HOST array of ncols int64, receives low(R_j), -1 for a zero
 * column. stats (optional, HOST) receives counts and times. VRPH_EINVAL for
 * a malformed matrix (also a row outside [0, j)) or ncols >= 2^31. */
typedef struct {
  int64_t columns;     /* ncols */
  int64_t zero;        /* zero columns of the input */
  int64_t stable;      /* columns the scan settled (zero, pivots, cleared) */
  int64_t scan_pivots; /* pivots the scan found (Alg. 5) */
  int64_t unstable;    /* columns reduced on the host */
  int64_t additions;   /* column additions of the host reduction (Alg. 2) */
  int64_t compress_additions; /* column additions made by the compression */
  int64_t compressed;  /* entries the compression removed without an addition */
  double scan_ms;      /* the four scan kernels (HIP events) */
  double host_ms;      /* compression, host reduction and result assembly */
} vrph_boundary_stats;

vrph_status vrph_boundary_pivots(vrph_ctx* ctx, int64_t ncols, const int64_t* col_ptr,
                                 const int64_t* rows, uint32_t flags, void* hip_stream,
                                 int64_t* low_out, vrph_boundary_stats* stats);

/* ---- extended persistence of graphs (Sec. 7.2, Alg. 27-28) ---------------
 * A consumer of persistence on a different input: graphs with a value f(v)
 * per vertex, as used for graph readouts (Ch. 7). The extended filtration of
 * the coned graph (Eq. 7.3-7.4: the lower filtration of G, edges at
 * F_low(u, v) = max(f(u), f(v)), then the upper filtration of the cone, cone
 * edges at f(v) and cone triangles at F_up(u, v) = min(f(u), f(v)),
 * descending) gives four barcodes (Theorem 7.6.2):
 *   VRPH_EXT_ORD0  birth a vertex, death an edge (lower filtration)      n - C bars
 *   VRPH_EXT_REL1  birth a vertex, death an edge (upper filtration)      n - C bars
 *   VRPH_EXT_EXT0  birth a component's minimum vertex, death its maximum   C bars
 *   VRPH_EXT_EXT1  birth an edge (lower), death an edge (upper)      m - n + C bars
 * (C components), n + m bars per graph in all. Ties are broken by an exact
 * order: vertices by (f, vertex), lower edges by (F_low, F_up, edge id),
 * upper edges by (F_up, F_low, edge id) descending. birth_vertex /
 * death_vertex name the vertex whose f is the bar's value (for a lower edge
 * value the endpoint with the larger (f, vertex), for an upper one the
 * smaller), where a loss's gradient with respect to f goes. */
#define VRPH_EXT_ORD0 0
#define VRPH_EXT_REL1 1
#define VRPH_EXT_EXT0 2
#define VRPH_EXT_EXT1 3
typedef struct {
  int32_t kind;         /* VRPH_EXT_* */
  int32_t birth;        /* vertex (ORD0, REL1, EXT0) or edge id (EXT1), local to the graph */
  int32_t death;        /* edge id (ORD0, REL1, EXT1) or vertex (EXT0) */
  float birth_value;
  float death_value;
  int32_t birth_vertex;
  int32_t death_vertex;
} vrph_ext_bar;

/* The four barcodes of each of `count` graphs. v_off and e_off are HOST
 * arrays of count + 1 offsets (v_off[0] = e_off[0] = 0, non-decreasing):
 * graph g has vertices [v_off[g], v_off[g+1]) and edges [e_off[g],
 * e_off[g+1]). f (v_off[count] floats, finite) and edges (2 e_off[count]
 * int32: the two endpoints of each edge, numbered within its graph, distinct)
 * are DEVICE arrays; a repeated edge is allowed (a multigraph). bars is a
 * caller-owned DEVICE array of v_off[count] + e_off[count] records: graph
 * g's n + m bars fill [v_off[g] + e_off[g], v_off[g+1] + e_off[g+1]), Ord0
 * and Rel1 bars first in the order their union-find passes find them, then
 * Ext0, then Ext1 in the order of their death edges in the upper
 * filtration. 1 <= n <= 4096 per graph, totals below 2^31. VRPH_EINVAL for
 * bad offsets, an endpoint outside its graph, a loop or a value that is not
 * finite (checked on the device before anything else runs; bars is then
 * left unwritten). */
vrph_status vrph_graph_extended(vrph_ctx* ctx, int32_t count, const int64_t* v_off,
                                const int64_t* e_off, const float* f, const int32_t* edges,
                                vrph_ext_bar* bars, void* hip_stream);

/* The backward of the readout (the bars as a differentiable layer over f,
 * Ch. 7; Sec. 7.2's values are f at the vertices the bars name): for the
 * bars of a vrph_graph_extended call with the same count, v_off and e_off
 * (HOST arrays, checked as there), adds g_birth[i] to g_f at bar i's
 * birth_vertex and g_death[i] at its death_vertex (vertex numbers within
 * the bar's graph, which is fixed by its position). bars (v_off[count] +
 * e_off[count] records), g_birth and g_death (one float per bar; either may
 * be NULL for zero) and g_f (v_off[count] floats, caller-owned, accumulated
 * into, not zeroed) are DEVICE arrays. The pairing is piecewise constant in
 * f, so this is the gradient wherever the vertex values are distinct.
 * VRPH_EINVAL for bad offsets or a bar whose vertices are not in its graph
 * (checked before anything is written). */
vrph_status vrph_graph_extended_backward(vrph_ctx* ctx, int32_t count, const int64_t* v_off,
                                         const int64_t* e_off, const vrph_ext_bar* bars,
                                         const float* g_birth, const float* g_death, float* g_f,
                                         void* hip_stream);

#ifdef __cplusplus
}
#endif
#endif
