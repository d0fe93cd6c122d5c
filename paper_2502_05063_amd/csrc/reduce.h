// Host submatrix reduction over the non-apparent columns (Sec. 5.5.1).
#pragma once

#include <cstdint>
#include <vector>

#include "vrph_internal.h"

namespace vrph {

// Read-only view of one cloud's filtration data on the host.
struct HostComplex {
  int n = 0;
  // n x n weights (float bits, kInf above tau_eff); may be null once Wr is
  // attached (the weights are then rank_bits[Wr])
  const uint32_t* W = nullptr;
  // Ranks of the same weights among the distinct finite ones (kInf stays
  // kInf) and the weight of each rank; filled by build_ranks. Only the
  // reduction reads them.
  const uint32_t* Wr = nullptr;
  const uint32_t* rank_bits = nullptr;
  uint32_t nranks = 0;
  // Neighbour bitmaps (row v: bit x set iff edge (v, x) is within tau_eff;
  // nbw 64-bit words per row) and whether the complex is sparse enough for
  // the reduction to walk them instead of every vertex.
  const uint64_t* nb = nullptr;
  int nbw = 0;
  bool sparse = false;
  const uint64_t* binom = nullptr;  // k-major binomial table, (kmax + 1) x (n + 1)
  int kmax = 0;
  uint64_t C(int v, int k) const { return binom[(size_t)k * (size_t)(n + 1) + (size_t)v]; }
  uint32_t w(int a, int b) const { return W[(size_t)a * (size_t)n + (size_t)b]; }
  uint32_t wr(int a, int b) const { return Wr[(size_t)a * (size_t)n + (size_t)b]; }
};

// Weight ranks for the host reduction. By the order invariance of the
// barcode (Obs. 5.6.8) the pairs depend only on the order of the distances,
// so the reduction compares dense ranks (equal weights share a rank) instead
// of float bit patterns and maps ranks back to weights on output.
struct RankTable {
  std::vector<uint32_t> Wr;    // n x n, symmetric, kInf where W is kInf
  std::vector<uint32_t> bits;  // weight (float bits) of each rank, increasing
  std::vector<uint64_t> nb;    // neighbour bitmaps, n rows of nbw words
  int nbw = 0;
  bool sparse = false;         // fewer than a quarter of the edges are finite
  void build(int n, const uint32_t* W);
  // The same table from the m finite edges of the lower triangle, sorted by
  // weight: e[k].key_hi = weight bits, e[k].cidx = a << 32 | b with a > b.
  // When the previous build was this one at the same n, only the entries it
  // wrote are reset (O(m) instead of O(n^2)).
  void build_from_edges(int n, const Column* e, size_t m);
  // entries written by the last build_from_edges (a << 32 | b), valid while
  // tracked_n == n
  std::vector<uint64_t> last;
  int tracked_n = 0;
  void attach(HostComplex& H) const {
    H.Wr = Wr.data();
    H.rank_bits = bits.data();
    H.nranks = (uint32_t)bits.size();
    H.nb = nb.data();
    H.nbw = nbw;
    H.sparse = sparse;
  }
};

struct PairRec {
  uint64_t birth, death;  // death = ~0 for an essential class
  uint32_t bdiam, ddiam;  // float bits; ddiam = kInf for an essential class
};

struct ReduceStats {
  int64_t additions = 0;
  int64_t emergent = 0;  // columns paired at their first pivot, with no addition
};

// Reduce the non-apparent columns of dimension d, given in coboundary order,
// with the reduction-matrix technique (Sec. 5.2.9: R = D V; a column adds the
// reduced columns of earlier pivots, so its pivot only moves up). H must
// carry a RankTable: rows are compared by weight rank. The working column
// keeps its rows in buckets over rank ranges, with sorted runs for the
// bucket the pivot is in.
// Pivot lookups go to a table of the pairs found so far, then to the apparent
// pairs, recognised on the fly from Def. 5.3.4 instead of a stored array.
// While a column's pivot is the cofacet of an apparent pair, the addition it
// makes depends on no other non-apparent column; every column follows that
// chain on its own, on `threads` host threads, first. The columns left with
// a pivot that another column took are then reduced in order, in blocks:
// blocks of long columns on all `threads` threads, with the same additions
// as the sequential pass (a column stops at a pivot only once every earlier
// unfinished column's pivot has moved past it), blocks of short columns on
// one thread; `always_wide` puts every block on all threads (for tests). A
// column whose first pivot is free is paired without building it (the
// emergent case of Sec. 5.2.11). Appends the pairs of dimension d to `pairs`
// in column order and the death indices to `deaths`.
void reduce_dimension(const HostComplex& H, int d, const Column* cols, int64_t ncols,
                      int threads, std::vector<PairRec>& pairs, std::vector<uint64_t>& deaths,
                      ReduceStats& stats, bool always_wide = false);

// Vertices v[d] > ... > v[0] of simplex `c` of dimension d (Eq. 5.6).
void decode_simplex(const HostComplex& H, uint64_t c, int d, int* v);

// Diameter edge (u > v) of simplex c of dimension d >= 1: among the longest
// edges, the one with the largest edge index.
void diameter_edge(const HostComplex& H, uint64_t c, int d, int32_t* u, int32_t* v);

// Alg. 2 (R = D V, only columns to the left added) on the unstable columns
// of an explicit n x n matrix in CSC form (ptr, rows: rows strictly
// increasing within a column, each below its column), given the pivots the
// device scan fixed: lookup[r] = the column whose lowest 1 is the leftmost
// 1 of row r, else -1 (such a column is reduced as it is). unstable: the
// other columns, increasing. low[0..n) receives low(R_j), -1 for zero.
// Long columns are reduced on `threads` threads at once with exactly the
// sequential additions (a column's lowest row only falls, so column j may
// stop at row l once every earlier unfinished column's lowest row is below
// l); `always_wide` forces that for every block (for tests). Returns false
// if a column's pivot row belongs to a column to its right (the matrix is
// not one Alg. 2 can reduce with this lookup).
bool reduce_explicit_columns(int64_t n, const int64_t* ptr, const int64_t* rows,
                             const int32_t* lookup, const int64_t* unstable, int64_t nun,
                             int threads, int64_t* low, int64_t* additions,
                             bool always_wide = false);

// Compression before the reduction of an explicit boundary matrix (Sec.
// 4.3.3, Alg. 8-9), in this reading: a row r whose column holds the leftmost
// 1 of some row (destroyer[r]; that column keeps a pivot, Lemma 4.2.5) never
// holds a pivot of a boundary matrix (Lemma 4.2.4), so row r is zeroed in
// every column; and an entry at a row that is the scan's pivot of a column
// p to the left is removed by adding column p, compressed first, which is
// free when the compressed column p is that single entry (the stable
// columns "having all nonzero entries above compressible" of Alg. 9). Only
// zeroed rows and additions of a column to a column on its right are used,
// so the pivots of Alg. 2 do not change. The scan's pivot columns are
// compressed in increasing order, then the unstable columns on `threads`
// threads. Writes the compressed matrix (those columns; every other column
// zero) to cptr / crows in the layout of ptr / rows, adds the additions made
// to *additions and the entries removed without one to *dropped. Returns
// false if a scan pivot's own row would be removed (not a boundary matrix).
bool compress_explicit(int64_t n, const int64_t* ptr, const int64_t* rows, const int32_t* lookup,
                       const uint8_t* destroyer, const int64_t* unstable, int64_t nun,
                       int threads, std::vector<int64_t>& cptr, std::vector<int64_t>& crows,
                       int64_t* additions, int64_t* dropped);

}  // namespace vrph
