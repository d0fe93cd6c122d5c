// Internal declarations shared by the HIP kernels (kernels.hip, sort.hip)
// and the host runtime (vrph_api.cpp, reduce.cpp). Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "vrph.h"

namespace vrph {

// Edge weights are the IEEE bit patterns of the float32 distances, which
// order like the values for non-negative floats. Entries above the effective
// threshold (and the diagonal) hold kInf, larger than any finite pattern.
constexpr uint32_t kInf = 0xFFFFFFFFu;
constexpr int kMaxDim = 6;        // largest max_dim
constexpr int kMaxN = 16384;      // largest single cloud
constexpr int kBatchMaxN = 4096;  // largest cloud of a batch (one-workgroup H0 in LDS)
constexpr int kH0LdsN = 4096;     // largest cloud whose H0 finish sorts its forest in LDS
constexpr int kBlock = 256;       // threads per workgroup of the streaming kernels
// clouds up to kLdsMaxN points enumerate from a 16-bit rank matrix in LDS
// (at most 80,000 bytes, two workgroups of kLdsBlock per 160 KB CU)
constexpr int kLdsMaxN = 200;
constexpr int kLdsBlock = 1024;
// Row stride, in 16-bit entries, of the rank matrix in LDS: 8q >= n with q
// odd. Rows start on 16-byte boundaries, so 8 consecutive entries of a row
// are one 128-bit read; with q odd, the rows of 8 (32 banks) or 16 (64
// banks) consecutive vertices start on distinct 4-bank groups, so lanes that
// read the rows of consecutive vertices do not conflict. For n <= kLdsMaxN
// the stride is at most kLdsMaxN.
__host__ __device__ constexpr int lds_stride(int n) {
  return 8 * ((((n + 7) / 8) & 1) ? (n + 7) / 8 : (n + 7) / 8 + 1);
}
static_assert(lds_stride(kLdsMaxN) <= kLdsMaxN, "rank matrix of kLdsMaxN points fits its LDS");
// A dispatch counts its work-items in 32 bits: launches of kBlock-thread
// workgroups stay at or below this many workgroups and stride over the rest.
constexpr int kMaxGroups = 1 << 22;

// A non-apparent column of the coboundary matrix. Sorting ascending by
// (cloud, key_hi, cidx) gives coboundary order within each cloud: diameter
// descending (key_hi = ~diameter bits), index ascending (Sec. 5.2.1).
struct Column {
  uint32_t key_hi;
  uint32_t cloud;
  uint64_t cidx;
};
static_assert(sizeof(Column) == 16, "Column is 16 bytes");

// An apparent pair (s, t) (Def. 5.3.4) with their common diameter.
struct ApparentPair {
  uint64_t s;
  uint64_t t;
  uint32_t diam;
  uint32_t cloud;
};
static_assert(sizeof(ApparentPair) == 24, "ApparentPair is 24 bytes");

// An H0 pair: vertex birth (diameter 0) and edge death, or essential.
struct H0Pair {
  uint64_t death;  // edge index, or ~0 for an essential class
  uint32_t birth;  // vertex
  uint32_t diam;   // death diameter bits (kInf for essential)
};
static_assert(sizeof(H0Pair) == 16, "H0Pair is 16 bytes");

// Per-call device scalars, read back once per stage.
struct Scalars {
  uint32_t err;       // bit0 non-finite, bit1 negative, bit2 asymmetric, bit3 diagonal
  uint32_t r_bits;    // enclosing radius
  uint32_t tau_bits;  // effective threshold
  uint32_t h0_count;  // H0 pairs written
  unsigned long long columns, apparent, nonapparent, candidates, apparent_written, scan_steps;
  unsigned long long facet_steps;  // facets of t whose diameter Condition 2 computed
};

// Where the enumeration kernels (d >= 2) put their records (non-apparent
// columns; apparent pairs when every pair is requested). Every wave appends
// to one of kSinkBuckets regions of `seg` records, each with its own counter
// (counters 128 bytes apart): one shared counter would serialise the appends
// of the whole device on one address. A region that fills up spills into
// the overflow region (ovf_cap records, its counter after the region
// counters). A gather kernel then packs everything into one array and
// stores the total.
constexpr int kSinkBuckets = 256;
constexpr int kSinkStride = 16;  // 64-bit counters per 128 bytes
constexpr size_t kSinkCounters = (size_t)(kSinkBuckets + 1) * kSinkStride;
template <class T>
struct RecordSink {
  T* recs;                    // kSinkBuckets * seg region records, then ovf_cap
  unsigned long long* ctr;    // kSinkCounters entries, zeroed before a launch
  uint64_t seg;
  uint64_t ovf_cap;
};
using ColumnSink = RecordSink<Column>;
using PairSink = RecordSink<ApparentPair>;
// a sink for up to `cap` records: region size (a quarter above the mean
// load, so that regions seldom spill) and records of its buffer
inline uint64_t sink_seg(uint64_t cap) { return (cap + cap / 4) / kSinkBuckets + 64; }
inline uint64_t sink_records(uint64_t cap) { return sink_seg(cap) * kSinkBuckets + cap; }

// The clearing set of one dimension (Alg. 17's cleared columns: deaths and
// apparent cofacets of the dimension below). A bitmap over all C(n, d+1)
// indices where that fits the budget, otherwise an open-addressing hash set
// of the indices (linear probing, at most kClearProbes slots per index; an
// insert that finds no free slot within them sets *overflow and the
// dimension below runs again with a larger table). Exactly one of bits and
// keys is non-null, or neither (nothing cleared).
constexpr unsigned long long kClearEmpty = ~0ull;
constexpr int kClearProbes = 64;
struct ClearSet {
  uint32_t* bits;
  unsigned long long* keys;
  uint64_t mask;        // slots - 1, slots a power of two
  uint32_t* overflow;
};

// The prefixes of a dimension-3 (or 2) enumeration listed explicitly: the
// edges (v_3 > v_2) within the threshold packed v_3 << 16 | v_2 (or the
// vertices v_2), with cum[p] the work units of the prefixes before p (cum has
// count + 1 entries). Used where most vertex pairs are not edges: the
// global-memory kernel then enumerates each prefix's suffixes over common
// neighbours. v == nullptr: every prefix, numbered as in the dense unit
// table.
struct PrefixList {
  const uint64_t* cum;
  const uint32_t* v;
  uint32_t count;
};

// Per-cloud description for the batched kernels.
struct Cloud {
  int64_t x_off;    // first point of the cloud in the packed point array
  int64_t w_off;    // offset of the cloud's n*n weight block
  int64_t e_off;    // first edge of the cloud in the flat edge numbering
  int64_t bm_off;   // first 32-bit word of the cloud's edge-clearing bitmap
  int32_t n;
  uint32_t tau_bits;  // requested threshold (bits); the effective one is stored in CloudState
};

struct CloudState {
  uint32_t r_bits;
  uint32_t tau_bits;
  uint32_t err;
  uint32_t h0_count;
};

// ---- launchers (kernels.hip) ----
hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s);
hipError_t launch_batch_pdist(const float* X, int m, const Cloud* clouds, int count,
                              int64_t total_points, float* D, hipStream_t s);
// Validation of every cloud's D (finite unless allow_inf admits +inf, >= 0,
// zero diagonal, and symmetric unless check_sym is off: D made by pdist is
// symmetric by construction and the check reads columns) with the row
// maxima of the enclosing radius, then the weights W; finite_lower (if not
// null; zeroed by the caller) receives the number of finite weights below
// the diagonal.
hipError_t launch_batch_validate_weights(const float* D, const Cloud* clouds, int count,
                                         int64_t total_points, bool enclosing, uint32_t* W,
                                         CloudState* st, hipStream_t s,
                                         bool allow_inf = false, bool check_sym = true,
                                         unsigned long long* finite_lower = nullptr);
// Sparse input: D (n x n) <- +inf off the diagonal, 0 on it, then the nnz
// given entries in both orientations; input errors are or-ed into st->err.
hipError_t launch_sparse_matrix(const int32_t* row, const int32_t* col, const float* val,
                                int64_t nnz, int n, float* D, CloudState* st, hipStream_t s);
hipError_t launch_batch_h0(const uint32_t* W, const Cloud* clouds, int count, CloudState* st,
                           H0Pair* out, int64_t out_stride, uint32_t* bitmaps, hipStream_t s);
// H0 of one cloud (W: its n x n weights, 1 <= n <= kMaxN) with the Boruvka
// row scans spread over the chip; scratch: h0_wide_scratch_bytes(n) bytes of
// device memory. Same outputs as launch_batch_h0 for that cloud. With
// `edges` (the m finite edges of the lower triangle as launch_finite_edges
// writes them, in any order) the rounds scan that list instead of W's rows.
size_t h0_wide_scratch_bytes(int n);
hipError_t launch_h0_wide(const uint32_t* W, int n, CloudState* st, H0Pair* out, uint32_t* bm,
                          void* scratch, hipStream_t s, const Column* edges = nullptr,
                          int64_t m = 0);
// Rank-matrix variant of the same: Wr holds n rows of lds_stride(n) 16-bit
// weight ranks (0xFFFF above tau_eff, on the diagonal and in the padding
// past column n-1), n <= kLdsMaxN; rank_bits maps a rank to its weight.
// chunk (suffixes per work unit, one wave each) is a positive multiple of 64.
hipError_t launch_enum_apparent_lds(int d, const uint16_t* Wr, const uint32_t* rank_bits, int n,
                                    const uint64_t* binom, int chunk, const uint64_t* unit_cum,
                                    uint64_t units, PrefixList pl, unsigned max_groups,
                                    ClearSet clear_in, ClearSet clear_out, ColumnSink sink,
                                    PairSink aps, Scalars* sc, hipStream_t s);
// The paper's unfused order (measurement only), d = 2 or 3, rank matrix in
// LDS, dense units, bitmap clearing: launch_enum_filter_lds writes every
// column that survives the threshold and clearing set clear_in into sink
// (not tested; counts columns and candidates into sc), and, once those are
// gathered and sorted, launch_apparent_sorted_lds tests the min(*count,
// cap) sorted columns cols, writes the non-apparent ones into sink and sets the
// apparent cofacets' bits in clear_out (a bitmap, or none); grid
// workgroups stride over the columns.
hipError_t launch_enum_filter_lds(int d, const uint16_t* Wr, const uint32_t* rank_bits, int n,
                                  const uint64_t* binom, int chunk, const uint64_t* unit_cum,
                                  uint64_t units, unsigned max_groups, ClearSet clear_in,
                                  ColumnSink sink, Scalars* sc, hipStream_t s);
hipError_t launch_apparent_sorted_lds(int d, const uint16_t* Wr, const uint32_t* rank_bits, int n,
                                      const uint64_t* binom, const Column* cols,
                                      const unsigned long long* count, uint64_t cap,
                                      unsigned grid, ClearSet clear_out, ColumnSink sink,
                                      Scalars* sc, hipStream_t s);
// d >= 2; unit_cum (n+1 entries, device) and units from enum_units() on the
// host; at most max_groups workgroups, which stride over the units
hipError_t launch_enum_apparent(int d, const uint32_t* W, int n, const uint64_t* binom, int chunk,
                                const uint64_t* unit_cum, uint64_t units, PrefixList pl,
                                unsigned max_groups, ClearSet clear_in, ClearSet clear_out,
                                ColumnSink sink, PairSink aps, Scalars* sc, hipStream_t s);
// Pack a sink's records into out (at most out_cap of them) and store their
// total count in *total (more than out_cap: some were not kept).
hipError_t launch_gather_columns(ColumnSink sink, Column* out, uint64_t out_cap,
                                 unsigned long long* total, hipStream_t s);
hipError_t launch_gather_pairs(PairSink sink, ApparentPair* out, uint64_t out_cap,
                               unsigned long long* total, hipStream_t s);
hipError_t launch_batch_edges(const uint32_t* W, const Cloud* clouds, int count,
                              int64_t total_edges, const uint32_t* bitmaps, Column* cols,
                              uint64_t cols_cap, ApparentPair* ap, uint64_t ap_cap,
                              ClearSet clear_out, unsigned long long* counters, int grid,
                              hipStream_t s);
// Dimension-1 columns of one cloud in neighbour mode (sparse complexes): a
// one-wave workgroup per vertex a lists N(a) in LDS and tests the columns
// (a, b), b < a; same outputs as launch_batch_edges with one cloud. bm1: the
// dimension-1 clearing bitmap (the forest edges).
hipError_t launch_edges_nb(const uint32_t* W, int n, const uint32_t* bm1, Column* cols,
                           uint64_t cols_cap, ApparentPair* ap, uint64_t ap_cap,
                           ClearSet clear_out, unsigned long long* counters, int grid,
                           hipStream_t s);
hipError_t launch_set_bits(const uint64_t* idx, int64_t count, uint32_t* bitmap, hipStream_t s);
// Insert count indices into a clearing set (bitmap or hash).
hipError_t launch_clear_insert(const uint64_t* idx, int64_t count, ClearSet set, hipStream_t s);

// GPU scan of an explicit boundary matrix (Alg. 3-6): left/lookup/stable/
// destroyer have n entries, unstable room for n; *count and *err must be
// zero on entry. destroyer[j] = 1 iff column j holds the leftmost 1 of some
// row. Requires n < 2^31.
hipError_t launch_boundary_scan(int64_t n, const int64_t* col_ptr, const int64_t* rows, int64_t nnz,
                                uint32_t* left, int32_t* lookup, uint8_t* stable,
                                uint8_t* destroyer, int64_t* unstable, unsigned long long* count,
                                uint32_t* err, bool clearing, hipStream_t s);
// `bad` (one device word) is set when an edge entry is neither -1 nor in
// [0, n_total); then the scatter reads and writes nothing.
hipError_t launch_backward(const float* X, int64_t n_total, int m, const int32_t* edges,
                           int64_t npairs, const float* g_birth, const float* g_death, float* gX,
                           uint32_t* bad, hipStream_t s);

// ---- reduce_dev.hip ----
// Dimension-1 submatrix reduction on the device, one workgroup per cloud
// of up to kDredThreads lanes.
constexpr int kDredThreads = 1024;
// Per-cloud regions of the device reduction's buffers.
struct DredCloud {
  int64_t tri_off;    // first word of the cloud's triangle bitmap (the working column)
  int64_t tri_words;  // ceil(C(n, 3) / 32)
  int64_t log_off;    // first entry of its log of toggled bitmap words
  int64_t tab_off;    // first slot of its pivot table
  int64_t v_off;      // first entry of its V arena
  int64_t vt_off;     // first entry of its log of toggled V words
  int32_t log_cap, tab_cap, v_cap, vt_cap;
};
// Per-cloud outcome: additions made, columns paired at their first pivot,
// and a nonzero err when a table overflowed (the cloud is then reduced on
// the host instead).
struct DredStats {
  unsigned long long additions;
  uint32_t emergent;
  uint32_t err;
};
struct DredArgs {
  const Cloud* clouds;
  const DredCloud* dc;
  int count;
  const Column* cols;                // non-apparent columns, sorted (cloud, coboundary order)
  const unsigned long long* ncols;   // their number (device)
  uint32_t* col_begin_w;             // per cloud [begin, end) in cols
  uint32_t* col_end_w;
  const uint32_t* col_begin;
  const uint32_t* col_end;
  const uint32_t* epos;              // n x n per cloud: position of the edge, ~0 off edges
  const uint32_t* eat;               // per position: a << 16 | b
  const uint32_t* egrp;              // per position: first position of its weight class
  const uint32_t* egend;             // per position: one past the last position of its class
  const uint32_t* ew;                // per position: weight bits
  uint32_t* cnt;                     // per position: live triangles with that diameter edge
  uint32_t* tri;                     // triangle bitmaps
  uint32_t* tlog;
  unsigned long long* tab_keys;
  uint32_t* tab_vals;
  uint32_t* varena;
  uint32_t* vbits;                   // V bitmaps over edges (Cloud::bm_off layout)
  uint32_t* vtouch;
  unsigned long long* out_death;     // per column: death triangle, ~0 if essential
  uint32_t* out_ddiam;               // death diameter bits (kInf if essential)
  uint32_t* out_dedge;               // death diameter edge a << 16 | b
  uint32_t* col_voff;                // per paired column: its V in the arena
  uint32_t* col_vlen;
  DredStats* stats;                  // per cloud
  const uint32_t* skip;              // per cloud: nonzero = reduced on host threads (null: none)
};
// Edge positions of every cloud: records into rec (total_edges), sorted
// with rec_tmp and sort_work, then ew / eat / egrp / egend per position and
// epos per vertex pair.
hipError_t launch_dred_prepare(const uint32_t* W, const Cloud* clouds, int count,
                               int64_t total_edges, int cloud_bits, Column* rec, Column* rec_tmp,
                               void* sort_work, uint32_t* ew, uint32_t* eat, uint32_t* egrp,
                               uint32_t* egend, uint32_t* epos, hipStream_t s);
// Column ranges per cloud, then the reduction (one workgroup per cloud).
// The bitmaps, counts and V bitmaps must be zero on entry; they are zero
// again on exit.
// threads: the workgroup size per cloud, 256, 512 or 1024 (kDredThreads).
hipError_t launch_dred_reduce(const DredArgs& args, int64_t cols_cap, int max_n, int threads,
                              hipStream_t s);

// ---- graph_ext.hip ----
// Extended persistence of a batch of graphs (Sec. 7.2, Alg. 27-28): v_off /
// e_off are device copies of the count + 1 offsets; lower / upper / tmp
// hold total_edges records; pos_list total_edges, adj_off total_vertices +
// count + 1, adj 2 total_vertices, stack total_vertices entries; err one
// word (nonzero: invalid input, nothing indexed); bars v_off[count] +
// e_off[count] records. Every graph has 1 <= n <= max_n <= kGraphMaxN.
constexpr int kGraphMaxN = 4096;
hipError_t launch_graph_ext(const int64_t* v_off, const int64_t* e_off, int count,
                            int64_t total_vertices, int64_t total_edges, int max_n,
                            const float* f, const int32_t* edges, Column* lower, Column* upper,
                            Column* tmp, void* sort_work, uint32_t* pos_list, uint32_t* adj_off,
                            uint32_t* adj, uint32_t* stack, uint32_t* err, vrph_ext_bar* bars,
                            hipStream_t s);
// The gradient of a loss in the bar values with respect to f: g_f (v_off[
// count] floats, accumulated into) receives g_birth[i] at bar i's birth
// vertex and g_death[i] at its death vertex (either array may be null).
// *bad (zeroed by the caller) is set, and nothing written, if a bar's
// vertices are not in its graph.
hipError_t launch_graph_ext_grad(const int64_t* v_off, const int64_t* e_off, int count,
                                 int64_t nbars, const vrph_ext_bar* bars, const float* g_birth,
                                 const float* g_death, float* g_f, uint32_t* bad, hipStream_t s);

// ---- noalloc.hip ----
// Words of the fixed per-device scratch array of the allocation-free entry
// points (256 bytes): word 0 is the backward's edge-check flag.
constexpr int kNoAllocScratchWords = 64;
// Looks up the scratch array's address on `device`, which must be the
// current device; once per device (later calls return at once).
hipError_t noalloc_scratch_setup(int device);
// The address found by noalloc_scratch_setup, or NULL before it ran.
uint32_t* noalloc_scratch(int device);

// ---- edges.hip ----
// The finite entries of the lower triangle of the n x n weights W, appended
// to `out` as Column{weight bits, 0, a << 32 | b} (a > b) in no particular
// order, at most `cap` of them; *count (zeroed by the caller) receives their
// number, also past `cap`. out = nullptr only counts.
hipError_t launch_finite_edges(const uint32_t* W, int n, Column* out, uint64_t cap,
                               unsigned long long* count, hipStream_t s);

// ---- sort.hip ----
// Stable LSD radix sort of Column records ascending by (cloud, key_hi, cidx),
// looking only at the low `cidx_bits` of cidx, all 32 bits of key_hi and the
// low `cloud_bits` of cloud. `tmp` has room for n records; `work` for
// radix_sort_work_bytes(n) bytes. With n_dev, the count is min(*n_dev, n)
// read on the device (n is then the capacity). The result ends in `a`, or,
// when result_in_tmp is given, possibly in `tmp` (*result_in_tmp says which),
// which avoids a copy node in a recorded graph.
size_t radix_sort_work_bytes(int64_t n);
hipError_t radix_sort_columns(Column* a, Column* tmp, int64_t n, int cidx_bits, int cloud_bits,
                              void* work, hipStream_t s,
                              const unsigned long long* n_dev = nullptr,
                              bool* result_in_tmp = nullptr);
hipError_t launch_init_states(CloudState* st, int count, hipStream_t s);

}  // namespace vrph
