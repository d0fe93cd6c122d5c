// Submatrix reduction of dimension 1 on the device, one workgroup per cloud.
//
// The columns are a cloud's non-apparent edges in coboundary order
// (diameter descending, index ascending; Alg. 18), the rows its triangles.
// Each column is reduced in turn with the reduction-matrix technique of Sec.
// 5.2.9 (R = D V; adding a finished column k adds the coboundaries of its
// edge and of every edge of V_k) and the two-layer pivot lookup of Fig.
// 5.10: first a hash table of the pivots of the columns reduced so far, then
// the apparent pairs, recognised from Def. 5.3.4 on the fly (the pivot t's
// youngest facet of equal diameter, and whether t is that facet's oldest
// cofacet of equal diameter). A column whose first pivot has no owner is
// paired at once without building anything (the emergent case of Sec.
// 5.2.11); otherwise the working column is built and reduced:
//
//  - Edges are numbered by their position in the filtration (weight
//    ascending, index ascending); a triangle's diameter edge is its edge of
//    largest position (among its longest edges, the one with the largest
//    index), the max of epos[a][b] over its three edges. Positions of equal
//    weight form a class [start, end). Keys (class start << 34 | (2^34 - 1
//    - triangle index)) order rows by the filtration: the pivot is the
//    smallest key. A row is not older than the pivot iff its diameter edge
//    lies at or after the end of the pivot's class, or within the class and
//    its triangle index is at most the pivot's.
//  - The working column is a bitmap over the triangle indices (toggled with
//    atomic XOR: Z/2 addition) and a count of live triangles per diameter
//    edge (global) and per 1024 positions (LDS). The pivot only moves up
//    while a column is reduced, so rows below it are never pushed (they
//    cancel in the column added), and the next pivot is found from the
//    counts: the first nonzero block, the first nonzero position in it,
//    then the largest live triangle index over the positions of that weight
//    class, each triangle tested on its diameter edge in parallel.
//  - V of a column is kept as a bitmap over edges; when the column is
//    paired, its set edges are stored in an arena for later additions.
//  - Every toggled word is logged, so that the bitmaps and counts return to
//    zero at the end of each column (or are cleared whole on overflow).
//
// A cloud whose tables overflow is flagged and left to the host reduction.
//
// All of a cloud's state is touched by its own workgroup only (one compute
// unit), so its atomics and coherent loads are workgroup-scoped and
// ordered by the workgroup barrier alone.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vrph_internal.h"

namespace vrph {

namespace {

constexpr uint64_t kTriMask = (1ull << 34) - 1;
constexpr unsigned long long kNoKey = ~0ull;
constexpr uint32_t kNoPos = 0xFFFFFFFFu;           // epos of a pair that is not an edge
constexpr uint32_t kDredMaxAdditions = 1u << 20;  // per column

__device__ __forceinline__ uint64_t c2(uint64_t v) { return v * (v - 1) / 2; }
__device__ __forceinline__ uint64_t c3(uint64_t v) { return v * (v - 1) * (v - 2) / 6; }

// index of triangle {p, q, x}, p > q, x distinct from both (Eq. 5.6)
__device__ __forceinline__ uint64_t tri_index(int p, int q, int x) {
  if (x > p) return c3(x) + c2(p) + (uint64_t)q;
  if (x > q) return c3(p) + c2(x) + (uint64_t)q;
  return c3(p) + c2(q) + (uint64_t)x;
}

__device__ __forceinline__ void edge_of(uint64_t c, int& a, int& b) {
  double r = sqrt(8.0 * (double)c + 1.0);
  int64_t x = (int64_t)((1.0 + r) * 0.5);
  while ((uint64_t)x * (uint64_t)(x - 1) / 2 > c) --x;
  while ((uint64_t)(x + 1) * (uint64_t)x / 2 <= c) ++x;
  a = (int)x;
  b = (int)(c - (uint64_t)x * (uint64_t)(x - 1) / 2);
}

// workgroup-scoped atomics and loads on the cloud's global state
__device__ __forceinline__ uint32_t wg_load(const uint32_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t wg_xor(uint32_t* p, uint32_t v) {
  return __hip_atomic_fetch_xor(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void wg_add(uint32_t* p, uint32_t v) {
  __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ uint32_t wg_exch(uint32_t* p, uint32_t v) {
  return __hip_atomic_exchange(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
  for (int o = 32; o >= 1; o >>= 1) {
    unsigned lo = __shfl_xor((unsigned)v, o), hi = __shfl_xor((unsigned)(v >> 32), o);
    const unsigned long long w = ((unsigned long long)hi << 32) | lo;
    v = w < v ? w : v;
  }
  return v;
}

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
  for (int o = 32; o >= 1; o >>= 1) {
    unsigned lo = __shfl_xor((unsigned)v, o), hi = __shfl_xor((unsigned)(v >> 32), o);
    const unsigned long long w = ((unsigned long long)hi << 32) | lo;
    v = w > v ? w : v;
  }
  return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t w = __shfl_xor(v, o);
    v = w < v ? w : v;
  }
  return v;
}

__device__ __forceinline__ uint64_t table_hash(uint64_t t) { return (t * 0x9E3779B97F4A7C15ull) >> 17; }

// Workgroup-shared state of the reduction kernel.
struct Shared {
  unsigned long long red;       // reduction cell
  uint32_t tv[3];               // vertices of the pivot triangle, v2 > v1 > v0
  int32_t owner;                // -1 free, -2 apparent partner, else global column
  uint32_t partner;             // apparent partner (edge index)
  uint32_t partner_uv;          // its vertices (a << 16 | b)
  uint32_t partner_pos;         // its position
  uint32_t gend;                // end of the pivot's weight class
  uint32_t misc[4];
  uint32_t tlog_n, vt_n, arena_n;
  uint32_t tlog_ovf, vt_ovf;
  uint32_t pmin, pmax;
  uint32_t list_n;
  uint32_t err;
  uint32_t list[kDredThreads];   // positions of a weight class with live triangles
  uint32_t sedge[kDredThreads];  // summand vertices (a << 16 | b)
  uint32_t spos[kDredThreads];   // summand positions
};

// the vertices v2 > v1 > v0 of triangle t (Eq. 5.6): the largest v2 with
// C(v2, 3) <= t (cube root, then an exact fix-up), then the edge t - C(v2, 3)
__device__ __forceinline__ void tri_vertices(uint64_t t, uint32_t* tv) {
  int64_t v2 = (int64_t)cbrt(6.0 * (double)t) + 1;
  while (v2 > 2 && c3((uint64_t)v2) > t) --v2;
  while (c3((uint64_t)v2 + 1) <= t) ++v2;
  int v1, v0;
  edge_of(t - c3((uint64_t)v2), v1, v0);
  tv[0] = (uint32_t)v2;
  tv[1] = (uint32_t)v1;
  tv[2] = (uint32_t)v0;
}

}  // namespace

// ---------------------------------------------------------------------------
// edge positions
// ---------------------------------------------------------------------------

// every vertex pair of every cloud as a record (weight, cloud, local edge
// index) at its flat edge number; non-edges carry kInf and sort last
__global__ void dred_edges_kernel(const uint32_t* __restrict__ W, const Cloud* __restrict__ clouds,
                                  int count, int64_t total_edges, Column* __restrict__ rec) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total_edges;
       g += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = count - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (clouds[mid].e_off <= g)
        lo = mid;
      else
        hi = mid - 1;
    }
    const Cloud cl = clouds[lo];
    const uint64_t local = (uint64_t)(g - cl.e_off);
    int a, b;
    edge_of(local, a, b);
    rec[g] = Column{W[cl.w_off + (int64_t)a * cl.n + b], (uint32_t)lo, local};
  }
}

// after the sort: the weight and the vertices at every position
__global__ void dred_positions_kernel(const Column* __restrict__ srt, int64_t total_edges,
                                      uint32_t* __restrict__ ew, uint32_t* __restrict__ eat) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total_edges;
       g += (int64_t)gridDim.x * blockDim.x) {
    const Column r = srt[g];
    int a, b;
    edge_of(r.cidx, a, b);
    ew[g] = r.key_hi;
    eat[g] = ((uint32_t)a << 16) | (uint32_t)b;
  }
}

// the weight class [start, end) of every position, and epos of every vertex pair
__global__ void dred_groups_kernel(const Column* __restrict__ srt, const Cloud* __restrict__ clouds,
                                   int64_t total_edges, const uint32_t* __restrict__ ew,
                                   uint32_t* __restrict__ egrp, uint32_t* __restrict__ egend,
                                   uint32_t* __restrict__ epos) {
  for (int64_t g = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; g < total_edges;
       g += (int64_t)gridDim.x * blockDim.x) {
    const Column r = srt[g];
    const Cloud cl = clouds[r.cloud];
    const int64_t end = cl.e_off + (int64_t)cl.n * (cl.n - 1) / 2;
    const uint32_t w = ew[g];
    // first and one-past-last position of w among the cloud's (ascending) weights
    int64_t lo = cl.e_off, hi = g;
    while (lo < hi) {
      const int64_t mid = (lo + hi) >> 1;
      if (ew[mid] < w)
        lo = mid + 1;
      else
        hi = mid;
    }
    int64_t lo2 = g + 1, hi2 = end;
    while (lo2 < hi2) {
      const int64_t mid = (lo2 + hi2) >> 1;
      if (ew[mid] <= w)
        lo2 = mid + 1;
      else
        hi2 = mid;
    }
    const uint32_t pos = (uint32_t)(g - cl.e_off);
    egrp[g] = (uint32_t)(lo - cl.e_off);
    egend[g] = (uint32_t)(lo2 - cl.e_off);
    int a, b;
    edge_of(r.cidx, a, b);
    const uint32_t v = w == kInf ? kNoPos : pos;
    epos[cl.w_off + (int64_t)a * cl.n + b] = v;
    epos[cl.w_off + (int64_t)b * cl.n + a] = v;
  }
}

// [begin, end) of every cloud's columns in the sorted column array
__global__ void dred_ranges_kernel(const Column* __restrict__ cols, const unsigned long long* ncols,
                                   int64_t cap, int count, uint32_t* __restrict__ begin,
                                   uint32_t* __restrict__ end) {
  const int64_t n = (int64_t)(*ncols < (unsigned long long)cap ? *ncols : cap);
  for (int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t c = cols[j].cloud;
    if (c >= (uint32_t)count) continue;
    if (j == 0 || cols[j - 1].cloud != c) begin[c] = (uint32_t)j;
    if (j == n - 1 || cols[j + 1].cloud != c) end[c] = (uint32_t)(j + 1);
  }
}

// ---------------------------------------------------------------------------
// the reduction
// ---------------------------------------------------------------------------

// Pushes the coboundaries of the summands sedge[0..m) (positions spos) into
// the working column: every cofacet not older than the pivot (class start
// gstart, class end gend, triangle tp; gend = 0 pushes everything) toggles
// its bit and moves its counts.
template <int T>
__device__ __forceinline__ void push_rows(const DredArgs& A, const Cloud& cl,
                                          const DredCloud& dc, Shared& sh, uint32_t* cnt1, int m,
                                          uint32_t gstart, uint32_t gend, uint64_t tp) {
  const int n = cl.n;
  const int64_t items = (int64_t)m * n;
  const int lane = threadIdx.x & 63;
  for (int64_t base = 0; base < items; base += T) {
    const int64_t it = base + threadIdx.x;
    bool toggled = false;
    uint32_t word = 0, lo = 0xFFFFFFFFu, hi = 0;
    if (it < items) {
      const int i = (int)(it / n), x = (int)(it - (int64_t)i * n);
      const uint32_t e = sh.sedge[i];
      const int p = (int)(e >> 16), q = (int)(e & 0xFFFF);
      const uint32_t e1 = A.epos[cl.w_off + (int64_t)p * n + x];
      const uint32_t e2 = A.epos[cl.w_off + (int64_t)q * n + x];
      uint32_t pm = sh.spos[i] > e1 ? sh.spos[i] : e1;
      pm = pm > e2 ? pm : e2;
      if (pm != kNoPos && pm >= gstart) {
        const uint64_t t = tri_index(p, q, x);
        if (pm >= gend || t <= tp) {
          word = (uint32_t)(t >> 5);
          const uint32_t bit = 1u << (t & 31);
          const uint32_t old = wg_xor(&A.tri[dc.tri_off + word], bit);
          const uint32_t delta = (old & bit) ? 0xFFFFFFFFu : 1u;
          wg_add(&A.cnt[cl.e_off + pm], delta);
          atomicAdd(&cnt1[pm >> 10], delta);
          lo = hi = pm;
          toggled = true;
        }
      }
    }
    // log the toggled words (wave-aggregated slots) and the range of positions touched
    const unsigned long long bal = __ballot(toggled);
    if (bal) {
      for (int o = 32; o >= 1; o >>= 1) {
        const uint32_t l2 = __shfl_xor(lo, o), h2 = __shfl_xor(hi, o);
        lo = l2 < lo ? l2 : lo;
        hi = h2 > hi ? h2 : hi;
      }
      uint32_t first = 0;
      if (lane == 0) {
        first = atomicAdd(&sh.tlog_n, (uint32_t)__popcll(bal));
        atomicMin(&sh.pmin, lo);
        atomicMax(&sh.pmax, hi);
      }
      first = __shfl(first, 0);
      if (toggled) {
        const uint32_t k = first + (uint32_t)__popcll(bal & ((1ull << lane) - 1));
        if (k < (uint32_t)dc.log_cap)
          A.tlog[dc.log_off + k] = word;
        else
          sh.tlog_ovf = 1;
      }
    }
  }
}

// Stages summands [from, from + m) of the current addition: the first is an
// edge index `first`, the others V entries starting at voff. Toggles their
// bits in V of the column being reduced.
template <int T>
__device__ __forceinline__ void stage_summands(const DredArgs& A, const Cloud& cl,
                                               const DredCloud& dc, Shared& sh, int64_t from,
                                               int m, uint32_t first, uint32_t voff) {
  const int lane = threadIdx.x & 63;
  bool toggled = false;
  uint32_t word = 0;
  if ((int)threadIdx.x < m) {
    const int64_t k = from + threadIdx.x;
    const uint32_t e = k == 0 ? first : A.varena[dc.v_off + voff + (uint32_t)(k - 1)];
    int a, b;
    edge_of(e, a, b);
    sh.sedge[threadIdx.x] = ((uint32_t)a << 16) | (uint32_t)b;
    sh.spos[threadIdx.x] = A.epos[cl.w_off + (int64_t)a * cl.n + b];
    word = e >> 5;
    wg_xor(&A.vbits[cl.bm_off + word], 1u << (e & 31));
    toggled = true;
  }
  const unsigned long long bal = __ballot(toggled);
  if (bal) {
    uint32_t f = 0;
    if (lane == 0) f = atomicAdd(&sh.vt_n, (uint32_t)__popcll(bal));
    f = __shfl(f, 0);
    if (toggled) {
      const uint32_t k = f + (uint32_t)__popcll(bal & ((1ull << lane) - 1));
      if (k < (uint32_t)dc.vt_cap)
        A.vtouch[dc.vt_off + k] = word;
      else
        sh.vt_ovf = 1;
    }
  }
}

// The next pivot of the working column (every row in it is younger than the
// current pivot, whose class starts at gstart): returns kNoKey if the column
// is zero; sets sh.tv and sh.gend.
template <int T>
__device__ unsigned long long find_pivot(const DredArgs& A, const Cloud& cl, const DredCloud& dc,
                                         Shared& sh, uint32_t* cnt1, int nblk, int64_t E,
                                         uint32_t gstart) {
  const int n = cl.n;
  // first block holding live rows
  int blk = -1;
  for (int b0 = (int)(gstart >> 10); b0 < nblk; b0 += T) {
    if (threadIdx.x == 0) sh.misc[0] = 0xFFFFFFFFu;
    __syncthreads();
    const int b = b0 + (int)threadIdx.x;
    if (b < nblk && cnt1[b] != 0) atomicMin(&sh.misc[0], (uint32_t)b);
    __syncthreads();
    const uint32_t f = sh.misc[0];
    __syncthreads();
    if (f != 0xFFFFFFFFu) {
      blk = (int)f;
      break;
    }
  }
  if (blk < 0) return kNoKey;
  // the block's counts, classes and edges in one round: the first position
  // p1 >= gstart with live rows (positions below gstart hold none), then the
  // live positions of p1's weight class [g1, gend1) in the block
  if (threadIdx.x == 0) {
    sh.misc[1] = 0xFFFFFFFFu;
    sh.list_n = 0;
    sh.red = 0;
  }
  __syncthreads();
  constexpr int P = 1024 / T;  // positions of the block per lane
  uint32_t cb[P], gb[P], ge[P], uvb[P];
  uint32_t mine = 0xFFFFFFFFu;
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const int64_t pb = (int64_t)blk * 1024 + k * T + threadIdx.x;
    cb[k] = gb[k] = ge[k] = uvb[k] = 0;
    if (pb < E && (uint32_t)pb >= gstart) {
      cb[k] = wg_load(&A.cnt[cl.e_off + pb]);
      gb[k] = A.egrp[cl.e_off + pb];
      ge[k] = A.egend[cl.e_off + pb];
      uvb[k] = A.eat[cl.e_off + pb];
    }
    if (cb[k] != 0 && (uint32_t)pb < mine) mine = (uint32_t)pb;
  }
  {
    const uint32_t wmin = wave_min_u32(mine);
    if ((threadIdx.x & 63) == 0 && wmin != 0xFFFFFFFFu) atomicMin(&sh.misc[1], wmin);
  }
  __syncthreads();
  const uint32_t p1 = sh.misc[1];
  if (p1 == 0xFFFFFFFFu) {  // counts out of step: leave the cloud to the host
    if (threadIdx.x == 0) sh.err = 3;
    __syncthreads();
    return kNoKey;
  }
#pragma unroll
  for (int k = 0; k < P; ++k)
    if ((uint32_t)((int64_t)blk * 1024 + k * T + threadIdx.x) == p1) {
      sh.misc[2] = gb[k];
      sh.misc[3] = ge[k];
    }
  __syncthreads();
  const uint32_t g1 = sh.misc[2], gend1 = sh.misc[3];
#pragma unroll
  for (int k = 0; k < P; ++k) {
    const uint32_t pb = (uint32_t)((int64_t)blk * 1024 + k * T + threadIdx.x);
    if (cb[k] != 0 && pb >= p1 && pb < gend1) {
      const uint32_t q = atomicAdd(&sh.list_n, 1u);
      sh.list[q] = pb;
      sh.sedge[q] = uvb[k];  // free here: staging starts after the search
    }
  }
  // the largest live triangle index over the listed positions; a class that
  // runs past the block continues one window of T positions at a time
  for (int64_t w0 = (int64_t)blk * 1024 + 1024;; w0 += T) {
    __syncthreads();
    const int L = (int)sh.list_n;
    const int64_t items = (int64_t)L * n;
    unsigned long long best = 0;
    for (int64_t it = threadIdx.x; it < items; it += T) {
      const int i = (int)(it / n), x = (int)(it - (int64_t)i * n);
      const uint32_t pos = sh.list[i];
      const uint32_t uv = sh.sedge[i];
      const int u = (int)(uv >> 16), v = (int)(uv & 0xFFFF);
      const uint32_t e1 = A.epos[cl.w_off + (int64_t)u * n + x];
      const uint32_t e2 = A.epos[cl.w_off + (int64_t)v * n + x];
      if (e1 < pos && e2 < pos) {  // (u, v) is the diameter edge of {u, v, x}
        const uint64_t t = tri_index(u, v, x);
        const uint32_t wd = wg_load(&A.tri[dc.tri_off + (t >> 5)]);
        if ((wd >> (t & 31)) & 1u) best = t + 1 > best ? t + 1 : best;
      }
    }
    best = wave_max_u64(best);
    if ((threadIdx.x & 63) == 0 && best) atomicMax(&sh.red, best);
    if (w0 >= (int64_t)gend1) break;
    __syncthreads();
    if (threadIdx.x == 0) sh.list_n = 0;
    __syncthreads();
    const int64_t p = w0 + threadIdx.x;
    if (p < (int64_t)gend1 && wg_load(&A.cnt[cl.e_off + p]) != 0) {
      const uint32_t k = atomicAdd(&sh.list_n, 1u);
      sh.list[k] = (uint32_t)p;
      sh.sedge[k] = A.eat[cl.e_off + p];
    }
  }
  __syncthreads();
  const unsigned long long best = sh.red;
  __syncthreads();
  if (best == 0) {  // no live triangle where the counts said: leave the cloud to the host
    if (threadIdx.x == 0) sh.err = 4;
    __syncthreads();
    return kNoKey;
  }
  const uint64_t t = best - 1;
  if (threadIdx.x == 0) {
    tri_vertices(t, sh.tv);
    sh.gend = gend1;
  }
  __syncthreads();
  return ((unsigned long long)g1 << 34) | (kTriMask - t);
}

// Owner of the pivot t = sh.tv with key `key` (class [gD, sh.gend)): sets
// sh.owner (global column of a finished column, -2 for an apparent partner
// in sh.partner, -1 free).
template <int T>
__device__ void find_owner(const DredArgs& A, const Cloud& cl, const DredCloud& dc, Shared& sh,
                           uint32_t tcap, unsigned long long key) {
  const int n = cl.n;
  const uint64_t t = kTriMask - (key & kTriMask);
  const uint32_t gD = (uint32_t)(key >> 34), gendD = sh.gend;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (threadIdx.x == 0) {
    sh.owner = -1;
    sh.misc[2] = 0;
  }
  __syncthreads();
  if (wave == 0) {
    // the table of finished columns' pivots (linear probing)
    uint64_t h = table_hash(t) & (tcap - 1);
    for (uint32_t probed = 0; probed < tcap; probed += 64) {
      const uint64_t sl = (h + lane) & (tcap - 1);
      const unsigned long long k = A.tab_keys[dc.tab_off + sl];
      const unsigned long long hit = __ballot(k == t), empty = __ballot(k == kNoKey);
      if (hit && (!empty || __ffsll(hit) < __ffsll(empty))) {
        const int src = __ffsll(hit) - 1;
        if (lane == src) sh.owner = (int32_t)A.tab_vals[dc.tab_off + sl];
        break;
      }
      if (empty) break;
      h = (h + 64) & (tcap - 1);
    }
  } else {
    // Def. 5.3.4: s = the facet of t of smallest index with t's diameter
    // (its edge lies in t's class); apparent iff no x above t's third vertex
    // makes an equal-diameter cofacet of s (t is then s's oldest cofacet of
    // that diameter). The rows of all three vertices are read at once, before
    // s is known.
    const int v2 = (int)sh.tv[0], v1 = (int)sh.tv[1], v0 = (int)sh.tv[2];
    const int64_t wo = cl.w_off;
    const uint32_t f10 = A.epos[wo + (int64_t)v1 * n + v0];
    const uint32_t f20 = A.epos[wo + (int64_t)v2 * n + v0];
    const uint32_t f21 = A.epos[wo + (int64_t)v2 * n + v1];
    const int x0 = v0 + 1 + (int)threadIdx.x - 64, stride = T - 64;
    uint32_t r2[4], r1[4], r0[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int x = x0 + k * stride;
      const bool ok = x < n;
      r2[k] = ok ? A.epos[wo + (int64_t)v2 * n + x] : kNoPos;
      r1[k] = ok ? A.epos[wo + (int64_t)v1 * n + x] : kNoPos;
      r0[k] = ok ? A.epos[wo + (int64_t)v0 * n + x] : kNoPos;
    }
    int p, q, r, which;
    uint32_t fpq;
    if (f10 >= gD) {
      p = v1; q = v0; r = v2; which = 0; fpq = f10;
    } else if (f20 >= gD) {
      p = v2; q = v0; r = v1; which = 1; fpq = f20;
    } else {
      p = v2; q = v1; r = v0; which = 2; fpq = f21;
    }
    bool older = false;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int x = x0 + k * stride;
      const uint32_t ep = which == 0 ? r1[k] : r2[k];
      const uint32_t eq = which == 2 ? r1[k] : r0[k];
      older |= x > r && x != p && x != q && ep < gendD && eq < gendD;
    }
    for (int x = x0 + 4 * stride; x < n; x += stride) {  // n > 3904 only
      if (x <= r || x == p || x == q) continue;
      const uint32_t ep = A.epos[wo + (int64_t)p * n + x];
      const uint32_t eq = A.epos[wo + (int64_t)q * n + x];
      older |= ep < gendD && eq < gendD;
    }
    if (__ballot(older) && lane == 0) sh.misc[2] = 1;
    if (threadIdx.x == 64) {
      sh.partner = (uint32_t)(c2((uint64_t)p) + (uint64_t)q);
      sh.partner_uv = ((uint32_t)p << 16) | (uint32_t)q;
      sh.partner_pos = fpq;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0 && sh.owner < 0 && sh.misc[2] == 0) sh.owner = -2;
  __syncthreads();
}

template <int T>
__global__ __launch_bounds__(T) void dred_reduce_kernel(DredArgs A) {
  extern __shared__ uint32_t cnt1[];
  __shared__ Shared sh;
  const int c = blockIdx.x;
  if (A.skip && A.skip[c]) {  // the host reduces this cloud (same value for the whole workgroup)
    if (threadIdx.x == 0) A.stats[c] = DredStats{0, 0, 0};
    return;
  }
  const Cloud cl = A.clouds[c];
  const DredCloud dc = A.dc[c];
  const int n = cl.n;
  const int64_t E = (int64_t)n * (n - 1) / 2;
  const int nblk = (int)((E + 1023) / 1024);
  const int tid = threadIdx.x;
  for (int b = tid; b < nblk; b += T) cnt1[b] = 0;
  const uint32_t jb = A.col_begin[c], je = A.col_end[c];
  const uint32_t ncol = je > jb ? je - jb : 0;
  uint32_t tcap = 64;
  while (tcap < 2 * ncol) tcap <<= 1;
  if (tid == 0) {
    sh.arena_n = 0;
    sh.err = tcap > (uint32_t)dc.tab_cap ? 1u : 0u;
    sh.tv[0] = sh.tv[1] = sh.tv[2] = 0;
    sh.gend = 0;
  }
  __syncthreads();
  if (sh.err) {
    if (tid == 0) A.stats[c] = DredStats{0, 0, sh.err};
    return;
  }
  for (uint32_t s = tid; s < tcap; s += T) A.tab_keys[dc.tab_off + s] = kNoKey;
  __syncthreads();
  unsigned long long additions = 0;
  uint32_t emergent = 0;

  for (uint32_t j = jb; j < je && !sh.err; ++j) {
    const uint64_t scidx = A.cols[j].cidx;
    int a, b;
    edge_of(scidx, a, b);
    const uint32_t es = A.epos[cl.w_off + (int64_t)a * n + b];
    // the first pivot, from the coboundary alone: the oldest cofacet, i.e.
    // the smallest diameter-edge position's class, then the largest index
    uint32_t pmin = kNoPos;
    for (int x = tid; x < n; x += T) {
      const uint32_t e1 = A.epos[cl.w_off + (int64_t)a * n + x];
      const uint32_t e2 = A.epos[cl.w_off + (int64_t)b * n + x];
      uint32_t pm = es > e1 ? es : e1;
      pm = pm > e2 ? pm : e2;
      pmin = pm < pmin ? pm : pmin;
    }
    pmin = wave_min_u32(pmin);
    if (tid == 0) sh.misc[0] = kNoPos;
    __syncthreads();
    if ((tid & 63) == 0 && pmin != kNoPos) atomicMin(&sh.misc[0], pmin);
    __syncthreads();
    const uint32_t p0 = sh.misc[0];
    if (p0 == kNoPos) {  // no cofacet within the threshold: an essential class
      if (tid == 0) {
        A.out_death[j] = kNoKey;
        A.out_ddiam[j] = kInf;
        A.out_dedge[j] = kInf;
        A.col_vlen[j] = 0;
      }
      __syncthreads();
      continue;
    }
    const uint32_t g0 = A.egrp[cl.e_off + p0], gend0 = A.egend[cl.e_off + p0];
    unsigned long long tbest = 0;
    for (int x = tid; x < n; x += T) {
      const uint32_t e1 = A.epos[cl.w_off + (int64_t)a * n + x];
      const uint32_t e2 = A.epos[cl.w_off + (int64_t)b * n + x];
      uint32_t pm = es > e1 ? es : e1;
      pm = pm > e2 ? pm : e2;
      if (pm != kNoPos && pm < gend0) {
        const unsigned long long t = tri_index(a, b, x) + 1;
        tbest = t > tbest ? t : tbest;
      }
    }
    tbest = wave_max_u64(tbest);
    if (tid == 0) sh.red = 0;
    __syncthreads();
    if ((tid & 63) == 0 && tbest) atomicMax(&sh.red, tbest);
    __syncthreads();
    unsigned long long key = ((unsigned long long)g0 << 34) | (kTriMask - (sh.red - 1));
    if (tid == 0) {
      tri_vertices(sh.red - 1, sh.tv);
      sh.gend = gend0;
      sh.tlog_n = sh.vt_n = 0;
      sh.tlog_ovf = sh.vt_ovf = 0;
      sh.pmin = 0xFFFFFFFFu;
      sh.pmax = 0;
    }
    __syncthreads();
    bool built = false;
    uint32_t nadd = 0;
    for (;;) {
      find_owner<T>(A, cl, dc, sh, tcap, key);
      const int32_t owner = sh.owner;
      if (owner == -1) break;  // a free pivot: the column is paired with it
      if (!built) {
        // the working column: the coboundary of the column's own edge
        if (tid == 0) {
          sh.sedge[0] = ((uint32_t)a << 16) | (uint32_t)b;
          sh.spos[0] = es;
        }
        __syncthreads();
        push_rows<T>(A, cl, dc, sh, cnt1, 1, 0, 0, 0);
        built = true;
      }
      // add the owner's column: its edge, then V (finished columns only)
      const uint32_t gstart = (uint32_t)(key >> 34), gend = sh.gend;
      const uint64_t tp = kTriMask - (key & kTriMask);
      if (owner == -2) {
        // an apparent column: its edge, known from the lookup
        __syncthreads();
        if (tid == 0) {
          const uint32_t e = sh.partner;
          sh.sedge[0] = sh.partner_uv;
          sh.spos[0] = sh.partner_pos;
          wg_xor(&A.vbits[cl.bm_off + (e >> 5)], 1u << (e & 31));
          const uint32_t k = sh.vt_n++;
          if (k < (uint32_t)dc.vt_cap)
            A.vtouch[dc.vt_off + k] = e >> 5;
          else
            sh.vt_ovf = 1;
        }
        __syncthreads();
        push_rows<T>(A, cl, dc, sh, cnt1, 1, gstart, gend, tp);
      } else {
        const uint32_t first = (uint32_t)A.cols[owner].cidx;
        const uint32_t voff = A.col_voff[owner], vlen = A.col_vlen[owner];
        const int64_t total = 1 + (int64_t)vlen;
        for (int64_t from = 0; from < total; from += T) {
          const int m = (int)(total - from < T ? total - from : T);
          __syncthreads();
          stage_summands<T>(A, cl, dc, sh, from, m, first, voff);
          __syncthreads();
          push_rows<T>(A, cl, dc, sh, cnt1, m, gstart, gend, tp);
        }
      }
      ++nadd;
      __syncthreads();
      const unsigned long long prev = key;
      key = find_pivot<T>(A, cl, dc, sh, cnt1, nblk, E, gstart);
      if (key == kNoKey) break;  // the column is zero: an essential class
      // an addition cancels the pivot, so the next one is younger; a column
      // that would not move on, or that needs more additions than a column
      // is given here, goes to the host
      if (key <= prev || nadd >= kDredMaxAdditions) {
        if (tid == 0) sh.err = key <= prev ? 5u : 6u;
        __syncthreads();
        key = kNoKey;
        break;
      }
    }
    additions += nadd;
    const bool paired = key != kNoKey;
    if (paired && nadd == 0) ++emergent;
    if (tid == 0) {
      if (paired) {
        const uint64_t t = kTriMask - (key & kTriMask);
        const uint32_t gD = (uint32_t)(key >> 34);
        A.out_death[j] = t;
        A.out_ddiam[j] = A.ew[cl.e_off + gD];
        // diameter edge: the largest position among the three edges
        const int v2 = (int)sh.tv[0], v1 = (int)sh.tv[1], v0 = (int)sh.tv[2];
        const uint32_t x0 = A.epos[cl.w_off + (int64_t)v2 * n + v1];
        const uint32_t x1 = A.epos[cl.w_off + (int64_t)v2 * n + v0];
        const uint32_t x2 = A.epos[cl.w_off + (int64_t)v1 * n + v0];
        uint32_t de = ((uint32_t)v2 << 16) | (uint32_t)v1, m = x0;
        if (x1 > m) { m = x1; de = ((uint32_t)v2 << 16) | (uint32_t)v0; }
        if (x2 > m) { de = ((uint32_t)v1 << 16) | (uint32_t)v0; }
        A.out_dedge[j] = de;
      } else {
        A.out_death[j] = kNoKey;
        A.out_ddiam[j] = kInf;
        A.out_dedge[j] = kInf;
      }
      sh.misc[3] = sh.arena_n;
    }
    __syncthreads();
    // V of the column: the edges whose bits are set, moved to the arena (and
    // the bits cleared)
    const uint32_t vstart = sh.misc[3];
    if (nadd > 0) {
      const bool full = sh.vt_ovf != 0;
      const int64_t words = full ? (E + 31) / 32 : (int64_t)sh.vt_n;
      for (int64_t k = tid; k < words; k += T) {
        const uint32_t wdi = full ? (uint32_t)k : A.vtouch[dc.vt_off + k];
        const uint32_t bits = wg_exch(&A.vbits[cl.bm_off + wdi], 0u);
        if (bits && paired) {
          const uint32_t at = atomicAdd(&sh.arena_n, (uint32_t)__popc(bits));
          uint32_t bb = bits;
          for (uint32_t o = at; bb; ++o, bb &= bb - 1) {
            if (o < (uint32_t)dc.v_cap)
              A.varena[dc.v_off + o] = wdi * 32 + (uint32_t)(__ffs(bb) - 1);
            else
              sh.err = 2;
          }
        }
      }
    }
    __syncthreads();
    if (tid == 0) {
      A.col_voff[j] = vstart;
      A.col_vlen[j] = paired ? sh.arena_n - vstart : 0;
    }
    // the pivot goes into the table
    if (paired && tid < 64) {
      const uint64_t t = kTriMask - (key & kTriMask);
      uint64_t h = table_hash(t) & (tcap - 1);
      for (uint32_t probed = 0; probed < tcap; probed += 64) {
        const uint64_t sl = (h + tid) & (tcap - 1);
        const unsigned long long empty = __ballot(A.tab_keys[dc.tab_off + sl] == kNoKey);
        if (empty) {
          if (tid == __ffsll(empty) - 1) {
            A.tab_keys[dc.tab_off + sl] = t;
            A.tab_vals[dc.tab_off + sl] = j;
          }
          break;
        }
        h = (h + 64) & (tcap - 1);
      }
    }
    // the working column back to zero
    if (built) {
      if (sh.tlog_ovf) {
        for (int64_t k = tid; k < dc.tri_words; k += T) A.tri[dc.tri_off + k] = 0;
      } else {
        for (uint32_t k = tid; k < sh.tlog_n; k += T) A.tri[dc.tri_off + A.tlog[dc.log_off + k]] = 0;
      }
      const uint32_t q0 = sh.pmin, q1 = sh.pmax;
      if (q0 <= q1) {
        for (int64_t p = (int64_t)q0 + tid; p <= (int64_t)q1; p += T) A.cnt[cl.e_off + p] = 0;
        for (int b2 = (int)(q0 >> 10) + tid; b2 <= (int)(q1 >> 10); b2 += T) cnt1[b2] = 0;
      }
    }
    __syncthreads();
  }
  if (tid == 0) A.stats[c] = DredStats{additions, emergent, sh.err};
}

hipError_t launch_dred_prepare(const uint32_t* W, const Cloud* clouds, int count,
                               int64_t total_edges, int cloud_bits, Column* rec, Column* rec_tmp,
                               void* sort_work, uint32_t* ew, uint32_t* eat, uint32_t* egrp,
                               uint32_t* egend, uint32_t* epos, hipStream_t s) {
  if (total_edges <= 0) return hipSuccess;
  int64_t blocks = (total_edges + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  dred_edges_kernel<<<(int)blocks, kBlock, 0, s>>>(W, clouds, count, total_edges, rec);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  bool in_tmp = false;
  // stable: equal weights keep the ascending edge index they were written in
  e = radix_sort_columns(rec, rec_tmp, total_edges, 0, cloud_bits, sort_work, s, nullptr, &in_tmp);
  if (e != hipSuccess) return e;
  const Column* srt = in_tmp ? rec_tmp : rec;
  dred_positions_kernel<<<(int)blocks, kBlock, 0, s>>>(srt, total_edges, ew, eat);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  dred_groups_kernel<<<(int)blocks, kBlock, 0, s>>>(srt, clouds, total_edges, ew, egrp, egend,
                                                    epos);
  return hipGetLastError();
}

hipError_t launch_dred_reduce(const DredArgs& args, int64_t cols_cap, int max_n, int threads,
                              hipStream_t s) {
  hipError_t e = launch_fill_u32(args.col_begin_w, args.count, 0u, s);
  if (e != hipSuccess) return e;
  if ((e = launch_fill_u32(args.col_end_w, args.count, 0u, s)) != hipSuccess) return e;
  int64_t blocks = (cols_cap + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  if (blocks < 1) blocks = 1;
  dred_ranges_kernel<<<(int)blocks, kBlock, 0, s>>>(args.cols, args.ncols, cols_cap, args.count,
                                                    args.col_begin_w, args.col_end_w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const int64_t emax = (int64_t)max_n * (max_n - 1) / 2;
  const size_t lds = (size_t)((emax + 1023) / 1024) * sizeof(uint32_t);
  switch (threads) {
    case 256:
      dred_reduce_kernel<256><<<args.count, 256, lds, s>>>(args);
      break;
    case 512:
      dred_reduce_kernel<512><<<args.count, 512, lds, s>>>(args);
      break;
    case 1024:
      dred_reduce_kernel<1024><<<args.count, 1024, lds, s>>>(args);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace vrph
