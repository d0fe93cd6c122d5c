// HIP kernels of the Vietoris–Rips hot path for gfx950 (wave64).
//
// Stages (Zhang, Ch. 5): distances (Def. 5.1.1), enclosing radius
// (Sec. 5.2.12), H0 by a minimum spanning forest and union-find with the
// elder rule (Sec. 5.2.5), and per dimension d >= 1 the enumeration of
// d-simplices in the combinatorial number system (Eq. 5.6) with threshold
// and clearing (Alg. 17) fused with the apparent-pairs test (Lemma 5.3.6,
// Alg. 13). Every column is tested independently (Cor. 5.3.7) and clearing
// does not change the apparent set (Prop. 5.3.9), so the test runs on the
// enumerated candidates directly and only the few non-apparent columns are
// compacted for the coboundary-order sort and the host reduction.
#include <hip/hip_runtime.h>

#include <type_traits>

#include <cstdint>

#include "vrph_internal.h"

namespace vrph {

// ---------------------------------------------------------------------------
// small device helpers
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint32_t float_key(float x) {
  // +0.0 and -0.0 compare equal; give both the pattern of +0.0
  return x == 0.0f ? 0u : __float_as_uint(x);
}

__device__ __forceinline__ unsigned long long shfl_u64(unsigned long long x, int src) {
  unsigned lo = (unsigned)x, hi = (unsigned)(x >> 32);
  lo = __shfl(lo, src);
  hi = __shfl(hi, src);
  return ((unsigned long long)hi << 32) | lo;
}

__device__ __forceinline__ unsigned long long shfl_xor_u64(unsigned long long x, int m) {
  unsigned lo = (unsigned)x, hi = (unsigned)(x >> 32);
  lo = __shfl_xor(lo, m);
  hi = __shfl_xor(hi, m);
  return ((unsigned long long)hi << 32) | lo;
}

// Edge index C(a,2) + b (a > b) and its inverse.
__device__ __forceinline__ uint64_t edge_index(int a, int b) {
  return (uint64_t)a * (uint64_t)(a - 1) / 2 + (uint64_t)b;
}

__device__ __forceinline__ void edge_vertices(uint64_t c, int& a, int& b) {
  // largest a with a(a-1)/2 <= c, from the square root and a one-step fix-up
  double r = sqrt(8.0 * (double)c + 1.0);
  int64_t x = (int64_t)((1.0 + r) * 0.5);
  while ((uint64_t)x * (uint64_t)(x - 1) / 2 > c) --x;
  while ((uint64_t)(x + 1) * (uint64_t)x / 2 <= c) ++x;
  a = (int)x;
  b = (int)(c - (uint64_t)x * (uint64_t)(x - 1) / 2);
}

// ---- clearing sets (bitmap or hash, see ClearSet) ----
__device__ __forceinline__ uint64_t clear_slot(const ClearSet& cs, uint64_t c) {
  return (c * 0x9E3779B97F4A7C15ull) >> 20 & cs.mask;  // multiplicative hash
}
__device__ __forceinline__ bool clear_contains(const ClearSet& cs, uint64_t c) {
  if (cs.bits) return (cs.bits[c >> 5] >> (c & 31)) & 1u;
  if (!cs.keys) return false;
  uint64_t sl = clear_slot(cs, c);
  for (int i = 0; i < kClearProbes; ++i, sl = (sl + 1) & cs.mask) {
    const unsigned long long k = cs.keys[sl];
    if (k == c) return true;
    if (k == kClearEmpty) return false;
  }
  return false;  // never inserted: an insert stays within kClearProbes slots
}
__device__ __forceinline__ void clear_insert(const ClearSet& cs, uint64_t c) {
  if (cs.bits) {
    atomicOr(&cs.bits[c >> 5], 1u << (c & 31));
    return;
  }
  if (!cs.keys) return;
  uint64_t sl = clear_slot(cs, c);
  for (int i = 0; i < kClearProbes; ++i, sl = (sl + 1) & cs.mask) {
    const unsigned long long prev = atomicCAS(&cs.keys[sl], kClearEmpty, (unsigned long long)c);
    if (prev == kClearEmpty || prev == c) return;
  }
  atomicExch(cs.overflow, 1u);
}

__device__ __forceinline__ int find_cloud(const Cloud* clouds, int count, int64_t key,
                                          int64_t Cloud::*field) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (clouds[mid].*field <= key)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

// ---------------------------------------------------------------------------
// fill
// ---------------------------------------------------------------------------

__global__ void fill_u32_kernel(uint32_t* p, int64_t count, uint32_t v) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

__global__ void init_states_kernel(CloudState* st, int count) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
    st[i].r_bits = kInf;
    st[i].tau_bits = 0;
    st[i].err = 0;
    st[i].h0_count = 0;
  }
}

hipError_t launch_init_states(CloudState* st, int count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  init_states_kernel<<<(count + kBlock - 1) / kBlock, kBlock, 0, s>>>(st, count);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, int64_t count, uint32_t v, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  fill_u32_kernel<<<(int)blocks, kBlock, 0, s>>>(p, count, v);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// distances (Def. 5.1.1): binary64 differences, squares, left-to-right sum and
// square root, one rounding to float32 (compiled with -ffp-contract=off).
// One workgroup per point (row); rows of all clouds are numbered together.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void batch_pdist_kernel(const float* __restrict__ X, int m,
                                                             const Cloud* __restrict__ clouds,
                                                             int count, float* __restrict__ D) {
  const int64_t row = blockIdx.x;
  const int c = find_cloud(clouds, count, row, &Cloud::x_off);
  const Cloud cl = clouds[c];
  const int i = (int)(row - cl.x_off);
  const float* xi = X + (cl.x_off + i) * (int64_t)m;
  for (int j = threadIdx.x; j < cl.n; j += blockDim.x) {
    const float* xj = X + (cl.x_off + j) * (int64_t)m;
    double s = 0.0;
    for (int k = 0; k < m; ++k) {
      double d = (double)xi[k] - (double)xj[k];
      double sq = d * d;
      s = s + sq;
    }
    D[cl.w_off + (int64_t)i * cl.n + j] = (float)sqrt(s);
  }
}

hipError_t launch_batch_pdist(const float* X, int m, const Cloud* clouds, int count,
                              int64_t total_points, float* D, hipStream_t s) {
  if (total_points <= 0) return hipSuccess;
  if (total_points > kMaxGroups) return hipErrorInvalidValue;
  batch_pdist_kernel<<<(unsigned)total_points, kBlock, 0, s>>>(X, m, clouds, count, D);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// validation and enclosing radius (Sec. 5.2.12): R = min_i max_j D_ij.
// Max and min are order-free, so the float-bit atomics are deterministic.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void batch_validate_kernel(const float* __restrict__ D,
                                                                const Cloud* __restrict__ clouds,
                                                                int count,
                                                                CloudState* __restrict__ st,
                                                                int allow_inf, int check_sym) {
  __shared__ uint32_t red[kBlock / 64];
  __shared__ uint32_t errs;
  const int64_t row = blockIdx.x;
  const int c = find_cloud(clouds, count, row, &Cloud::x_off);
  const Cloud cl = clouds[c];
  const int i = (int)(row - cl.x_off);
  const float* Drow = D + cl.w_off + (int64_t)i * cl.n;
  if (threadIdx.x == 0) errs = 0;
  __syncthreads();
  uint32_t mx = 0, err = 0;
  for (int j = threadIdx.x; j < cl.n; j += blockDim.x) {
    float x = Drow[j];
    // a sparse matrix holds +inf where a pair is not an edge; it then also
    // takes part in the row maximum of the enclosing radius
    if (!isfinite(x) && !(allow_inf && x == INFINITY)) err |= 1u;
    if (x < 0.0f) err |= 2u;
    // (column reads: skipped where D is pdist's own output, symmetric by
    // construction)
    if (check_sym && x != D[cl.w_off + (int64_t)j * cl.n + i]) err |= 4u;
    if (j == i && x != 0.0f) err |= 8u;
    uint32_t k = float_key(x);
    if (!isnan(x) && x >= 0.0f && k > mx) mx = k;
  }
  for (int o = 32; o > 0; o >>= 1) mx = max(mx, (uint32_t)__shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = mx;
  if (err) atomicOr(&errs, err);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t m2 = red[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m2 = max(m2, red[w]);
    atomicMin(&st[c].r_bits, m2);
    if (errs) atomicOr(&st[c].err, errs);
  }
}

// Weights: W_ij = bits(D_ij) if i != j and D_ij <= tau_eff, else kInf.
__global__ __launch_bounds__(kBlock) void batch_weights_kernel(const float* __restrict__ D,
                                                               const Cloud* __restrict__ clouds,
                                                               int count, int enclosing,
                                                               uint32_t* __restrict__ W,
                                                               CloudState* __restrict__ st,
                                                               unsigned long long* __restrict__ finite_lower) {
  __shared__ uint32_t lower[kBlock / 64];
  const int64_t row = blockIdx.x;
  const int c = find_cloud(clouds, count, row, &Cloud::x_off);
  const Cloud cl = clouds[c];
  const int i = (int)(row - cl.x_off);
  uint32_t tau = cl.tau_bits;
  if (enclosing) tau = min(tau, st[c].r_bits);
  if (i == 0 && threadIdx.x == 0) st[c].tau_bits = tau;
  const float* Drow = D + cl.w_off + (int64_t)i * cl.n;
  uint32_t* Wrow = W + cl.w_off + (int64_t)i * cl.n;
  uint32_t fin = 0;  // finite entries left of the diagonal
  for (int j = threadIdx.x; j < cl.n; j += blockDim.x) {
    uint32_t k = float_key(Drow[j]);
    // +inf (a pair that is not an edge of a sparse matrix) is never an edge
    const bool edge = j != i && k <= tau && k < 0x7F800000u;
    Wrow[j] = edge ? k : kInf;
    fin += (edge && j < i) ? 1u : 0u;
  }
  if (finite_lower) {
    for (int o = 32; o > 0; o >>= 1) fin += (uint32_t)__shfl_xor(fin, o);
    if ((threadIdx.x & 63) == 0) lower[threadIdx.x >> 6] = fin;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += lower[w];
      if (t) atomicAdd(finite_lower, (unsigned long long)t);
    }
  }
}

hipError_t launch_batch_validate_weights(const float* D, const Cloud* clouds, int count,
                                         int64_t total_points, bool enclosing, uint32_t* W,
                                         CloudState* st, hipStream_t s, bool allow_inf,
                                         bool check_sym, unsigned long long* finite_lower) {
  if (total_points <= 0) return hipSuccess;
  if (total_points > kMaxGroups) return hipErrorInvalidValue;
  batch_validate_kernel<<<(unsigned)total_points, kBlock, 0, s>>>(D, clouds, count, st,
                                                                  allow_inf ? 1 : 0,
                                                                  check_sym ? 1 : 0);
  batch_weights_kernel<<<(unsigned)total_points, kBlock, 0, s>>>(D, clouds, count,
                                                                 enclosing ? 1 : 0, W, st,
                                                                 finite_lower);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sparse input: the n x n matrix with +inf where a pair is not given and 0 on
// the diagonal, then the given entries in both orientations. A repeated pair
// finds a finite value already in one of its two cells (both writes are
// exchanges, so of two writers to a cell the second sees the first). Errors
// go to st->err: bit 0 a value that is not finite, bit 1 a negative value,
// bit 4 an index out of range or on the diagonal, bit 5 a repeated pair.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void sparse_init_kernel(float* __restrict__ D, int n) {
  const int64_t nn = (int64_t)n * n;
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < nn;
       q += (int64_t)gridDim.x * kBlock)
    D[q] = (q / n == q % n) ? 0.0f : INFINITY;
}

__global__ __launch_bounds__(kBlock) void sparse_fill_kernel(const int32_t* __restrict__ row,
                                                             const int32_t* __restrict__ col,
                                                             const float* __restrict__ val,
                                                             int64_t nnz, int n,
                                                             float* __restrict__ D,
                                                             CloudState* __restrict__ st) {
  const uint32_t inf_bits = 0x7F800000u;
  uint32_t* const Db = reinterpret_cast<uint32_t*>(D);
  for (int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x; q < nnz;
       q += (int64_t)gridDim.x * kBlock) {
    const int i = row[q], j = col[q];
    const float v = val[q];
    uint32_t err = 0;
    if (i < 0 || i >= n || j < 0 || j >= n || i == j) err |= 16u;
    if (!isfinite(v)) err |= 1u;
    if (v < 0.0f) err |= 2u;
    if (!err) {
      const uint32_t b = __float_as_uint(v == 0.0f ? 0.0f : v);  // -0 stored as +0
      const uint32_t p1 = atomicExch(&Db[(int64_t)i * n + j], b);
      const uint32_t p2 = atomicExch(&Db[(int64_t)j * n + i], b);
      if (p1 != inf_bits || p2 != inf_bits) err |= 32u;
    }
    if (err) atomicOr(&st->err, err);
  }
}

hipError_t launch_sparse_matrix(const int32_t* row, const int32_t* col, const float* val,
                                int64_t nnz, int n, float* D, CloudState* st, hipStream_t s) {
  if (n < 1) return hipErrorInvalidValue;
  const int64_t nn = (int64_t)n * n;
  const int64_t bi = (nn + kBlock - 1) / kBlock;
  const unsigned gi = (unsigned)(bi < 4096 ? bi : 4096);
  sparse_init_kernel<<<gi, kBlock, 0, s>>>(D, n);
  if (nnz > 0) {
    const int64_t bf = (nnz + kBlock - 1) / kBlock;
    const unsigned gf = (unsigned)(bf < 4096 ? bf : 4096);
    sparse_fill_kernel<<<gf, kBlock, 0, s>>>(row, col, val, nnz, n, D, st);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// H0 (Sec. 5.2.5): the pairs of dimension 0 are the merges of Kruskal's
// algorithm over the edges in filtration order, i.e. the edges of the minimum
// spanning forest under that total order (unique, since the order is total).
// One workgroup per cloud:
//   1. Boruvka rounds build the forest: every component takes its minimum
//      outgoing edge (key = diameter bits, then reversed edge index, so the
//      minimum key is the oldest edge), components hook along those edges,
//      pointer jumping relabels; at most log2(n) rounds;
//   2. a bitonic sort in LDS puts the forest edges in filtration order;
//   3. one lane runs union-find with the elder rule: each component is
//      represented by its oldest vertex (the largest index); a merge kills
//      the component whose representative is younger.
// The forest edges are the deaths of H0 pairs and are cleared for dim 1.
// ---------------------------------------------------------------------------

constexpr int kH0Threads = 1024;

__device__ __forceinline__ unsigned long long edge_key(uint32_t w, int a, int b) {
  const uint64_t e = a > b ? edge_index(a, b) : edge_index(b, a);
  return ((unsigned long long)w << 32) | (0xFFFFFFFFu - (uint32_t)e);
}

// Root of x under path halving. Every root is the oldest (largest) vertex of
// its component, since a merge links the younger root below the older one.
__device__ __forceinline__ int h0_find(int* parent, int x) {
  int p = parent[x];
  while (p != x) {
    const int pp = parent[p];
    parent[x] = pp;
    x = p;
    p = pp;
  }
  return x;
}

// Phases 2 and 3 of one cloud, by one workgroup of kH0Threads lanes: the
// m forest edge keys in mst (LDS, room for a power of two >= m) are sorted,
// cleared in the dimension-1 bitmap bm and paired by union-find with the
// elder rule (parent, mark: LDS scratch of n entries each); the pairs go to
// o and their number to *count.
//
// The union-find runs on one wave, 64 edges at a time. A component's root is
// its oldest vertex, so a merge of roots A and B kills min(A, B) (the
// birth of the pair) and links it below max(A, B). At the start of a block
// every lane finds the roots of its edge's two vertices (concurrent path
// halving only shortens paths: nothing is linked meanwhile). An edge whose
// two roots appear in no other edge of the block merges them as they are:
// no other merge of the block renames them or is renamed by it (the lanes
// count their roots in mark to find such edges). The other edges merge in
// edge order on their labels in registers: merge j reads lane j's two
// current labels, and every lane renames the killed root to the survivor,
// so each later merge sees the roots as of its own turn. Each edge joins
// two components (it is a forest edge), so every merge kills a root once;
// the block's links are written to parent at its end.
__device__ void h0_pair(const unsigned long long* mst, int m, int* parent, int* mark, int n,
                        uint32_t* bm, H0Pair* o, uint32_t* count);
__device__ void h0_finish(unsigned long long* mst, int m, int* parent, int* mark, int n,
                          uint32_t* bm, H0Pair* o, uint32_t* count) {
  const int tid = threadIdx.x;
  // bitonic sort of the m forest edges, ascending (padding with ~0)
  int P = 1;
  while (P < m) P <<= 1;
  for (int i = m + tid; i < P; i += kH0Threads) mst[i] = ~0ull;
  for (int v = tid; v < n; v += kH0Threads) {
    parent[v] = v;
    mark[v] = 0;
  }
  __syncthreads();
  // Stages whose partner distance j is below 64 pair elements of the same
  // 64-element chunk: a wave sorts a chunk in registers with shuffles (every
  // k <= 64 at once, then the j < 64 tail of each larger k); only the stages
  // with j >= 64 go through LDS with a workgroup barrier each.
  const int wave = tid >> 6, lane = tid & 63;
  auto chunk_stages = [&](int k_from, int k_to) {
    for (int c0 = wave * 64; c0 < P; c0 += kH0Threads) {
      const int i = c0 + lane;
      unsigned long long x = mst[i];
      for (int k = k_from; k <= k_to; k <<= 1) {
        const bool up = (i & k) == 0;
        for (int j = (k >> 1) < 32 ? (k >> 1) : 32; j > 0; j >>= 1) {
          const unsigned long long y = shfl_xor_u64(x, j);
          const bool low = (lane & j) == 0;  // the smaller index of the pair
          x = ((x > y) == (low == up)) ? y : x;
        }
      }
      mst[i] = x;
    }
  };
  if (P >= 2) chunk_stages(2, P < 64 ? P : 64);
  __syncthreads();
  for (int k = 128; k <= P; k <<= 1) {
    for (int j = k >> 1; j >= 64; j >>= 1) {
      for (int i = tid; i < P; i += kH0Threads) {
        int l = i ^ j;
        if (l > i) {
          unsigned long long a = mst[i], b = mst[l];
          bool up = (i & k) == 0;
          if ((a > b) == up) {
            mst[i] = b;
            mst[l] = a;
          }
        }
      }
      __syncthreads();
    }
    chunk_stages(k, k);
    __syncthreads();
  }

  h0_pair(mst, m, parent, mark, n, bm, o, count);
}

// Phase 3 of h0_finish on keys already sorted ascending (in LDS or in
// global memory), with parent[v] = v and mark[v] = 0 for every vertex; all
// threads of the workgroup call it.
__device__ void h0_pair(const unsigned long long* mst, int m, int* parent, int* mark, int n,
                        uint32_t* bm, H0Pair* o, uint32_t* count) {
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  // the forest edges are H0 deaths: clear them for dimension 1
  for (int i = tid; i < m; i += kH0Threads) {
    uint32_t e = 0xFFFFFFFFu - (uint32_t)mst[i];
    atomicOr(&bm[e >> 5], 1u << (e & 31));
  }
  if (tid >= 64) return;  // the rest is one wave's

  for (int base = 0; base < m; base += 64) {
    const int i = base + lane;
    const bool live = i < m;
    const unsigned long long key = live ? mst[i] : 0ull;
    const uint64_t e = 0xFFFFFFFFu - (uint32_t)key;
    int la = 0, lb = 0;
    if (live) {
      int a, b;
      edge_vertices(e, a, b);
      la = h0_find(parent, a);
      lb = h0_find(parent, b);
      __hip_atomic_fetch_add(&mark[la], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
      __hip_atomic_fetch_add(&mark[lb], 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    __builtin_amdgcn_wave_barrier();
    bool twice = false;  // a root of this edge is in another edge of the block
    if (live) twice = (mark[la] | mark[lb]) > 1;
    __builtin_amdgcn_wave_barrier();
    if (live) {
      mark[la] = 0;
      mark[lb] = 0;
    }
    int dead = la < lb ? la : lb, keep = la < lb ? lb : la;
    for (unsigned long long rest = __ballot(twice); rest; rest &= rest - 1) {
      const int j = __builtin_ctzll(rest);
      const int A = __builtin_amdgcn_readlane(la, j), B = __builtin_amdgcn_readlane(lb, j);
      const int young = A < B ? A : B, old = A < B ? B : A;
      if (lane == j) {
        dead = young;
        keep = old;
      }
      la = la == young ? old : la;
      lb = lb == young ? old : lb;
    }
    if (live) {
      o[i].death = e;
      o[i].birth = (uint32_t)dead;
      o[i].diam = (uint32_t)(key >> 32);
      parent[dead] = keep;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }
  // the roots left are the components' oldest vertices: essential classes,
  // in increasing vertex order after the m pairs
  int k = m;
  for (int v0 = 0; v0 < n; v0 += 64) {
    const int v = v0 + lane;
    const bool root = v < n && parent[v] == v;
    const unsigned long long bal = __ballot(root);
    if (root) {
      const int pos = k + __popcll(bal & ((1ull << lane) - 1ull));
      o[pos].death = ~0ull;
      o[pos].birth = (uint32_t)v;
      o[pos].diam = kInf;
    }
    k += __popcll(bal);
  }
  if (lane == 0) *count = (uint32_t)k;
}

__global__ __launch_bounds__(kH0Threads) void batch_h0_kernel(const uint32_t* __restrict__ W,
                                                              const Cloud* __restrict__ clouds,
                                                              CloudState* __restrict__ st,
                                                              H0Pair* __restrict__ out,
                                                              int64_t out_stride,
                                                              uint32_t* __restrict__ bitmaps) {
  __shared__ unsigned long long best[kBatchMaxN];  // per component root: its minimum outgoing edge
  __shared__ unsigned long long mst[kBatchMaxN];
  __shared__ int comp[kBatchMaxN];                 // component root of every vertex
  __shared__ int hookto[kBatchMaxN];               // where a root moves this round
  __shared__ int m_sh, changed;
  constexpr unsigned long long kNone = ~0ull;

  const int c = blockIdx.x;
  const Cloud cl = clouds[c];
  const int n = cl.n;
  const uint32_t* Wc = W + cl.w_off;
  const int tid = threadIdx.x;

  for (int v = tid; v < n; v += kH0Threads) comp[v] = v;
  if (tid == 0) m_sh = 0;
  __syncthreads();

  for (;;) {
    for (int v = tid; v < n; v += kH0Threads) best[v] = kNone;
    if (tid == 0) changed = 0;
    __syncthreads();
    // minimum outgoing edge of every vertex, folded into its component: a
    // wave takes a row, its lanes stride along it (coalesced, several loads
    // in flight), then a wave minimum and one LDS atomic per row
    {
      const int wave = tid >> 6, lane = tid & 63;
      for (int u = wave; u < n; u += kH0Threads / 64) {
        const int cu = comp[u];
        const uint32_t* Wu = Wc + (int64_t)u * n;
        unsigned long long mk = kNone;
        for (int v = lane; v < n; v += 64) {
          const uint32_t w = Wu[v];
          if (w != kInf && comp[v] != cu) {
            const unsigned long long k = edge_key(w, u, v);
            mk = k < mk ? k : mk;
          }
        }
        for (int o = 32; o > 0; o >>= 1) {
          const unsigned long long t = shfl_xor_u64(mk, o);
          mk = t < mk ? t : mk;
        }
        if (lane == 0 && mk != kNone) atomicMin(&best[cu], mk);
      }
    }
    __syncthreads();
    // every root decides, while best[] is read-only: its minimum edge goes to
    // the forest (a mutual minimum edge, chosen by both components, is taken
    // once, by the smaller root) and the root hooks to the other component
    // (for a mutual edge only the larger root moves, so no cycle forms)
    for (int r = tid; r < n; r += kH0Threads) {
      hookto[r] = r;
      if (comp[r] != r || best[r] == kNone) continue;
      const unsigned long long k = best[r];
      int a, b;
      edge_vertices(0xFFFFFFFFu - (uint32_t)k, a, b);
      const int other = comp[a] == r ? comp[b] : comp[a];
      const bool mutual = best[other] == k;
      if (!mutual || r < other) {
        const int slot = atomicAdd(&m_sh, 1);
        mst[slot] = k;
      }
      if (!mutual || r > other) hookto[r] = other;
      changed = 1;
    }
    __syncthreads();
    if (!changed) break;
    for (int r = tid; r < n; r += kH0Threads)
      if (comp[r] == r) comp[r] = hookto[r];
    __syncthreads();
    // relabel every vertex with its new root by pointer jumping
    for (int it = 0; it < 32; ++it) {  // depth halves every step; 2^32 > n
      int moved = 0;
      for (int v = tid; v < n; v += kH0Threads) {
        const int p = comp[v], pp = comp[p];
        if (p != pp) {
          comp[v] = pp;
          moved = 1;
        }
      }
      __syncthreads();
      if (!__syncthreads_or(moved)) break;
    }
  }
  const int m = m_sh;
  __syncthreads();
  h0_finish(mst, m, comp, hookto, n, bitmaps + cl.bm_off, out + (int64_t)c * out_stride,
            &st[c].h0_count);
}

hipError_t launch_batch_h0(const uint32_t* W, const Cloud* clouds, int count, CloudState* st,
                           H0Pair* out, int64_t out_stride, uint32_t* bitmaps, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  batch_h0_kernel<<<count, kH0Threads, 0, s>>>(W, clouds, st, out, out_stride, bitmaps);
  return hipGetLastError();
}

// The same for one large cloud, with the row scans of every Boruvka round
// spread over the chip: a wave per row (n / 16 workgroups) folds the row's
// minimum outgoing edge into its component with a 64-bit atomicMin in
// global memory; one workgroup then decides, hooks and relabels (O(n) work).
// Every round halves the components that still have an outgoing edge, so
// ceil(log2 n) + 1 rounds suffice; the host launches that many without
// waiting, and a round that changes nothing sets `done`, which turns the
// launches after it into no-ops. One workgroup finishes as above.
struct H0Wide {
  unsigned long long* best;  // per component root: its minimum outgoing edge
  int* comp;                 // component root of every vertex
  int* hookto;               // where a root moves this round
  unsigned long long* mst;   // forest edge keys
  int* m;                    // forest edges so far
  int* done;                 // set once a round changes nothing
};

__global__ __launch_bounds__(kH0Threads) void h0w_init_kernel(int n, H0Wide w) {
  for (int v = blockIdx.x * kH0Threads + threadIdx.x; v < n; v += gridDim.x * kH0Threads) {
    w.comp[v] = v;
    w.best[v] = ~0ull;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *w.m = 0;
    *w.done = 0;
  }
}

__global__ __launch_bounds__(kH0Threads) void h0w_scan_kernel(const uint32_t* __restrict__ W, int n,
                                                              H0Wide w) {
  if (*w.done) return;
  const int lane = (int)(threadIdx.x & 63);
  const int u = (int)(blockIdx.x * (kH0Threads / 64) + (threadIdx.x >> 6));
  if (u >= n) return;  // whole waves
  const int cu = w.comp[u];
  const uint32_t* Wu = W + (int64_t)u * n;
  unsigned long long mk = ~0ull;
  for (int v = lane; v < n; v += 64) {
    const uint32_t x = Wu[v];
    if (x != kInf && w.comp[v] != cu) {
      const unsigned long long k = edge_key(x, u, v);
      mk = k < mk ? k : mk;
    }
  }
  for (int o = 32; o > 0; o >>= 1) {
    const unsigned long long t = shfl_xor_u64(mk, o);
    mk = t < mk ? t : mk;
  }
  if (lane == 0 && mk != ~0ull) atomicMin(&w.best[cu], mk);
}

// The same minimum outgoing edge per component from a list of the finite
// edges (records {weight bits, 0, a << 32 | b}): each edge between two
// components offers its key to both. O(edges) a round instead of O(n^2).
__global__ __launch_bounds__(kBlock) void h0w_scan_edges_kernel(const Column* __restrict__ e,
                                                                int64_t m, H0Wide w) {
  if (*w.done) return;
  for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < m;
       k += (int64_t)gridDim.x * kBlock) {
    const Column r = e[k];
    const int a = (int)(r.cidx >> 32), b = (int)(uint32_t)r.cidx;
    const int ca = w.comp[a], cb = w.comp[b];
    if (ca != cb) {
      const unsigned long long key = edge_key(r.key_hi, a, b);
      atomicMin(&w.best[ca], key);
      atomicMin(&w.best[cb], key);
    }
  }
}

__global__ __launch_bounds__(kH0Threads) void h0w_hook_kernel(int n, H0Wide w) {
  __shared__ int changed;
  if (*w.done) return;  // the same value for the whole workgroup
  const int tid = threadIdx.x;
  if (tid == 0) changed = 0;
  __syncthreads();
  // roots decide while best[] is read-only (the rules of the one-workgroup
  // kernel: a mutual minimum edge is taken once, only its larger root moves)
  for (int r = tid; r < n; r += kH0Threads) {
    w.hookto[r] = r;
    if (w.comp[r] != r || w.best[r] == ~0ull) continue;
    const unsigned long long k = w.best[r];
    int a, b;
    edge_vertices(0xFFFFFFFFu - (uint32_t)k, a, b);
    const int other = w.comp[a] == r ? w.comp[b] : w.comp[a];
    const bool mutual = w.best[other] == k;
    if (!mutual || r < other) w.mst[atomicAdd(w.m, 1)] = k;
    if (!mutual || r > other) w.hookto[r] = other;
    changed = 1;
  }
  __syncthreads();
  if (!changed) {
    if (tid == 0) *w.done = 1;
    return;
  }
  for (int r = tid; r < n; r += kH0Threads)
    if (w.comp[r] == r) w.comp[r] = w.hookto[r];
  __syncthreads();
  for (int it = 0; it < 32; ++it) {  // pointer jumping; depth halves every step
    int moved = 0;
    for (int v = tid; v < n; v += kH0Threads) {
      const int p = w.comp[v], pp = w.comp[p];
      if (p != pp) {
        w.comp[v] = pp;
        moved = 1;
      }
    }
    __syncthreads();
    if (!__syncthreads_or(moved)) break;
  }
  for (int v = tid; v < n; v += kH0Threads) w.best[v] = ~0ull;  // for the next round
}

__global__ __launch_bounds__(kH0Threads) void h0w_finish_kernel(int n, H0Wide w,
                                                                CloudState* __restrict__ st,
                                                                H0Pair* __restrict__ out,
                                                                uint32_t* __restrict__ bm) {
  __shared__ unsigned long long mst[kH0LdsN];
  __shared__ int parent[kH0LdsN];
  __shared__ int mark[kH0LdsN];
  const int m = *w.m;  // < n <= kH0LdsN
  for (int i = threadIdx.x; i < m; i += kH0Threads) mst[i] = w.mst[i];
  __syncthreads();
  h0_finish(mst, m, parent, mark, n, bm, out, &st->h0_count);
}

// Clouds above kH0LdsN points: the forest's keys do not fit LDS next to the
// union-find's arrays, so they are sorted in global memory by the radix sort
// (as Column records: the weight bits, then the reversed edge index, which
// orders them as the 64-bit keys) and read from there by the same pairing
// as above, with parent and mark in dynamic LDS (8 bytes per vertex).
__global__ void h0w_keys_to_cols_kernel(H0Wide w, Column* __restrict__ cols,
                                        unsigned long long* __restrict__ m64) {
  const int m = *w.m;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x) {
    const unsigned long long k = w.mst[i];
    cols[i] = Column{(uint32_t)(k >> 32), 0u, (uint64_t)(uint32_t)k};
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *m64 = (unsigned long long)m;
}

__global__ void h0w_cols_to_keys_kernel(const Column* __restrict__ cols, H0Wide w) {
  const int m = *w.m;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < m; i += gridDim.x * blockDim.x)
    w.mst[i] = ((unsigned long long)cols[i].key_hi << 32) | cols[i].cidx;
}

__global__ __launch_bounds__(kH0Threads) void h0w_finish_big_kernel(int n, H0Wide w,
                                                                    CloudState* __restrict__ st,
                                                                    H0Pair* __restrict__ out,
                                                                    uint32_t* __restrict__ bm) {
  extern __shared__ int h0_lds[];  // parent[n], then mark[n]
  int* const parent = h0_lds;
  int* const mark = h0_lds + n;
  for (int v = threadIdx.x; v < n; v += kH0Threads) {
    parent[v] = v;
    mark[v] = 0;
  }
  __syncthreads();
  h0_pair(w.mst, *w.m, parent, mark, n, bm, out, &st->h0_count);
}

// scratch of launch_h0_wide: best, mst, comp, hookto, m, done; above
// kH0LdsN points also two Column arrays, a 64-bit count and the sort's work
// (the Column arrays start on a 256-byte boundary)
static size_t h0_wide_base(int n) { return ((size_t)n * 24 + 256 + 255) & ~(size_t)255; }
size_t h0_wide_scratch_bytes(int n) {
  size_t b = h0_wide_base(n);
  if (n > kH0LdsN) b += (size_t)n * 32 + 256 + ((radix_sort_work_bytes(n) + 255) & ~(size_t)255);
  return b;
}

hipError_t launch_h0_wide(const uint32_t* W, int n, CloudState* st, H0Pair* out, uint32_t* bm,
                          void* scratch, hipStream_t s, const Column* edges, int64_t m) {
  if (n < 1 || n > kMaxN) return hipErrorInvalidValue;
  char* p = static_cast<char*>(scratch);
  const size_t base = h0_wide_base(n);
  H0Wide w;
  w.best = reinterpret_cast<unsigned long long*>(p);
  w.mst = reinterpret_cast<unsigned long long*>(p + (size_t)n * 8);
  w.comp = reinterpret_cast<int*>(p + (size_t)n * 16);
  w.hookto = reinterpret_cast<int*>(p + (size_t)n * 20);
  w.m = reinterpret_cast<int*>(p + (size_t)n * 24);
  w.done = w.m + 1;
  const unsigned scan_groups = (unsigned)((n + kH0Threads / 64 - 1) / (kH0Threads / 64));
  h0w_init_kernel<<<(n + kH0Threads - 1) / kH0Threads, kH0Threads, 0, s>>>(n, w);
  int rounds = 1;
  while ((1 << (rounds - 1)) < n) ++rounds;  // ceil(log2 n) + 1
  const int64_t eg = (m + kBlock - 1) / kBlock;
  const unsigned edge_groups = (unsigned)(eg < 1 ? 1 : eg > 4096 ? 4096 : eg);
  for (int r = 0; r < rounds; ++r) {
    if (edges)
      h0w_scan_edges_kernel<<<edge_groups, kBlock, 0, s>>>(edges, m, w);
    else
      h0w_scan_kernel<<<scan_groups, kH0Threads, 0, s>>>(W, n, w);
    h0w_hook_kernel<<<1, kH0Threads, 0, s>>>(n, w);
  }
  if (n <= kH0LdsN) {
    h0w_finish_kernel<<<1, kH0Threads, 0, s>>>(n, w, st, out, bm);
    return hipGetLastError();
  }
  Column* cols = reinterpret_cast<Column*>(p + base);
  Column* tmp = cols + n;
  unsigned long long* m64 = reinterpret_cast<unsigned long long*>(tmp + n);
  void* work = p + base + (size_t)n * 32 + 256;
  const unsigned cg = (unsigned)((n + kBlock - 1) / kBlock);
  h0w_keys_to_cols_kernel<<<cg, kBlock, 0, s>>>(w, cols, m64);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  bool in_tmp = false;
  if ((e = radix_sort_columns(cols, tmp, n, 32, 0, work, s, m64, &in_tmp)) != hipSuccess) return e;
  h0w_cols_to_keys_kernel<<<cg, kBlock, 0, s>>>(in_tmp ? tmp : cols, w);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  const size_t lds = (size_t)n * 2 * sizeof(int);
  if ((e = hipFuncSetAttribute(reinterpret_cast<const void*>(&h0w_finish_big_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)) != hipSuccess)
    return e;
  h0w_finish_big_kernel<<<1, kH0Threads, lds, s>>>(n, w, st, out, bm);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Reads of one cloud's weight matrix.
// BufferRows: the whole wave works on one cloud. Raw buffer loads take the
// row offset in a scalar register and the column offset per lane (32 bits
// each), so a read is one instruction with no 64-bit address arithmetic;
// `row` must be the same for every lane of the wave. The descriptor covers
// exactly the n x n matrix (word 3 = 0x00020000, the raw 32-bit format of
// the gfx9 family).
// GlobalRows: lanes may belong to different clouds (batched edges).
// ---------------------------------------------------------------------------

struct BufferRows {
  static constexpr uint32_t kInfV = kInf;  // the weight of an edge above tau_eff
  __amdgpu_buffer_rsrc_t rs;
  int n;
  __device__ BufferRows(const uint32_t* W, int n_)
      : rs(__builtin_amdgcn_make_buffer_rsrc((void*)W, (short)0, n_ * n_ * 4, 0x00020000)),
        n(n_) {}
  // W[row][col], row uniform across the wave
  __device__ __forceinline__ uint32_t row_at(int row, int col) const {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, col * 4, row * n * 4, 0);
  }
  // W[row][col], both per lane
  __device__ __forceinline__ uint32_t lane_at(int row, int col) const {
    return __builtin_amdgcn_raw_buffer_load_b32(rs, (row * n + col) * 4, 0, 0);
  }
  // float bits of a weight
  __device__ __forceinline__ uint32_t bits(uint32_t w) const { return w; }
};

// LdsRows: the cloud's weights replaced by their dense ranks (16 bits; the
// order, which is all the filtration uses, is the same) and staged in LDS
// in rows of lds_stride(n) entries, so the reads leave the vector-memory
// address path altogether; rank_bits maps a rank back to its weight for
// the outputs.
struct LdsRows {
  static constexpr uint32_t kInfV = 0xFFFFu;
  const uint16_t* s;
  int n;
  int stride;
  const uint32_t* __restrict__ rank_bits;
  // row * stride < 2^16: a 24-bit multiply
  __device__ __forceinline__ uint32_t row_at(int row, int col) const {
    return s[__umul24(row, stride) + col];
  }
  __device__ __forceinline__ uint32_t lane_at(int row, int col) const {
    return s[__umul24(row, stride) + col];
  }
  // entries col .. col+7 of a row (col a multiple of 8) as 4 words, two
  // 16-bit ranks each, the lower column in the low half
  __device__ __forceinline__ uint4 row8(int row, int col) const {
    return *reinterpret_cast<const uint4*>(s + __umul24(row, stride) + col);
  }
  __device__ __forceinline__ uint32_t bits(uint32_t w) const { return rank_bits[w]; }
};

// Two unsigned 16-bit values packed in 32 bits: elementwise max, min and
// saturating difference.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ uint32_t max_u16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t min_u16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_min(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t addsat_u16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_add_sat(__builtin_bit_cast(u16x2, a),
                                                                    __builtin_bit_cast(u16x2, b)));
}
__device__ __forceinline__ uint32_t subsat_u16x2(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_sub_sat(__builtin_bit_cast(u16x2, a),
                                                                    __builtin_bit_cast(u16x2, b)));
}

struct GlobalRows {
  const uint32_t* __restrict__ W;
  int n;
  __device__ __forceinline__ uint32_t row_at(int row, int col) const {
    return W[(int64_t)row * n + col];
  }
  __device__ __forceinline__ uint32_t lane_at(int row, int col) const {
    return W[(int64_t)row * n + col];
  }
};

// Condition 2 of the apparent-pairs test for the cofacet t = s + {x}: the
// facets of t with a smaller index than s are t minus a vertex u > x; taking
// them in the order of increasing u, the first one whose diameter equals
// diam(s) makes s not apparent. The facets looked at (up
// to the deciding one) are counted. Usually x lies above every vertex of s
// and there is nothing to look at: the branches then skip the whole test,
// loads included, for the wave.
template <int D, class Rows>
__device__ __forceinline__ bool no_equal_facet_below(const Rows& rows, const int (&v)[D + 1], int x,
                                                     const uint32_t (&pw)[D + 1][D + 1],
                                                     uint32_t diam, uint32_t& facets) {
  if (v[D] < x) return true;  // x above every vertex of s
  uint32_t mv[D + 1];
#pragma unroll
  for (int i = 0; i <= D; ++i) mv[i] = rows.lane_at(x, v[i]);
#pragma unroll
  for (int u = 0; u <= D; ++u) {
    if (v[u] < x) continue;
    ++facets;
    uint32_t mx = 0;
#pragma unroll
    for (int i = 0; i <= D; ++i) {
      if (i == u) continue;
      mx = max(mx, mv[i]);
#pragma unroll
      for (int j = 0; j < i; ++j)
        if (j != u) mx = max(mx, pw[i][j]);
    }
    if (mx == diam) return false;
  }
  return true;
}

// ---------------------------------------------------------------------------
// The apparent-pairs test of one column (Lemma 5.3.6, Alg. 13).
//
// s has vertices v[D] > ... > v[0], pairwise weights pw and diameter diam.
// Condition 1: t is the lexicographically greatest cofacet with diam(t) =
// diam(s): scanning the added vertex x from n-1 down (cofacet indices
// decrease with x, Alg. 14), the first x with max_i W(v_i, x) <= diam.
// Condition 2: no facet of t with a smaller index than s has the same
// diameter. The facets below s are t minus a vertex u > x (Alg. 16: removing
// a higher vertex gives a smaller index). If no cofacet keeps the diameter,
// s is not apparent. Returns the added vertex x, or -1 if s is not apparent.
// ---------------------------------------------------------------------------

template <int D, class Rows>
__device__ __forceinline__ int apparent_cofacet(const Rows& rows, int n, const int (&v)[D + 1],
                                                const uint32_t (&pw)[D + 1][D + 1],
                                                uint32_t diam, uint32_t& steps,
                                                uint32_t& facets) {
  // Condition 1, kScan values of x per round trip: their loads are issued
  // together instead of one dependent load-compare-branch per x. A vertex of
  // s is never taken: its own row holds kInf on the diagonal. W is
  // symmetric, so row x (the same for every lane of the wave, as x moves in
  // lockstep) is read at the lanes' vertices; v[0] is consecutive across
  // neighbouring lanes and the loads coalesce. Rows below 0 are clamped to
  // row 0 and their result forced to kInf (or-ing the sign of x - j), which
  // keeps the loads unconditional.
  constexpr int kScan = 4;
  int found = -1;
  for (int x = n - 1; x >= 0 && found < 0; x -= kScan) {
    uint32_t mx[kScan];
#pragma unroll
    for (int j = 0; j < kScan; ++j) {
      const int xj = x - j;
      const int r = max(xj, 0);
      uint32_t m = 0;
#pragma unroll
      for (int i = 0; i <= D; ++i) m = max(m, rows.row_at(r, v[i]));
      mx[j] = m | (uint32_t)(xj >> 31);
    }
#pragma unroll
    for (int j = kScan - 1; j >= 0; --j)  // the largest x with the diameter kept
      if (mx[j] <= diam) found = x - j;
  }
  // cofacets the definition examines: every non-vertex x from n-1 down to
  // the one found (or all of them)
  int above = 0;
#pragma unroll
  for (int i = 0; i <= D; ++i) above += v[i] > found;
  steps += (uint32_t)(found >= 0 ? n - found - above : n - (D + 1));
  if (found < 0) return -1;
  // Condition 2 on t = s + {x}
  return no_equal_facet_below<D>(rows, v, found, pw, diam, facets) ? found : -1;
}

// The same test on the rank matrix in LDS. Condition 1 reads 8 values of x
// per round: the entries x-7..x of the row of each vertex of s (W is
// symmetric) come as one 128-bit read per vertex, and their maximum over
// the vertices is taken two ranks at a time. Rounds start at multiples of
// 8; columns past n-1 are padding that holds the 0xFFFF of an edge above
// the threshold, as do the diagonal entries, so neither a padding column
// nor a vertex of s is ever taken.
template <int D>
__device__ __forceinline__ int apparent_cofacet_lds(const LdsRows& rows, int n,
                                                    const int (&v)[D + 1],
                                                    const uint32_t (&pw)[D + 1][D + 1],
                                                    uint32_t diam, uint32_t& steps,
                                                    uint32_t& facets) {
  int found = -1;
  for (int g = (n - 1) & ~7; g >= 0 && found < 0; g -= 8) {
    uint4 m = rows.row8(v[0], g);
#pragma unroll
    for (int i = 1; i <= D; ++i) {
      const uint4 r = rows.row8(v[i], g);
      m.x = max_u16x2(m.x, r.x);
      m.y = max_u16x2(m.y, r.y);
      m.z = max_u16x2(m.z, r.z);
      m.w = max_u16x2(m.w, r.w);
    }
    // the largest x = g + j with the diameter kept; j is an inline
    // constant of the selects and g is added once
    const uint32_t w[4] = {m.x, m.y, m.z, m.w};
    int j_kept = -1;
#pragma unroll
    for (int j = 0; j < 8; ++j)
      if (((w[j >> 1] >> ((j & 1) * 16)) & 0xFFFFu) <= diam) j_kept = j;
    if (j_kept >= 0) found = g + j_kept;
  }
  int above = 0;
#pragma unroll
  for (int i = 0; i <= D; ++i) above += v[i] > found;
  steps += (uint32_t)(found >= 0 ? n - found - above : n - (D + 1));
  if (found < 0) return -1;
  return no_equal_facet_below<D>(rows, v, found, pw, diam, facets) ? found : -1;
}

// The same test in neighbour mode: condition 1 walks the prefix's common
// neighbours nb[0..count) from the top instead of every x from n-1 down (a
// vertex outside them keeps no diameter). The walk is in lockstep across the
// lanes, so nb[i] and its row are the same for the whole wave; the lane's own
// vertices are skipped. The cofacets counted are those of the definition, as
// in the full scan.
template <int D, class Rows>
__device__ __forceinline__ int apparent_cofacet_nb(const Rows& rows, int n, const int (&v)[D + 1],
                                                   const uint32_t (&pw)[D + 1][D + 1],
                                                   uint32_t diam, const uint16_t* nb,
                                                   uint32_t count, uint32_t& steps,
                                                   uint32_t& facets) {
  int found = -1;
  for (int i = (int)count - 1; i >= 0 && found < 0; --i) {
    const int x = nb[i];
    if (x == v[0] || x == v[1]) continue;
    uint32_t m = 0;
#pragma unroll
    for (int j = 0; j <= D; ++j) m = max(m, rows.row_at(x, v[j]));
    if (m <= diam) found = x;
  }
  int above = 0;
#pragma unroll
  for (int i = 0; i <= D; ++i) above += v[i] > found;
  steps += (uint32_t)(found >= 0 ? n - found - above : n - (D + 1));
  if (found < 0) return -1;
  return no_equal_facet_below<D>(rows, v, found, pw, diam, facets) ? found : -1;
}

// Index of the cofacet s + {x} (Eq. 5.6): vertices above x move up one position.
template <int D>
__device__ __forceinline__ uint64_t cofacet_index(const int (&v)[D + 1], int x,
                                                  const uint64_t* __restrict__ binom, int np1) {
  uint64_t c = 0;
  int p = D + 1;
  bool placed = false;
#pragma unroll
  for (int i = D; i >= 0; --i) {
    if (!placed && x > v[i]) {
      c += binom[(p + 1) * np1 + x];
      --p;
      placed = true;
    }
    c += binom[(p + 1) * np1 + v[i]];
    --p;
  }
  if (!placed) c += (uint64_t)x;  // C(x, 1)
  return c;
}

// Wave-aggregated append: every active lane with `take` gets a distinct slot
// from one atomic per wave. All lanes of the wave must call it together.
__device__ __forceinline__ uint64_t wave_append(bool take, unsigned long long* counter,
                                                bool& any) {
  const unsigned long long mask = __ballot(take);
  any = mask != 0;
  if (!any) return 0;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
  base = shfl_u64(base, leader);
  const unsigned long long below = lane ? (mask & ((~0ull) >> (64 - lane))) : 0ull;
  return base + (uint64_t)__popcll(below);
}

// Place the records of one wave-aggregated reservation into a RecordSink:
// the wave holds slots b .. b+cnt-1 of region r (b from the region counter;
// this lane's slot is b + below). Slots past the region's end go to the
// overflow region, for which one more atomic is taken only then. All lanes
// of the wave call it together; b, cnt and leader are uniform.
template <class T>
__device__ __forceinline__ void sink_place(const RecordSink<T>& k, int r, uint64_t b,
                                           uint32_t cnt, uint32_t below, int leader, bool take,
                                           const T& rec) {
  const uint64_t slot = b + below;
  T* const region = k.recs + (uint64_t)r * k.seg;
  if (b + cnt <= k.seg) {  // uniform
    if (take) region[slot] = rec;
    return;
  }
  const uint64_t first = b > k.seg ? b : k.seg;  // first slot past the region
  unsigned long long ob = 0;
  if ((int)(threadIdx.x & 63) == leader)
    ob = atomicAdd(k.ctr + (size_t)kSinkBuckets * kSinkStride, (unsigned long long)(b + cnt - first));
  ob = shfl_u64(ob, leader);
  if (take) {
    if (slot < k.seg)
      region[slot] = rec;
    else if (ob + (slot - first) < k.ovf_cap)
      k.recs[(uint64_t)kSinkBuckets * k.seg + ob + (slot - first)] = rec;
  }
}

// Wave-aggregated append into region r of a RecordSink, at once: one atomic
// per wave on the region's counter, then the writes.
template <class T>
__device__ __forceinline__ void sink_append(const RecordSink<T>& k, int r, bool take,
                                            const T& rec) {
  const unsigned long long mask = __ballot(take);
  if (!mask) return;
  const int lane = threadIdx.x & 63;
  const int leader = __ffsll((long long)mask) - 1;
  const uint32_t cnt = (uint32_t)__popcll(mask);
  unsigned long long base = 0;
  if (lane == leader) base = atomicAdd(k.ctr + (size_t)r * kSinkStride, (unsigned long long)cnt);
  base = shfl_u64(base, leader);
  const uint32_t below = (uint32_t)__popcll(lane ? (mask & ((~0ull) >> (64 - lane))) : 0ull);
  sink_place(k, r, base, cnt, below, leader, take, rec);
}

// The same in two steps, for Column records: reserve() takes the slots of
// the lanes with `take` (one atomic per wave) and keeps the records; flush()
// writes them once the atomic's result is back, the wave having done other
// work in between. All lanes of the wave call both together.
struct DeferredAppend {
  bool any = false;   // the last reserve() had a taking lane (uniform)
  bool take = false;
  int leader = 0;     // lane that holds the reserved base (uniform)
  uint32_t cnt = 0;   // taking lanes (uniform)
  uint32_t below = 0; // taking lanes below this one
  unsigned long long base = 0;
  Column rec;
  __device__ __forceinline__ void reserve(bool t, unsigned long long* counter, uint32_t key_hi,
                                          uint64_t cidx) {
    const unsigned long long mask = __ballot(t);
    any = mask != 0;
    if (!any) return;
    const int lane = threadIdx.x & 63;
    leader = __ffsll((long long)mask) - 1;
    cnt = (uint32_t)__popcll(mask);
    if (lane == leader) base = atomicAdd(counter, (unsigned long long)cnt);
    below = (uint32_t)__popcll(lane ? (mask & ((~0ull) >> (64 - lane))) : 0ull);
    take = t;
    rec.key_hi = key_hi;
    rec.cloud = 0;
    rec.cidx = cidx;
  }
  __device__ __forceinline__ void flush(const ColumnSink& k, int r) {
    if (!any) return;
    any = false;
    sink_place(k, r, shfl_u64(base, leader), cnt, below, leader, take, rec);
  }
};

// Sum per-lane counters over the workgroup and add each total to its global
// counter with one atomic (thread 0). All threads of the workgroup call it.
template <int BS, int N>
__device__ __forceinline__ void add_block_counters(unsigned long long (&v)[N],
                                                   unsigned long long* const (&dst)[N]) {
  __shared__ unsigned long long red[N][BS / 64];
  for (int o = 32; o > 0; o >>= 1)
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] += shfl_xor_u64(v[i], o);
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) red[i][threadIdx.x >> 6] = v[i];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int i = 0; i < N; ++i) {
      unsigned long long t = 0;
      for (int w = 0; w < BS / 64; ++w) t += red[i][w];
      atomicAdd(dst[i], t);
    }
}

// ---------------------------------------------------------------------------
// Dimension-d (d >= 2) enumeration + threshold + clearing + apparent test,
// one cloud. The d-simplices (v_d > ... > v_0) are split into work units:
// a unit fixes the prefix (v_d, ..., v_2) and covers a chunk of `chunk`
// consecutive suffix indices k = C(v_1, 2) + v_0 < C(v_2, 2). The simplex
// index (Eq. 5.6) is then base(prefix) + k, so consecutive lanes hold
// consecutive indices and no lane decodes an index: the suffix follows from
// one square root. Units are numbered with larger v_2 (more suffixes) first,
// so the biggest units start first. unit_cum[i] counts the units of all
// prefixes with v_2 > n-1-i (a table of n+1 entries built on the host).
// Outputs: non-apparent columns (compacted, any order; the sort that follows
// makes the order canonical), the clearing bits of the apparent cofacets for
// dimension d+1, counts, and optionally every apparent pair.
// ---------------------------------------------------------------------------

// Kernel variants (Mode bits): kModeHashed when a clearing set is hashed
// (the bitmap variant keeps the probe loops out of its hot loop),
// kModeListed when the units are listed prefixes (dimensions 2 and 3 only).
// The outputs beside the non-apparent columns: kModeTop when there is no
// clearing set for the next dimension and no pair output (the top
// dimension), kModePairs when every apparent pair is written (the clearing
// set out is then looked at at run time); neither: a clearing set out and
// no pair output. Code a launch cannot reach holds registers all the same
// (the hot loop spills scalars into vector lanes), so each case is a
// variant of its own. kModeFilter (with kModeTop, LDS kernel): the first
// stage of the paper's unfused order, which writes every column that
// survives the threshold and clearing and tests none (see
// apparent_sorted_lds_kernel).
constexpr int kModeHashed = 1, kModeListed = 2, kModeTop = 4, kModePairs = 8, kModeFilter = 16;

template <int D, int BS, int UL, int Mode, class Rows>
__device__ __forceinline__ void enum_units(
    const Rows& rows, int n, const uint64_t* __restrict__ binom, int chunk,
    const uint64_t* __restrict__ unit_cum, uint64_t units, const PrefixList& pl,
    const ClearSet& clear_in, const ClearSet& clear_out, const ColumnSink& sink,
    const PairSink& aps, Scalars* __restrict__ sc) {
  constexpr uint32_t kInfW = Rows::kInfV;
  constexpr bool kHashed = (Mode & kModeHashed) != 0;
  constexpr bool kListed = (Mode & kModeListed) != 0;
  constexpr bool kTop = (Mode & kModeTop) != 0;
  constexpr bool kPairs = (Mode & kModePairs) != 0;
  constexpr bool kFilter = (Mode & kModeFilter) != 0;
  static_assert(!kListed || D == 2 || D == 3, "listed prefixes are pairs or single vertices");
  static_assert(!kFilter || kTop, "the filter stage writes columns only");
  static_assert(!(kTop && kPairs), "the pair output needs the cofacet indices");
  const int np1 = n + 1;
  auto C = [&](int v, int k) -> uint64_t { return binom[(int64_t)k * np1 + v]; };
  unsigned long long n_cols = 0, n_app = 0, n_steps = 0, n_facets = 0, n_cand = 0;
  DeferredAppend pend;
  // the cofacet index of an apparent pair: for the clearing set out (the
  // launch takes the variant without kModeTop or kModePairs only with one)
  // or for the pair output
  const bool need_t =
      kPairs ? (clear_out.bits || (kHashed && clear_out.keys) || aps.recs) : !kTop;
  const int bucket = (int)((blockIdx.x * (BS / 64) +
                            (unsigned)__builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6))) %
                           kSinkBuckets);
  unsigned long long* const bucket_ctr = sink.ctr + (size_t)bucket * kSinkStride;

  // units are strided over groups of UL lanes (a dispatch holds < 2^32
  // work-items). UL = 64: a wave takes a unit on its own, so the unit's
  // prefix is decoded once and its last round of 64 candidates is the only
  // partial one. UL = BS: the waves of a workgroup share a unit, and with it
  // the rows of W it reads from the caches.
  // The group number is read from the first lane so that the compiler
  // knows it, and everything derived from it (the unit's decode), to be
  // uniform across the wave: scalar registers and scalar loads.
  static_assert(UL % 64 == 0 && BS % UL == 0, "unit groups are whole waves of a workgroup");
  const int lane = (int)(threadIdx.x % UL);
  const int group_in_block = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / UL));
  const uint64_t group0 = (uint64_t)blockIdx.x * (BS / UL) + (uint64_t)group_in_block;
  const uint64_t ngroups = (uint64_t)gridDim.x * (BS / UL);
  for (uint64_t u = group0; u < units; u += ngroups) {
  // ---- the unit: prefix (v_d..v_2) and its suffix range (uniform) ----
  int v[D + 1];
  uint64_t k_begin = 0, k_end = 0;
  bool listed = false;
  if constexpr (kListed) {
    {  // listed prefixes: the p with cum[p] <= u < cum[p+1]
      listed = true;
      uint32_t lo = 0, hi = pl.count - 1;
      while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (pl.cum[mid] <= u)
          lo = mid;
        else
          hi = mid - 1;
      }
      const uint32_t pv = pl.v[lo];
      if constexpr (D == 3) v[3] = (int)(pv >> 16);
      v[2] = (int)(pv & 0xFFFFu);
      const uint64_t suffixes = (uint64_t)v[2] * (uint64_t)(v[2] - 1) / 2;
      k_begin = (u - pl.cum[lo]) * (uint64_t)chunk;
      k_end = min(k_begin + (uint64_t)chunk, suffixes);
    }
  }
  if (!listed) {
  int lo = 0, hi = n - 2;  // largest i with unit_cum[i] <= u; v_2 = n-1-i
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (unit_cum[mid] <= u)
      lo = mid;
    else
      hi = mid - 1;
  }
  const int t = n - 1 - lo;
  const uint64_t suffixes = (uint64_t)t * (uint64_t)(t - 1) / 2;
  const uint64_t chunks = (suffixes + chunk - 1) / chunk;
  const uint64_t q = u - unit_cum[lo];
  uint64_t upper = q / chunks;  // rank of (v_d..v_3) among (d-2)-subsets of (t, n)
  k_begin = (q % chunks) * (uint64_t)chunk;
  k_end = min(k_begin + (uint64_t)chunk, suffixes);
  v[2] = t;
    int top = n - 1 - (t + 1);  // decode in the shifted range [0, n-1-t)
#pragma unroll
    for (int i = D - 2; i >= 1; --i) {  // position i of the upper part -> v[i+2]
      int a = i - 1, h = top;
      while (a < h) {
        int mid = (a + h + 1) >> 1;
        if (C(mid, i) <= upper)
          a = mid;
        else
          h = mid - 1;
      }
      v[i + 2] = a + t + 1;
      upper -= C(a, i);
      top = a - 1;
    }
  }  // dense unit table
  uint64_t base = 0;
#pragma unroll
  for (int i = 2; i <= D; ++i) base += C(v[i], i + 1);
  uint32_t pmax = 0;  // largest weight among the prefix vertices
#pragma unroll
  for (int i = 3; i <= D; ++i)
#pragma unroll
    for (int j = 2; j < i; ++j) pmax = max(pmax, rows.row_at(v[i], v[j]));
  // a prefix with an edge above the threshold spans no simplex of the
  // complex: the whole unit is skipped (uniform across the wave); this
  // is what keeps a threshold far below the enclosing radius cheap
  if (pmax == kInfW) continue;
  uint32_t u_steps = 0, u_facets = 0;

  // Neighbour mode (listed prefixes of dimension 2 or 3 in the
  // global-memory kernel, Sec. 5.3.12-5.3.13): the suffixes (v1 > v0) of a
  // prefix (v3, v2), or (v2), that can span a simplex are the pairs of
  // common neighbours of the prefix vertices below v2. The workgroup lists
  // the common neighbours in LDS in increasing order, and suffix k below is
  // then the k-th pair (i > j) of those below v2 instead of the k-th pair of
  // all vertices below v2.
  constexpr bool kNeighbours = kListed && !__is_same(Rows, LdsRows);
  // The list holds every common neighbour (below and above v2), so that the
  // cofacet scan can walk it too: a vertex outside it is not a neighbour of
  // some vertex of s, so no cofacet with it keeps the diameter.
  const uint16_t* nb = nullptr;
  uint32_t nb_all = 0;  // common neighbours; the first nb_below are below v2
  if constexpr (kNeighbours) {
    if (listed) {
      extern __shared__ uint16_t cn[];  // n entries: the launch sizes it
      __shared__ uint32_t wcount[BS / 64];
      const int wave = (int)(threadIdx.x >> 6), l64 = (int)(threadIdx.x & 63);
      uint32_t cnt = 0;
      for (int x0 = 0; x0 < n; x0 += BS) {
        const int x = x0 + (int)threadIdx.x;
        bool in = x < n && rows.row_at(v[2], x) != kInfW;  // the diagonal is kInf
        if constexpr (D == 3) in = in && rows.row_at(v[3], x) != kInfW;
        const unsigned long long m = __ballot(in);
        if (l64 == 0) wcount[wave] = (uint32_t)__popcll(m);
        __syncthreads();
        uint32_t off = cnt, all = 0;
        for (int w = 0; w < BS / 64; ++w) {
          if (w < wave) off += wcount[w];
          all += wcount[w];
        }
        if (in) cn[off + (uint32_t)__popcll(l64 ? (m & ((~0ull) >> (64 - l64))) : 0ull)] = (uint16_t)x;
        cnt += all;
        __syncthreads();
      }
      // the list is increasing: its entries below v2 come first
      uint32_t lo = 0, hi = cnt;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (cn[mid] < v[2])
          lo = mid + 1;
        else
          hi = mid;
      }
      nb = cn;
      nb_all = cnt;
      k_begin = 0;
      k_end = (uint64_t)lo * (lo - 1) / 2;  // pairs of the neighbours below v2
      if (threadIdx.x == 0) n_cand += k_end;
    }
  }

  // the clearing words of a lane's next candidate are read one round ahead,
  // so their latency overlaps the current candidate's work (dense suffixes
  // only: in neighbour mode consecutive k are not consecutive indices)
  uint32_t cw_next = 0;
  const uint32_t* __restrict__ clear_bits = kNeighbours ? nullptr : clear_in.bits;
  if (clear_bits && k_begin + lane < k_end) cw_next = clear_bits[(base + k_begin + lane) >> 5];
  for (uint64_t kb = k_begin; kb < k_end; kb += UL) {
    const uint64_t k = kb + lane;
    const uint32_t cw = cw_next;
    if (clear_bits && k + UL < k_end) cw_next = clear_bits[(base + k + UL) >> 5];
    bool is_col = false, is_app = false;
    uint32_t pw[D + 1][D + 1];
    uint32_t diam = kInfW;
    uint64_t c = 0, tcidx = 0;
    int vv[D + 1];
#pragma unroll
    for (int i = 2; i <= D; ++i) vv[i] = v[i];
    if (k < k_end) {
      // suffix: largest v1 with C(v1, 2) <= k, i.e. floor((1 + sqrt(8k+1))/2),
      // then v0. k < C(n, 2) < 2^27 (n <= 16384), so 8k + 1 < 2^30 is exact
      // in 32 bits and within a relative 2^-24 as a float; the hardware
      // square root adds at most 1 ulp (2^-8 below 2^15). The estimate is
      // then within 1e-2 of the exact quotient and its floor is off by at
      // most one either way: one exact integer step corrects it.
      const uint32_t k32 = (uint32_t)k;
      int v1 = (int)((1.0f + __builtin_amdgcn_sqrtf((float)(8u * k32 + 1u))) * 0.5f);
      uint32_t t1 = __umul24(v1, v1 - 1) >> 1;  // C(v1, 2); v1 <= n <= 2^14: < 2^28
      if (t1 > k32) {
        --v1;
        t1 -= v1;
      } else if (t1 + v1 <= k32) {
        t1 += v1;
        ++v1;
      }
      vv[1] = v1;
      vv[0] = (int)(k32 - t1);
      c = base + k;
      if constexpr (kNeighbours) {
        if (nb) {  // the k-th pair of common neighbours
          vv[1] = nb[v1];
          vv[0] = nb[k32 - t1];
          c = base + (uint64_t)vv[1] * (uint64_t)(vv[1] - 1) / 2 + (uint64_t)vv[0];
        }
      }
      diam = pmax;
      // rows of the prefix vertices are uniform; (v1, v0) is per lane
      pw[1][0] = rows.lane_at(vv[1], vv[0]);
      diam = max(diam, pw[1][0]);
#pragma unroll
      for (int i = 2; i <= D; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          pw[i][j] = rows.row_at(vv[i], vv[j]);
          diam = max(diam, pw[i][j]);
        }
#pragma unroll
      for (int i = 3; i <= D; ++i)
#pragma unroll
        for (int j = 2; j < i; ++j) pw[i][j] = rows.row_at(vv[i], vv[j]);
      // a hashed set (or a bitmap in neighbour mode) is probed only for
      // simplices of the complex
      bool cleared;
      if constexpr (kHashed || kNeighbours)
        cleared = clear_bits ? ((cw >> (c & 31)) & 1u)
                             : (diam != kInfW && clear_contains(clear_in, c));
      else
        cleared = (cw >> (c & 31)) & 1u;
      is_col = diam != kInfW && !cleared;
      if (is_col && kFilter) ++n_cols;
      if (is_col && !kFilter) {
        ++n_cols;
        int x;
        if constexpr (__is_same(Rows, LdsRows))
          x = apparent_cofacet_lds<D>(rows, n, vv, pw, diam, u_steps, u_facets);
        else if (nb)
          x = apparent_cofacet_nb<D>(rows, n, vv, pw, diam, nb, nb_all, u_steps, u_facets);
        else
          x = apparent_cofacet<D>(rows, n, vv, pw, diam, u_steps, u_facets);
        if (x >= 0) {
          is_app = true;
          ++n_app;
          // the cofacet's index is needed only to clear it in the next
          // dimension or to report the pair
          if (need_t) {
            tcidx = cofacet_index<D>(vv, x, binom, np1);
            if constexpr (kHashed)
              clear_insert(clear_out, tcidx);
            else if (clear_out.bits)
              atomicOr(&clear_out.bits[tcidx >> 5], 1u << (tcidx & 31));
          }
        }
      }
    }
    // non-apparent columns: the slots are reserved now and the records
    // written one round later, once the reserving atomic has returned
    pend.flush(sink, bucket);
    const bool nonapp = is_col && !is_app;
    uint32_t key_hi = 0;
    if (nonapp) key_hi = ~rows.bits(diam);
    pend.reserve(nonapp, bucket_ctr, key_hi, c);
    bool any;
    if constexpr (kPairs) {
      if (aps.recs) {
        ApparentPair p;
        p.s = c;
        p.t = tcidx;
        p.diam = is_app ? rows.bits(diam) : 0u;
        p.cloud = 0;
        sink_append(aps, bucket, is_app, p);
      }
    }
  }
  // a unit's counts fit 32 bits: at most chunk / BS candidates per lane,
  // fewer than n cofacets and D + 1 facets each
  n_steps += u_steps;
  n_facets += u_facets;
  if constexpr (kNeighbours)
    if (nb) __syncthreads();  // the next unit rewrites the neighbour list
  }  // units
  pend.flush(sink, bucket);
  // workgroup totals, one atomic each
  unsigned long long tot[5] = {n_cols, n_app, n_steps, n_facets, n_cand};
  unsigned long long* const dst[5] = {&sc->columns, &sc->apparent, &sc->scan_steps,
                                      &sc->facet_steps, &sc->candidates};
  add_block_counters<BS, 5>(tot, dst);
}

// 8 waves per SIMD (64 vector, 96 scalar registers) for D <= 3
template <int D, int Mode>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(D <= 3 ? 8 : 4)))
void enum_apparent_kernel(
    const uint32_t* __restrict__ W, int n, const uint64_t* __restrict__ binom, int chunk,
    const uint64_t* __restrict__ unit_cum, uint64_t units, PrefixList pl, ClearSet clear_in,
    ClearSet clear_out, ColumnSink sink, PairSink aps, Scalars* __restrict__ sc) {
  const BufferRows rows(W, n);
  enum_units<D, kBlock, kBlock, Mode>(rows, n, binom, chunk, unit_cum, units, pl, clear_in, clear_out,
                                sink, aps, sc);
}

// The same with the rank matrix (n <= kLdsMaxN, 16-bit ranks, n rows of
// lds_stride(n) entries) staged in LDS once per workgroup: 2 workgroups of
// kLdsBlock lanes fill a compute unit's 160 KB. Two of them are resident
// only at 8 waves per SIMD, which caps a wave at 64 vector and 96 scalar
// registers; the compiler is held to that for D <= 3 (above, the registers
// a wave needs leave room for one workgroup per compute unit).
template <int D, int Mode>
__global__ __launch_bounds__(kLdsBlock) __attribute__((amdgpu_waves_per_eu(D <= 3 ? 8 : 4)))
void enum_apparent_lds_kernel(
    const uint16_t* __restrict__ Wr, const uint32_t* __restrict__ rank_bits, int n,
    const uint64_t* __restrict__ binom, int chunk, const uint64_t* __restrict__ unit_cum,
    uint64_t units, PrefixList pl, ClearSet clear_in, ClearSet clear_out, ColumnSink sink,
    PairSink aps, Scalars* __restrict__ sc) {
  __shared__ uint4 sw[kLdsMaxN * kLdsMaxN / 8];
  const int stride = lds_stride(n);
  const int words = n * stride / 8;  // 16-byte words; stride is a multiple of 8
  const uint4* __restrict__ src = reinterpret_cast<const uint4*>(Wr);
  for (int i = threadIdx.x; i < words; i += kLdsBlock) sw[i] = src[i];
  __syncthreads();
  const LdsRows rows{reinterpret_cast<const uint16_t*>(sw), n, stride, rank_bits};
  enum_units<D, kLdsBlock, 64, Mode>(rows, n, binom, chunk, unit_cum, units, pl, clear_in, clear_out,
                               sink, aps, sc);
}

// The output bits of a launch (see kModeTop): dimensions 2 and 3 have a
// variant per case, the others one that decides at run time.
template <int D, int Base, class Launch>
static hipError_t with_outputs(const ClearSet& clear_out, const PairSink& aps, Launch&& go) {
  if constexpr (D == 2 || D == 3) {
    if (!aps.recs) {
      if (clear_out.bits || clear_out.keys) return go(std::integral_constant<int, Base>{});
      return go(std::integral_constant<int, Base | kModeTop>{});
    }
  }
  return go(std::integral_constant<int, Base | kModePairs>{});
}

// The paper's unfused order, kept to measure what the fusion saves (the
// kernels above test each column right after its diameter): Alg. 17 writes
// every column that survives the threshold and clearing (the enumeration
// kernel in mode kModeFilter), Alg. 18 sorts them into coboundary order (the
// radix sort), and this kernel then runs the apparent-pairs test (Lemma
// 5.3.6, Alg. 13) over the sorted columns: each lane decodes its column's
// index into vertices (Eq. 5.6, the largest v with C(v, k) <= the rest, by
// binary search), takes the diameter from the rank matrix in LDS and tests
// the column as the fused kernel does. Non-apparent columns go to the sink,
// apparent cofacets set the next dimension's clearing bits (a bitmap or
// none). The sorted columns are min(*count, cap) (count on the device).
template <int D>
__global__ __launch_bounds__(kLdsBlock) __attribute__((amdgpu_waves_per_eu(8)))
void apparent_sorted_lds_kernel(const uint16_t* __restrict__ Wr,
                                const uint32_t* __restrict__ rank_bits, int n,
                                const uint64_t* __restrict__ binom, const Column* __restrict__ cols,
                                const unsigned long long* __restrict__ count, uint64_t cap,
                                ClearSet clear_out, ColumnSink sink, Scalars* __restrict__ sc) {
  __shared__ uint4 sw[kLdsMaxN * kLdsMaxN / 8];
  const int stride = lds_stride(n);
  const int words = n * stride / 8;
  const uint4* __restrict__ src = reinterpret_cast<const uint4*>(Wr);
  for (int i = threadIdx.x; i < words; i += kLdsBlock) sw[i] = src[i];
  __syncthreads();
  const LdsRows rows{reinterpret_cast<const uint16_t*>(sw), n, stride, rank_bits};
  const int np1 = n + 1;
  const uint64_t total = min((uint64_t)*count, cap);
  const int lane = (int)(threadIdx.x & 63);
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int bucket = (int)((blockIdx.x * (kLdsBlock / 64) + (unsigned)wave) % kSinkBuckets);
  unsigned long long n_app = 0, n_steps = 0, n_facets = 0;
  const uint64_t step = (uint64_t)gridDim.x * kLdsBlock;
  for (uint64_t b0 = (uint64_t)blockIdx.x * kLdsBlock + (uint64_t)wave * 64; b0 < total; b0 += step) {
    const uint64_t i = b0 + (uint64_t)lane;
    bool nonapp = false;
    Column rec{0u, 0u, 0ull};
    if (i < total) {
      const uint64_t c = cols[i].cidx;
      int v[D + 1];
      uint64_t rest = c;
      int top = n - 1;
#pragma unroll
      for (int k = D + 1; k >= 1; --k) {
        int lo = k - 1, hi = top;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (binom[(int64_t)k * np1 + mid] <= rest)
            lo = mid;
          else
            hi = mid - 1;
        }
        v[k - 1] = lo;
        rest -= binom[(int64_t)k * np1 + lo];
        top = lo - 1;
      }
      uint32_t pw[D + 1][D + 1];
      uint32_t diam = 0;
#pragma unroll
      for (int a = 1; a <= D; ++a)
#pragma unroll
        for (int b = 0; b < a; ++b) {
          pw[a][b] = rows.lane_at(v[a], v[b]);
          diam = max(diam, pw[a][b]);
        }
      uint32_t steps = 0, facets = 0;
      const int x = apparent_cofacet_lds<D>(rows, n, v, pw, diam, steps, facets);
      n_steps += steps;
      n_facets += facets;
      if (x >= 0) {
        ++n_app;
        if (clear_out.bits) {
          const uint64_t t = cofacet_index<D>(v, x, binom, np1);
          atomicOr(&clear_out.bits[t >> 5], 1u << (t & 31));
        }
      } else {
        nonapp = true;
        rec.key_hi = ~rows.bits(diam);
        rec.cidx = c;
      }
    }
    sink_append(sink, bucket, nonapp, rec);
  }
  unsigned long long tot[3] = {n_app, n_steps, n_facets};
  unsigned long long* const dst[3] = {&sc->apparent, &sc->scan_steps, &sc->facet_steps};
  add_block_counters<kLdsBlock, 3>(tot, dst);
}

template <int D>
static hipError_t launch_enum_D(const uint32_t* W, int n, const uint64_t* binom, int chunk,
                                const uint64_t* unit_cum, uint64_t units, PrefixList pl,
                                unsigned grid, ClearSet clear_in, ClearSet clear_out,
                                ColumnSink sink, PairSink aps, Scalars* sc, hipStream_t s) {
  auto go = [&](auto mode) {
    constexpr int kMode = decltype(mode)::value;
    // listed units build a common-neighbour list of up to n entries in LDS
    const size_t lds = (kMode & kModeListed) ? (((size_t)n * 2 + 15) & ~(size_t)15) : 0;
    enum_apparent_kernel<D, kMode><<<grid, kBlock, lds, s>>>(
        W, n, binom, chunk, unit_cum, units, pl, clear_in, clear_out, sink, aps, sc);
    return hipGetLastError();
  };
  const bool hashed = clear_in.keys || clear_out.keys;
  if constexpr (D == 2 || D == 3) {
    if (pl.v)
      return hashed ? with_outputs<D, kModeListed | kModeHashed>(clear_out, aps, go)
                    : with_outputs<D, kModeListed>(clear_out, aps, go);
  } else {
    if (pl.v) return hipErrorInvalidValue;  // prefixes are listed for d = 2, 3 only
  }
  return hashed ? with_outputs<D, kModeHashed>(clear_out, aps, go)
                : with_outputs<D, 0>(clear_out, aps, go);
}

template <int D>
static hipError_t launch_enum_lds_D(const uint16_t* Wr, const uint32_t* rank_bits, int n,
                                    const uint64_t* binom, int chunk, const uint64_t* unit_cum,
                                    uint64_t units, PrefixList pl, unsigned grid,
                                    ClearSet clear_in, ClearSet clear_out, ColumnSink sink,
                                    PairSink aps, Scalars* sc, hipStream_t s) {
  if (pl.v) return hipErrorInvalidValue;  // the LDS kernel takes dense unit tables only
  auto go = [&](auto mode) {
    enum_apparent_lds_kernel<D, decltype(mode)::value><<<grid, kLdsBlock, 0, s>>>(
        Wr, rank_bits, n, binom, chunk, unit_cum, units, pl, clear_in, clear_out, sink, aps, sc);
    return hipGetLastError();
  };
  if (clear_in.keys || clear_out.keys) return with_outputs<D, kModeHashed>(clear_out, aps, go);
  return with_outputs<D, 0>(clear_out, aps, go);
}

hipError_t launch_enum_apparent_lds(int d, const uint16_t* Wr, const uint32_t* rank_bits, int n,
                                    const uint64_t* binom, int chunk, const uint64_t* unit_cum,
                                    uint64_t units, PrefixList pl, unsigned max_groups,
                                    ClearSet clear_in, ClearSet clear_out, ColumnSink sink,
                                    PairSink aps, Scalars* sc, hipStream_t s) {
  if (units == 0) return hipSuccess;
  if (n < 1 || n > kLdsMaxN || chunk < 64 || chunk % 64 || max_groups == 0)
    return hipErrorInvalidValue;
  const uint64_t need = (units + kLdsBlock / 64 - 1) / (kLdsBlock / 64);  // a unit per wave
  uint64_t g = need < (uint64_t)max_groups ? need : (uint64_t)max_groups;
  if (g > (uint64_t)kMaxGroups) g = kMaxGroups;
  const unsigned grid = (unsigned)g;
  switch (d) {
    case 2: return launch_enum_lds_D<2>(Wr, rank_bits, n, binom, chunk, unit_cum, units, pl, grid, clear_in, clear_out, sink, aps, sc, s);
    case 3: return launch_enum_lds_D<3>(Wr, rank_bits, n, binom, chunk, unit_cum, units, pl, grid, clear_in, clear_out, sink, aps, sc, s);
    case 4: return launch_enum_lds_D<4>(Wr, rank_bits, n, binom, chunk, unit_cum, units, pl, grid, clear_in, clear_out, sink, aps, sc, s);
    case 5: return launch_enum_lds_D<5>(Wr, rank_bits, n, binom, chunk, unit_cum, units, pl, grid, clear_in, clear_out, sink, aps, sc, s);
    case 6: return launch_enum_lds_D<6>(Wr, rank_bits, n, binom, chunk, unit_cum, units, pl, grid, clear_in, clear_out, sink, aps, sc, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_enum_filter_lds(int d, const uint16_t* Wr, const uint32_t* rank_bits, int n,
                                  const uint64_t* binom, int chunk, const uint64_t* unit_cum,
                                  uint64_t units, unsigned max_groups, ClearSet clear_in,
                                  ColumnSink sink, Scalars* sc, hipStream_t s) {
  if (units == 0) return hipSuccess;
  if (n < 1 || n > kLdsMaxN || chunk < 64 || chunk % 64 || max_groups == 0 || clear_in.keys)
    return hipErrorInvalidValue;
  const uint64_t need = (units + kLdsBlock / 64 - 1) / (kLdsBlock / 64);
  uint64_t g = need < (uint64_t)max_groups ? need : (uint64_t)max_groups;
  if (g > (uint64_t)kMaxGroups) g = kMaxGroups;
  const PrefixList pl{nullptr, nullptr, 0};
  const ClearSet none{nullptr, nullptr, 0, nullptr};
  const PairSink aps{nullptr, nullptr, 0, 0};
  constexpr int kMode = kModeFilter | kModeTop;
  if (d == 2)
    enum_apparent_lds_kernel<2, kMode><<<(unsigned)g, kLdsBlock, 0, s>>>(
        Wr, rank_bits, n, binom, chunk, unit_cum, units, pl, clear_in, none, sink, aps, sc);
  else if (d == 3)
    enum_apparent_lds_kernel<3, kMode><<<(unsigned)g, kLdsBlock, 0, s>>>(
        Wr, rank_bits, n, binom, chunk, unit_cum, units, pl, clear_in, none, sink, aps, sc);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_apparent_sorted_lds(int d, const uint16_t* Wr, const uint32_t* rank_bits, int n,
                                      const uint64_t* binom, const Column* cols,
                                      const unsigned long long* count, uint64_t cap,
                                      unsigned grid, ClearSet clear_out, ColumnSink sink,
                                      Scalars* sc, hipStream_t s) {
  if (n < 1 || n > kLdsMaxN || grid == 0 || clear_out.keys) return hipErrorInvalidValue;
  if (d == 2)
    apparent_sorted_lds_kernel<2><<<grid, kLdsBlock, 0, s>>>(Wr, rank_bits, n, binom, cols, count,
                                                             cap, clear_out, sink, sc);
  else if (d == 3)
    apparent_sorted_lds_kernel<3><<<grid, kLdsBlock, 0, s>>>(Wr, rank_bits, n, binom, cols, count,
                                                             cap, clear_out, sink, sc);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_enum_apparent(int d, const uint32_t* W, int n, const uint64_t* binom, int chunk,
                                const uint64_t* unit_cum, uint64_t units, PrefixList pl,
                                unsigned max_groups, ClearSet clear_in, ClearSet clear_out,
                                ColumnSink sink, PairSink aps, Scalars* sc, hipStream_t s) {
  if (units == 0) return hipSuccess;
  if (chunk < 64 || chunk % 64 || max_groups == 0) return hipErrorInvalidValue;
  // at most kMaxGroups workgroups: the dispatch counts work-items in 32 bits;
  // a grid of a few workgroups per compute unit that loops over the units
  // keeps the per-workgroup costs (dispatch, the counter atomics at its end)
  // off the critical path
  uint64_t g = units < (uint64_t)max_groups ? units : (uint64_t)max_groups;  // a unit per group
  if (g > (uint64_t)kMaxGroups) g = kMaxGroups;
  const unsigned grid = (unsigned)g;
  switch (d) {
    case 2: return launch_enum_D<2>(W, n, binom, chunk, unit_cum, units, pl, grid, clear_in, clear_out, sink, aps, sc, s);
    case 3: return launch_enum_D<3>(W, n, binom, chunk, unit_cum, units, pl, grid, clear_in, clear_out, sink, aps, sc, s);
    case 4: return launch_enum_D<4>(W, n, binom, chunk, unit_cum, units, pl, grid, clear_in, clear_out, sink, aps, sc, s);
    case 5: return launch_enum_D<5>(W, n, binom, chunk, unit_cum, units, pl, grid, clear_in, clear_out, sink, aps, sc, s);
    case 6: return launch_enum_D<6>(W, n, binom, chunk, unit_cum, units, pl, grid, clear_in, clear_out, sink, aps, sc, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Packing of a RecordSink: workgroup r < kSinkBuckets copies region r, the
// last one the overflow region; each adds up the kept counts of the regions
// before its own for its offset.
// ---------------------------------------------------------------------------

constexpr int kGatherThreads = 256;

template <class T>
__global__ __launch_bounds__(kGatherThreads) void gather_kernel(
    RecordSink<T> k, T* __restrict__ out, uint64_t out_cap, unsigned long long* __restrict__ total) {
  __shared__ unsigned long long part[kGatherThreads / 64];
  const int r = blockIdx.x;
  unsigned long long off = 0;
  for (int q = threadIdx.x; q < r; q += kGatherThreads) {
    const unsigned long long c = k.ctr[(size_t)q * kSinkStride];
    off += c < k.seg ? c : k.seg;
  }
  for (int o = 32; o > 0; o >>= 1) off += shfl_xor_u64(off, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = off;
  __syncthreads();
  off = 0;
  for (int w = 0; w < kGatherThreads / 64; ++w) off += part[w];
  const unsigned long long have = k.ctr[(size_t)r * kSinkStride];
  const uint64_t lim = r < kSinkBuckets ? k.seg : k.ovf_cap;
  const uint64_t count = have < lim ? have : lim;
  const T* __restrict__ src = k.recs + (uint64_t)r * k.seg;
  for (uint64_t i = threadIdx.x; i < count && off + i < out_cap; i += kGatherThreads)
    out[off + i] = src[i];
  if (r == kSinkBuckets && threadIdx.x == 0) *total = off + have;
}

hipError_t launch_gather_columns(ColumnSink sink, Column* out, uint64_t out_cap,
                                 unsigned long long* total, hipStream_t s) {
  gather_kernel<Column><<<kSinkBuckets + 1, kGatherThreads, 0, s>>>(sink, out, out_cap, total);
  return hipGetLastError();
}

hipError_t launch_gather_pairs(PairSink sink, ApparentPair* out, uint64_t out_cap,
                               unsigned long long* total, hipStream_t s) {
  gather_kernel<ApparentPair><<<kSinkBuckets + 1, kGatherThreads, 0, s>>>(sink, out, out_cap,
                                                                          total);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dimension-1 columns of a batch of clouds: thread <-> edge of some cloud.
// The edge index of a cloud is C(a,2)+b; the edge is a column iff its weight
// is finite (<= tau_eff) and it is not a forest edge (cleared by H0).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void batch_edges_kernel(
    const uint32_t* __restrict__ W, const Cloud* __restrict__ clouds, int count,
    int64_t total_edges, const uint32_t* __restrict__ bitmaps, Column* __restrict__ cols,
    uint64_t cols_cap, ApparentPair* __restrict__ ap, uint64_t ap_cap, ClearSet clear_out,
    const uint64_t* __restrict__ binom_g, int np1, unsigned long long* __restrict__ counters) {
  unsigned long long n_cols = 0, n_app = 0, n_steps = 0, n_facets = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < total_edges; base += stride) {
    const int64_t e = base + threadIdx.x;
    bool is_col = false, is_app = false;
    uint32_t diam = kInf;
    uint64_t le = 0, t = 0;
    int cidx_cloud = 0;
    if (e < total_edges) {
      const int c = find_cloud(clouds, count, e, &Cloud::e_off);
      const Cloud cl = clouds[c];
      cidx_cloud = c;
      le = (uint64_t)(e - cl.e_off);
      int a, b;
      edge_vertices(le, a, b);
      const uint32_t* Wc = W + cl.w_off;
      diam = Wc[(int64_t)a * cl.n + b];
      const bool cleared = (bitmaps[cl.bm_off + (le >> 5)] >> (le & 31)) & 1u;
      is_col = diam != kInf && !cleared;
      if (is_col) {
        ++n_cols;
        int v[2] = {b, a};
        uint32_t pw[2][2];
        pw[1][0] = diam;
        uint32_t st = 0, fa = 0;
        const int x = apparent_cofacet<1>(GlobalRows{Wc, cl.n}, cl.n, v, pw, diam, st, fa);
        n_steps += st;
        n_facets += fa;
        if (x >= 0) {
          is_app = true;
          ++n_app;
          // triangle index of {x, a, b} (Eq. 5.6)
          int hi = max(x, a), lo = min(x, b), mid = x + a + b - hi - lo;
          t = (uint64_t)hi * (hi - 1) * (hi - 2) / 6 + (uint64_t)mid * (mid - 1) / 2 + (uint64_t)lo;
          clear_insert(clear_out, t);
        }
      }
    }
    bool any;
    const uint64_t slot = wave_append(is_col && !is_app, &counters[2], any);
    if (is_col && !is_app && slot < cols_cap) {
      Column r;
      r.key_hi = ~diam;
      r.cloud = (uint32_t)cidx_cloud;
      r.cidx = le;
      cols[slot] = r;
    }
    if (ap) {
      const uint64_t as = wave_append(is_app, &counters[4], any);
      if (is_app && as < ap_cap) {
        ApparentPair p;
        p.s = le;
        p.t = t;
        p.diam = diam;
        p.cloud = (uint32_t)cidx_cloud;
        ap[as] = p;
      }
    }
  }
  // counters[] = &Scalars::columns: columns, apparent, nonapparent, candidates,
  // apparent_written, scan_steps, facet_steps
  unsigned long long tot[4] = {n_cols, n_app, n_steps, n_facets};
  unsigned long long* const dst[4] = {&counters[0], &counters[1], &counters[5], &counters[6]};
  add_block_counters<kBlock, 4>(tot, dst);
  (void)binom_g;
  (void)np1;
}

hipError_t launch_batch_edges(const uint32_t* W, const Cloud* clouds, int count,
                              int64_t total_edges, const uint32_t* bitmaps, Column* cols,
                              uint64_t cols_cap, ApparentPair* ap, uint64_t ap_cap,
                              ClearSet clear_out, unsigned long long* counters, int grid,
                              hipStream_t s) {
  if (total_edges <= 0) return hipSuccess;
  int64_t need = (total_edges + kBlock - 1) / kBlock;
  if (grid > need) grid = (int)need;
  batch_edges_kernel<<<grid, kBlock, 0, s>>>(W, clouds, count, total_edges, bitmaps, cols,
                                             cols_cap, ap, ap_cap, clear_out, nullptr, 0,
                                             counters);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Dimension-1 columns of one sparse cloud in neighbour mode (Sec. 5.3.13,
// Alg. 15 for d = 1): a one-wave workgroup takes a vertex a, lists its
// neighbours N(a) = {x : W(a, x) <= tau_eff} in LDS in increasing order (a
// ballot and a prefix count per 64 vertices of row a), and tests the
// columns (a, b) with b in N(a), b < a, not cleared. A cofacet {x, a, b}
// keeps the diameter only if x is in N(a), so condition 1 walks N(a) from
// the top instead of every x from n-1 down; everything else is the full
// scan's test.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(64) void edges_nb_kernel(
    const uint32_t* __restrict__ W, int n, const uint32_t* __restrict__ bm1,
    Column* __restrict__ cols, uint64_t cols_cap, ApparentPair* __restrict__ ap, uint64_t ap_cap,
    ClearSet clear_out, unsigned long long* __restrict__ counters) {
  extern __shared__ uint16_t nbl[];  // N(a), n entries at most
  const int lane = threadIdx.x;
  const BufferRows rows(W, n);
  const unsigned long long lower = (1ull << lane) - 1ull;
  unsigned long long n_cols = 0, n_app = 0, n_steps = 0, n_facets = 0;
  for (int a = blockIdx.x; a < n; a += gridDim.x) {
    uint32_t cnt = 0, below = 0;  // |N(a)| and its entries below a
    for (int x0 = 0; x0 < n; x0 += 64) {
      const int x = x0 + lane;
      const uint32_t w = rows.row_at(a, x < n ? x : n - 1);
      const bool in = x < n && w != kInf;  // the diagonal holds kInf
      const unsigned long long bal = __ballot(in);
      if (in) nbl[cnt + (uint32_t)__popcll(bal & lower)] = (uint16_t)x;
      cnt += (uint32_t)__popcll(bal);
      below += (uint32_t)__popcll(__ballot(in && x < a));
    }
    __syncthreads();
    for (uint32_t c0 = 0; c0 < below; c0 += 64) {
      const uint32_t ci = c0 + lane;
      bool is_col = false, is_app = false;
      uint32_t diam = kInf;
      uint64_t le = 0, t = 0;
      if (ci < below) {
        const int b = nbl[ci];
        le = edge_index(a, b);
        diam = rows.row_at(a, b);
        is_col = !((bm1[le >> 5] >> (le & 31)) & 1u);  // forest edges are cleared
        if (is_col) {
          ++n_cols;
          const int v[2] = {b, a};
          uint32_t pw[2][2];
          pw[1][0] = diam;
          uint32_t st = 0, fa = 0;
          const int x = apparent_cofacet_nb<1>(rows, n, v, pw, diam, nbl, cnt, st, fa);
          n_steps += st;
          n_facets += fa;
          if (x >= 0) {
            is_app = true;
            ++n_app;
            const int hi = max(x, a), lo = min(x, b), mid = x + a + b - hi - lo;
            t = (uint64_t)hi * (hi - 1) * (hi - 2) / 6 + (uint64_t)mid * (mid - 1) / 2 +
                (uint64_t)lo;
            clear_insert(clear_out, t);
          }
        }
      }
      bool any;
      const uint64_t slot = wave_append(is_col && !is_app, &counters[2], any);
      if (is_col && !is_app && slot < cols_cap) {
        Column r;
        r.key_hi = ~diam;
        r.cloud = 0;
        r.cidx = le;
        cols[slot] = r;
      }
      if (ap) {
        const uint64_t as = wave_append(is_app, &counters[4], any);
        if (is_app && as < ap_cap) {
          ApparentPair p;
          p.s = le;
          p.t = t;
          p.diam = diam;
          p.cloud = 0;
          ap[as] = p;
        }
      }
    }
    __syncthreads();  // the list is rebuilt for the next vertex
  }
  unsigned long long tot[4] = {n_cols, n_app, n_steps, n_facets};
  unsigned long long* const dst[4] = {&counters[0], &counters[1], &counters[5], &counters[6]};
  add_block_counters<64, 4>(tot, dst);
}

hipError_t launch_edges_nb(const uint32_t* W, int n, const uint32_t* bm1, Column* cols,
                           uint64_t cols_cap, ApparentPair* ap, uint64_t ap_cap,
                           ClearSet clear_out, unsigned long long* counters, int grid,
                           hipStream_t s) {
  if (n < 2) return hipSuccess;
  if (grid > n) grid = n;
  if (grid < 1) grid = 1;
  const size_t lds = ((size_t)n * sizeof(uint16_t) + 15) & ~(size_t)15;
  edges_nb_kernel<<<grid, 64, lds, s>>>(W, n, bm1, cols, cols_cap, ap, ap_cap, clear_out,
                                        counters);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// set clearing bits for the deaths found by the host reduction
// ---------------------------------------------------------------------------

__global__ void set_bits_kernel(const uint64_t* __restrict__ idx, int64_t count,
                                uint32_t* __restrict__ bitmap) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x) {
    uint64_t t = idx[i];
    atomicOr(&bitmap[t >> 5], 1u << (t & 31));
  }
}

__global__ void clear_insert_kernel(const uint64_t* __restrict__ idx, int64_t count,
                                    ClearSet set) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    clear_insert(set, idx[i]);
}

hipError_t launch_clear_insert(const uint64_t* idx, int64_t count, ClearSet set, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + kBlock - 1) / kBlock;
  if (blocks > 1024) blocks = 1024;
  clear_insert_kernel<<<(int)blocks, kBlock, 0, s>>>(idx, count, set);
  return hipGetLastError();
}

hipError_t launch_set_bits(const uint64_t* idx, int64_t count, uint32_t* bitmap, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  int64_t blocks = (count + kBlock - 1) / kBlock;
  if (blocks > 1024) blocks = 1024;
  set_bits_kernel<<<(int)blocks, kBlock, 0, s>>>(idx, count, bitmap);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// backward: scatter dL/d(value) onto the two points of each diameter edge
// ---------------------------------------------------------------------------

// Every edge entry must be -1 (no edge) or a point of X: a flag in device
// memory records any other value before the scatter reads X or writes gX.
__global__ void backward_check_kernel(const int32_t* __restrict__ edges, int64_t entries,
                                      int64_t n_total, uint32_t* __restrict__ bad) {
  bool out_of_range = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < entries;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e = edges[i];
    out_of_range |= e < -1 || (int64_t)e >= n_total;
  }
  if (__ballot(out_of_range) != 0 && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

__global__ void backward_kernel(const float* __restrict__ X, int m,
                                const int32_t* __restrict__ edges, int64_t npairs,
                                const float* __restrict__ g_birth,
                                const float* __restrict__ g_death, float* __restrict__ gX,
                                const uint32_t* __restrict__ bad) {
  if (*bad) return;  // an edge names no point of X: nothing is read or written
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < 2 * npairs;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t p = q >> 1;
    const int which = (int)(q & 1);  // 0 birth, 1 death
    const int u = edges[4 * p + 2 * which], v = edges[4 * p + 2 * which + 1];
    const float g = which ? g_death[p] : g_birth[p];
    if (u < 0 || v < 0 || g == 0.0f) continue;
    const float* xu = X + (int64_t)u * m;
    const float* xv = X + (int64_t)v * m;
    float s = 0.0f;
    for (int k = 0; k < m; ++k) {
      float d = xu[k] - xv[k];
      s += d * d;
    }
    if (s == 0.0f) continue;
    const float scale = g / sqrtf(s);
    for (int k = 0; k < m; ++k) {
      float d = (xu[k] - xv[k]) * scale;
      atomicAdd(&gX[(int64_t)u * m + k], d);
      atomicAdd(&gX[(int64_t)v * m + k], -d);
    }
  }
}

hipError_t launch_backward(const float* X, int64_t n_total, int m, const int32_t* edges,
                           int64_t npairs, const float* g_birth, const float* g_death, float* gX,
                           uint32_t* bad, hipStream_t s) {
  hipError_t e = launch_fill_u32(bad, 1, 0u, s);
  if (e != hipSuccess || npairs <= 0) return e;
  int64_t blocks = (4 * npairs + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  backward_check_kernel<<<(int)blocks, kBlock, 0, s>>>(edges, 4 * npairs, n_total, bad);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  blocks = (2 * npairs + kBlock - 1) / kBlock;
  if (blocks > 4096) blocks = 4096;
  backward_kernel<<<(int)blocks, kBlock, 0, s>>>(X, m, edges, npairs, g_birth, g_death, gX, bad);
  return hipGetLastError();
}

}  // namespace vrph
