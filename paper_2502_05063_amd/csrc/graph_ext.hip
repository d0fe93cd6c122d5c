// Extended persistence of graphs with vertex values (Sec. 7.2, Alg. 27 and
// its PH0 building block Alg. 28), for a batch of graphs.
//
// Every graph gets the four barcodes of the coned graph's extended
// filtration: Ord0 (a vertex killed by an edge in the lower filtration),
// Rel1 (the same in the upper filtration), Ext0 (a component's minimum and
// maximum) and Ext1 (an edge closing a cycle in the lower filtration,
// killed by the cone triangle over an edge in the upper one). Layout:
//
//  - The edges of every graph are sorted twice over the whole batch by the
//    segmented radix sort of the columns (graph first): in the lower order
//    (F_low ascending, then F_up ascending, then edge id) and in the upper
//    order (F_up descending, then F_low descending, then edge id
//    descending), values compared as order-preserving integer images of
//    their float bits. A vertex compares by (f, vertex).
//  - One workgroup of one wave per graph then runs Alg. 28 on each order:
//    union-find with the elder rule (lower: the component whose oldest
//    vertex, its smallest, is younger dies; upper: the one whose largest is
//    smaller), 64 edges at a time: every lane finds its edge's two roots,
//    then the block's merges run in edge order on those labels in
//    registers, each merge renaming the killed root in every lane.
//  - Ext0: the final upper components, as (smallest vertex, largest
//    vertex), the root being the largest (Alg. 27, lines 3-4).
//  - Ext1 (Alg. 27, lines 5-20): the upper pass's negative edges form a
//    spanning forest T, rooted by a depth-first walk; every positive edge
//    (u, v), in the upper order, closes a cycle with T; its edge of largest
//    lower key (found by walking u and v up to their meeting vertex) is cut
//    and (u, v) is linked in its place (the cut side is re-rooted at u or v
//    by reversing its parent pointers), giving the bar (F_low of the cut
//    edge, F_up(u, v)). The walk is sequential, on one lane; the graphs of
//    a batch run in parallel.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vrph_internal.h"

namespace vrph {

namespace {

// order-preserving image of a finite float (with -0 taken as +0)
__device__ __forceinline__ uint32_t sortable(float x) {
  const uint32_t b = x == 0.0f ? 0u : __float_as_uint(x);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}

__device__ __forceinline__ int graph_of(const int64_t* off, int count, int64_t i) {
  int lo = 0, hi = count - 1;  // the last graph with off[g] <= i
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (off[mid] <= i)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

__device__ __forceinline__ int uf_find(uint32_t* parent, int x) {
  uint32_t p = parent[x];
  while (p != (uint32_t)x) {  // path halving
    const uint32_t pp = parent[p];
    parent[x] = pp;
    x = (int)p;
    p = pp;
  }
  return x;
}

}  // namespace

// Validation and the two sort records of every edge. err: bit 0 an edge
// endpoint outside its graph, bit 1 a loop, bit 2 a value that is not finite.
__global__ void gext_records_kernel(const int64_t* __restrict__ v_off,
                                    const int64_t* __restrict__ e_off, int count,
                                    int64_t total_edges, int64_t total_vertices,
                                    const float* __restrict__ f, const int32_t* __restrict__ edges,
                                    Column* __restrict__ lower, Column* __restrict__ upper,
                                    uint32_t* __restrict__ err) {
  uint32_t bad = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; v < total_vertices; v += stride)
    if (!isfinite(f[v])) bad |= 4u;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < total_edges; i += stride) {
    const int g = graph_of(e_off, count, i);
    const int64_t n = v_off[g + 1] - v_off[g];
    const int32_t a = edges[2 * i], b = edges[2 * i + 1];
    const uint32_t id = (uint32_t)(i - e_off[g]);
    if (a < 0 || b < 0 || a >= n || b >= n) {
      bad |= 1u;
      lower[i] = Column{0u, (uint32_t)g, (uint64_t)id};
      upper[i] = Column{0u, (uint32_t)g, (uint64_t)id};
      continue;
    }
    if (a == b) bad |= 2u;
    const uint32_t sa = sortable(f[v_off[g] + a]), sb = sortable(f[v_off[g] + b]);
    const uint32_t lo = sa > sb ? sa : sb, up = sa > sb ? sb : sa;  // F_low, F_up images
    lower[i] = Column{lo, (uint32_t)g, ((uint64_t)up << 32) | id};
    upper[i] = Column{~up, (uint32_t)g, ((uint64_t)(~lo) << 32) | (uint64_t)(~id)};
  }
  if (bad) atomicOr(err, bad);  // invalid input only
}

// One graph per workgroup of one wave. Dynamic LDS: 5 arrays of max_n
// words and one of max_n double words.
__global__ __launch_bounds__(64) void gext_graph_kernel(
    const int64_t* __restrict__ v_off, const int64_t* __restrict__ e_off,
    const float* __restrict__ f, const int32_t* __restrict__ edges,
    const Column* __restrict__ lower, const Column* __restrict__ upper, int max_n,
    uint32_t* __restrict__ pos_list, uint32_t* __restrict__ adj_off, uint32_t* __restrict__ adj,
    uint32_t* __restrict__ stack, uint32_t* __restrict__ err,
    vrph_ext_bar* __restrict__ bars) {
  if (*err) return;  // invalid input: nothing is indexed
  extern __shared__ uint32_t lds[];
  uint32_t* sf = lds;                 // sortable f of every vertex
  uint32_t* parent = lds + max_n;     // union-find; later the tree's parent pointers
  uint32_t* aux = lds + 2 * max_n;    // degree, then the tree's parent edge
  uint32_t* aux2 = lds + 3 * max_n;   // component minima; later the walk's marks
  uint32_t* aux3 = lds + 4 * max_n;   // component minimum vertex
  // the lower key (F_low image, F_up image) of every tree vertex's parent edge
  unsigned long long* tkey = reinterpret_cast<unsigned long long*>(lds + 5 * max_n);
  __shared__ uint32_t nbar, npos;
  const int g = blockIdx.x, lane = threadIdx.x;
  const int64_t v0 = v_off[g], e0 = e_off[g];
  const int n = (int)(v_off[g + 1] - v0);
  const int64_t m = e_off[g + 1] - e0;
  const int32_t* E = edges + 2 * e0;
  vrph_ext_bar* out = bars + v0 + e0;
  // a graph has exactly n + m bars; a write past them would be an error of
  // this code, and is reported instead of made
  const int64_t nslots = (int64_t)n + m;
  for (int v = lane; v < n; v += 64) {
    sf[v] = sortable(f[v0 + v]);
    parent[v] = (uint32_t)v;
    aux[v] = 0;
  }
  if (lane == 0) {
    nbar = 0;
    npos = 0;
  }
  __syncthreads();
  auto vkey = [&](int v) -> unsigned long long {
    return ((unsigned long long)sf[v] << 32) | (unsigned)v;
  };
  auto fval = [&](int v) -> float { return f[v0 + v]; };

  // Alg. 28 on one order (upper = false: lower filtration)
  for (int pass = 0; pass < 2; ++pass) {
    const bool up = pass == 1;
    const Column* rec = (up ? upper : lower) + e0;
    if (up) {
      for (int v = lane; v < n; v += 64) parent[v] = (uint32_t)v;
      __syncthreads();
    }
    for (int64_t base = 0; base < m; base += 64) {
      const int64_t i = base + lane;
      const bool live = i < m;
      uint32_t id = 0;
      int a = 0, b = 0, ra = 0, rb = 0;
      if (live) {
        const uint64_t c = rec[i].cidx;
        id = up ? ~(uint32_t)c : (uint32_t)c;
        a = E[2 * id];
        b = E[2 * id + 1];
        ra = uf_find(parent, a);
        rb = uf_find(parent, b);
      }
      __builtin_amdgcn_wave_barrier();
      const int cnt = m - base < 64 ? (int)(m - base) : 64;
      bool merged = false;
      int young = 0, old = 0;
      for (int j = 0; j < cnt; ++j) {
        const int A = __builtin_amdgcn_readlane(ra, j), B = __builtin_amdgcn_readlane(rb, j);
        if (A == B) continue;  // a cycle: a positive edge of this order
        // the elder rule: lower keeps the smaller vertex key, upper the larger
        const bool a_older = up ? vkey(A) > vkey(B) : vkey(A) < vkey(B);
        const int yg = a_older ? B : A, od = a_older ? A : B;
        if (lane == j) {
          merged = true;
          young = yg;
          old = od;
        }
        ra = ra == yg ? od : ra;
        rb = rb == yg ? od : rb;
      }
      // bars of the merges; positive upper edges listed in order
      const unsigned long long mm = __ballot(live && merged);
      uint32_t first = 0;
      if (lane == 0 && mm) first = atomicAdd(&nbar, (uint32_t)__popcll(mm));
      first = __shfl(first, 0);
      if (live && merged) {
        const uint32_t k = first + (uint32_t)__popcll(mm & ((1ull << lane) - 1));
        // F_low's vertex: the endpoint with the larger key; F_up's: the smaller
        const int dv = up ? (vkey(a) < vkey(b) ? a : b) : (vkey(a) > vkey(b) ? a : b);
        vrph_ext_bar r;
        r.kind = up ? VRPH_EXT_REL1 : VRPH_EXT_ORD0;
        r.birth = young;
        r.death = (int32_t)id;
        r.birth_value = fval(young);
        r.death_value = fval(dv);
        r.birth_vertex = young;
        r.death_vertex = dv;
        if (k < (uint32_t)nslots)
          out[k] = r;
        else
          atomicOr(err, 16u);
        parent[young] = (uint32_t)old;
        if (up) {  // a tree edge of T: count it at both ends
          atomicAdd(&aux[a], 1u);
          atomicAdd(&aux[b], 1u);
        }
      }
      if (up) {
        const unsigned long long pm = __ballot(live && !merged);
        uint32_t pf = 0;
        if (lane == 0 && pm) pf = atomicAdd(&npos, (uint32_t)__popcll(pm));
        pf = __shfl(pf, 0);
        if (live && !merged) pos_list[e0 + pf + (uint32_t)__popcll(pm & ((1ull << lane) - 1))] = id;
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
      __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
  }

  // Ext0: every final component's smallest and largest vertex (its root)
  for (int v = lane; v < n; v += 64) aux2[v] = 0xFFFFFFFFu;
  __syncthreads();
  for (int v = lane; v < n; v += 64) atomicMin(&aux2[uf_find(parent, v)], sf[v]);
  __syncthreads();
  for (int v = lane; v < n; v += 64) aux3[v] = 0xFFFFFFFFu;
  __syncthreads();
  for (int v = lane; v < n; v += 64) {
    const int r = uf_find(parent, v);
    if (sf[v] == aux2[r]) atomicMin(&aux3[r], (uint32_t)v);
  }
  __syncthreads();
  for (int v = lane; v < n; v += 64) {
    if (parent[v] != (uint32_t)v) continue;
    const int mv = (int)aux3[v];
    const uint32_t k = atomicAdd(&nbar, 1u);
    if (k < (uint32_t)nslots)
      out[k] = vrph_ext_bar{VRPH_EXT_EXT0, mv, v, fval(mv), fval(v), mv, v};
    else
      atomicOr(err, 16u);
  }
  __syncthreads();

  // the forest T of the upper pass's negative edges (the deaths of the Rel1
  // bars) as adjacency lists of edge ids (degrees counted in aux), rooted at
  // the union-find roots by a depth-first walk: parent vertex in `parent`,
  // parent edge in aux
  const int64_t ab = 2 * v0;  // adjacency region of this graph: 2(n - 1) entries at most
  if (lane == 0) {
    uint32_t run = 0;
    for (int v = 0; v < n; ++v) {
      adj_off[v0 + g + v] = run;
      run += aux[v];
      aux[v] = adj_off[v0 + g + v];  // fill cursor
    }
    adj_off[v0 + g + n] = run;
  }
  __syncthreads();
  const uint32_t nb = nbar;
  for (uint32_t k = lane; k < nb; k += 64) {
    const vrph_ext_bar r = out[k];
    if (r.kind != VRPH_EXT_REL1) continue;
    const int a = E[2 * r.death], b = E[2 * r.death + 1];
    adj[ab + atomicAdd(&aux[a], 1u)] = (uint32_t)r.death;
    adj[ab + atomicAdd(&aux[b], 1u)] = (uint32_t)r.death;
  }
  __syncthreads();
  __shared__ uint32_t q_e[64], q_u[64], q_v[64];
  __shared__ unsigned long long q_k[64];
  __shared__ uint32_t stop;
  if (lane == 0) stop = 0;

  // lower key of an edge: (F_low image, F_up image, id)
  auto lkey_hi = [&](uint32_t e) -> unsigned long long {
    const uint32_t sa = sf[E[2 * e]], sb = sf[E[2 * e + 1]];
    return ((unsigned long long)(sa > sb ? sa : sb) << 32) | (sa > sb ? sb : sa);
  };

  uint32_t* tpar = parent;
  uint32_t* tpe = aux;
  uint32_t* mark = aux2;
  if (lane == 0) {  // the rooting walk is sequential
    uint32_t top = 0;
    for (int v = 0; v < n; ++v) {
      mark[v] = 0;
      if (parent[v] == (uint32_t)v) stack[v0 + top++] = (uint32_t)v;
    }
    for (uint32_t q = 0; q < top; ++q) {
      const uint32_t r = stack[v0 + q];
      mark[r] = 1;
      tpe[r] = 0xFFFFFFFFu;  // tpar[r] == r already
    }
    while (top > 0) {
      const int x = (int)stack[v0 + --top];
      for (uint32_t q = adj_off[v0 + g + x]; q < adj_off[v0 + g + x + 1]; ++q) {
        const uint32_t e = adj[ab + q];
        const int y = E[2 * e] == x ? E[2 * e + 1] : E[2 * e];
        if (mark[y]) continue;
        mark[y] = 1;
        tpar[y] = (uint32_t)x;
        tpe[y] = e;
        tkey[y] = lkey_hi(e);
        stack[v0 + top++] = (uint32_t)y;
      }
    }
    for (int v = 0; v < n; ++v) mark[v] = 0;
  }  // lane 0
  __syncthreads();

  uint32_t nbk = nb;
  const uint32_t np = npos;
  // every walk below stays within one tree, so it takes fewer than n steps;
  // a walk that does not is an error of this code, reported instead of looping
  const int kSteps = 2 * n + 2;
  // Alg. 27, lines 11-19, for the positive edge staged in slot qi (edge
  // number q in the upper order); false on an internal error
  auto ext1_step = [&](uint32_t q, uint32_t qi) -> bool {
    const uint32_t e = q_e[qi];
    const int u = (int)q_u[qi], v = (int)q_v[qi];
    const uint32_t tag = 2 * q + 2;  // marks of this walk: tag (u's side), tag + 1 (v's side)
    // walk up from both ends, alternately, until one side meets the other
    int x = u, y = v, lca = -1, steps = 0;
    mark[x] = tag;
    if (mark[y] == tag)
      lca = y;
    else
      mark[y] = tag + 1;
    while (lca < 0 && steps++ < kSteps) {
      if (tpar[x] != (uint32_t)x) {
        x = (int)tpar[x];
        if (mark[x] == tag + 1) {
          lca = x;
          break;
        }
        mark[x] = tag;
      }
      if (tpar[y] != (uint32_t)y) {
        y = (int)tpar[y];
        if (mark[y] == tag) {
          lca = y;
          break;
        }
        mark[y] = tag + 1;
      }
    }
    if (lca < 0) return false;
    // the edge of largest lower key on the cycle: e and the tree edges from
    // u and from v up to lca
    uint32_t best = e;
    unsigned long long bkey = q_k[qi];
    int cut_child = -1;  // the vertex below the cut edge, -1 if e itself
    bool cut_u_side = false;
    int guard = 0;
    for (int z = u; z != lca && guard < kSteps; z = (int)tpar[z], ++guard) {
      const unsigned long long k = tkey[z];
      if (k > bkey || (k == bkey && tpe[z] > best)) {
        best = tpe[z];
        bkey = k;
        cut_child = z;
        cut_u_side = true;
      }
    }
    for (int z = v; z != lca && guard < 2 * kSteps; z = (int)tpar[z], ++guard) {
      const unsigned long long k = tkey[z];
      if (k > bkey || (k == bkey && tpe[z] > best)) {
        best = tpe[z];
        bkey = k;
        cut_child = z;
        cut_u_side = false;
      }
    }
    if (guard >= kSteps || nbk >= (uint32_t)nslots) return false;
    if (cut_child >= 0) {
      // cut (cut_child, its parent) and link e: re-root the cut side at its
      // endpoint of e by reversing the parent pointers up to cut_child
      int z = cut_u_side ? u : v;
      uint32_t prev = (uint32_t)(cut_u_side ? v : u), prev_e = e;
      unsigned long long prev_k = q_k[qi];
      for (int g2 = 0; g2 <= n; ++g2) {
        const uint32_t nz = tpar[z], ne = tpe[z];
        const unsigned long long nk = tkey[z];
        tpar[z] = prev;
        tpe[z] = prev_e;
        tkey[z] = prev_k;
        if (z == cut_child) break;
        prev = (uint32_t)z;
        prev_e = ne;
        prev_k = nk;
        z = (int)nz;
      }
    }
    const int ba = E[2 * best], bb = E[2 * best + 1];
    const int bv = vkey(ba) > vkey(bb) ? ba : bb;  // F_low(best)'s vertex
    const int dv = vkey(u) < vkey(v) ? u : v;      // F_up(e)'s vertex
    out[nbk++] = vrph_ext_bar{VRPH_EXT_EXT1, (int32_t)best, (int32_t)e, fval(bv), fval(dv), bv, dv};
    return true;
  };
  for (uint32_t q0 = 0; q0 < np; q0 += 64) {
    // the next 64 positive edges, staged by the whole wave; the walks are
    // sequential, on lane 0
    if (q0 + lane < np) {
      const uint32_t e = pos_list[e0 + q0 + lane];
      q_e[lane] = e;
      q_u[lane] = (uint32_t)E[2 * e];
      q_v[lane] = (uint32_t)E[2 * e + 1];
      q_k[lane] = lkey_hi(e);
    }
    __syncthreads();
    if (lane == 0 && !stop) {
      const uint32_t qend = np - q0 < 64 ? np - q0 : 64;
      for (uint32_t qi = 0; qi < qend; ++qi)
        if (!ext1_step(q0 + qi, qi)) {
          atomicOr(err, 16u);
          stop = 1;
          break;
        }
    }
    __syncthreads();
  }
}

hipError_t launch_graph_ext(const int64_t* v_off, const int64_t* e_off, int count,
                            int64_t total_vertices, int64_t total_edges, int max_n,
                            const float* f, const int32_t* edges, Column* lower, Column* upper,
                            Column* tmp, void* sort_work, uint32_t* pos_list, uint32_t* adj_off,
                            uint32_t* adj, uint32_t* stack, uint32_t* err, vrph_ext_bar* bars,
                            hipStream_t s) {
  hipError_t e = launch_fill_u32(err, 1, 0u, s);
  if (e != hipSuccess) return e;
  int64_t work = total_edges > total_vertices ? total_edges : total_vertices;
  int64_t blocks = (work + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  if (blocks < 1) blocks = 1;
  gext_records_kernel<<<(int)blocks, kBlock, 0, s>>>(v_off, e_off, count, total_edges,
                                                     total_vertices, f, edges, lower, upper, err);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  int cloud_bits = 0;
  while ((1 << cloud_bits) < count) ++cloud_bits;
  if (total_edges > 0) {
    if ((e = radix_sort_columns(lower, tmp, total_edges, 64, cloud_bits, sort_work, s)))
      return e;
    if ((e = radix_sort_columns(upper, tmp, total_edges, 64, cloud_bits, sort_work, s)))
      return e;
  }
  const size_t lds = (size_t)7 * (size_t)max_n * sizeof(uint32_t);
  if (lds > 65536 &&
      (e = hipFuncSetAttribute(reinterpret_cast<const void*>(gext_graph_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds)))
    return e;
  gext_graph_kernel<<<count, 64, lds, s>>>(v_off, e_off, f, edges, lower, upper, max_n, pos_list,
                                           adj_off, adj, stack, err, bars);
  return hipGetLastError();
}

// The gradient of a loss in the bar values with respect to f (the readout
// as a differentiable layer, Ch. 7): a bar's birth (death) value is f at its
// birth (death) vertex, so d(loss)/d(f) is the scatter of the loss's partial
// derivatives onto those vertices. Graph g's bars are [v_off[g] + e_off[g],
// v_off[g+1] + e_off[g+1]); its vertices start at v_off[g]. Pass 0 checks
// that every bar's two vertices lie in its graph (else *bad = 1); pass 1
// scatters, unless *bad is set. g_birth or g_death may be null (zero).
__global__ void gext_grad_kernel(int pass, const int64_t* __restrict__ v_off,
                                 const int64_t* __restrict__ e_off, int count, int64_t nbars,
                                 const vrph_ext_bar* __restrict__ bars,
                                 const float* __restrict__ g_birth,
                                 const float* __restrict__ g_death, float* __restrict__ g_f,
                                 uint32_t* __restrict__ bad) {
  if (pass == 1 && *bad) return;
  bool out = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nbars;
       i += (int64_t)gridDim.x * blockDim.x) {
    int lo = 0, hi = count - 1;  // the graph g with bar_off[g] <= i
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (v_off[mid] + e_off[mid] <= i)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t v0 = v_off[lo], n = v_off[lo + 1] - v0;
    const int32_t bv = bars[i].birth_vertex, dv = bars[i].death_vertex;
    if (pass == 0) {
      out |= bv < 0 || bv >= n || dv < 0 || dv >= n;
      continue;
    }
    if (g_birth && g_birth[i] != 0.0f) atomicAdd(&g_f[v0 + bv], g_birth[i]);
    if (g_death && g_death[i] != 0.0f) atomicAdd(&g_f[v0 + dv], g_death[i]);
  }
  if (pass == 0 && __ballot(out) != 0 && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

hipError_t launch_graph_ext_grad(const int64_t* v_off, const int64_t* e_off, int count,
                                 int64_t nbars, const vrph_ext_bar* bars, const float* g_birth,
                                 const float* g_death, float* g_f, uint32_t* bad,
                                 hipStream_t s) {
  if (count < 1 || nbars < 1) return hipSuccess;
  int64_t blocks = (nbars + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  for (int pass = 0; pass < 2; ++pass) {
    gext_grad_kernel<<<(unsigned)blocks, 256, 0, s>>>(pass, v_off, e_off, count, nbars, bars,
                                                       g_birth, g_death, g_f, bad);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace vrph
