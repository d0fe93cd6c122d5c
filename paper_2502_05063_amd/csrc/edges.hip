// The finite edges of one cloud's weight matrix as a list.
//
// A large cloud whose complex is sparse (most vertex pairs beyond the
// threshold) hands the host reduction its E finite edges, sorted by weight,
// instead of the n x n weights: the host builds its rank table from them in
// O(E) and never reads the matrix.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "vrph_internal.h"

namespace vrph {

// Rows a = 1 .. n-1 are strided over the workgroups; the lanes read
// W[a][0, a) (coalesced) and append each finite entry as a record {weight
// bits, 0, a << 32 | b}, with one returning atomic per wave. With out ==
// nullptr only *count is advanced; records past `cap` are counted, not
// written.
__global__ __launch_bounds__(kBlock) void finite_edges_kernel(const uint32_t* __restrict__ W, int n,
                                                              Column* __restrict__ out, uint64_t cap,
                                                              unsigned long long* __restrict__ count) {
  const int lane = threadIdx.x & 63;
  for (int a = 1 + (int)blockIdx.x; a < n; a += (int)gridDim.x) {
    const uint32_t* row = W + (size_t)a * (size_t)n;
    for (int b0 = 0; b0 < a; b0 += kBlock) {
      const int b = b0 + (int)threadIdx.x;
      const uint32_t w = b < a ? row[b] : kInf;
      const bool fin = w != kInf;
      const unsigned long long bal = __ballot(fin);
      if (!bal) continue;  // the same for the whole wave
      unsigned long long base = 0;
      if (lane == 0) base = atomicAdd(count, (unsigned long long)__popcll(bal));
      const uint32_t lo = __shfl((uint32_t)base, 0), hi = __shfl((uint32_t)(base >> 32), 0);
      base = ((unsigned long long)hi << 32) | lo;
      if (fin && out) {
        const unsigned long long k = base + (unsigned long long)__popcll(bal & ((1ull << lane) - 1));
        if (k < cap) out[k] = Column{w, 0u, ((uint64_t)a << 32) | (uint64_t)(uint32_t)b};
      }
    }
  }
}

hipError_t launch_finite_edges(const uint32_t* W, int n, Column* out, uint64_t cap,
                               unsigned long long* count, hipStream_t s) {
  if (n < 2) return hipSuccess;
  const int grid = n - 1 < 8192 ? n - 1 : 8192;
  finite_edges_kernel<<<grid, kBlock, 0, s>>>(W, n, out, cap, count);
  return hipGetLastError();
}

}  // namespace vrph
