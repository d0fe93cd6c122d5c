// Explicit boundary matrices on the device: the GPU scan of HYPHA (Sec.
// 4.3.2, Alg. 3-6) that settles the columns no column addition can change
// before the host reduces the rest (Sec. 4.3.3).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vrph_internal.h"

namespace vrph {

// ---------------------------------------------------------------------------
// Explicit boundary matrices: the GPU scan of Sec. 4.3.2 (Alg. 3-6) over a
// CSC matrix of ncols columns whose rows (strictly increasing within a
// column, all below the column: faces come first in a filtration) index the
// same cells as the columns. One lane per column; a column is short, so the
// lanes of a wave read one contiguous stretch of the row array.
//   left[r]   smallest column with a 1 in row r (atomicMin), ~0 if none
//   lookup[r] the column whose lowest 1 is the leftmost 1 of row r, else -1:
//             no column to its left can ever be added to it (a pivot of the
//             reduced matrix, Alg. 5), so it is stable
//   stable[j] zero columns, those pivots' columns and, with clearing, the
//             columns named by their rows (they reduce to zero: Lemma 4.2.3)
//   unstable  the other columns, one atomic per wave (any order)
//   destroyer[j] column j holds the leftmost 1 of some row, so it keeps a
//             pivot whatever is added to it (Lemma 4.2.5): in a boundary
//             matrix row j then never holds a pivot (Lemma 4.2.4), which
//             the host's compression uses
// err (bits): 1 col_ptr decreasing or out of range, 2 rows not strictly
// increasing, 4 a row outside [0, column).
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(kBlock) void bscan_init_kernel(int64_t n, uint32_t* __restrict__ left,
                                                            int32_t* __restrict__ lookup,
                                                            uint8_t* __restrict__ stable) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * kBlock) {
    left[j] = ~0u;
    lookup[j] = -1;
    stable[j] = 0;
  }
}

__global__ __launch_bounds__(kBlock) void bscan_leftmost_kernel(
    int64_t n, const int64_t* __restrict__ col_ptr, const int64_t* __restrict__ rows,
    int64_t nnz, uint32_t* __restrict__ left, uint8_t* __restrict__ stable,
    uint32_t* __restrict__ err) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * kBlock) {
    const int64_t b = col_ptr[j], e = col_ptr[j + 1];
    if (b < 0 || e < b || e > nnz) {
      atomicOr(err, 1u);
      continue;
    }
    if (b == e) {
      stable[j] = 1;  // a zero column
      continue;
    }
    const int64_t len = e - b;
    if (len <= 4) {
      // the usual case (a simplex of dimension <= 3): all rows, then all
      // their current minima, are loaded before any is used, so the loads
      // of a lane are in flight together
      int64_t r[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) r[k] = k < len ? rows[b + k] : 0;
      uint32_t bad = 0;
      int64_t prev = -1;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < len) {
          if (r[k] <= prev) bad |= 2u;
          if (r[k] < 0 || r[k] >= j) bad |= 4u;
          prev = r[k];
        }
      if (bad) {
        atomicOr(err, bad);
        continue;
      }
      // the minimum only falls, so a value already <= j makes the atomic a
      // no-op; the check reads L2 (where the atomics land) rather than this
      // CU's cache, which would hold older, larger values
      uint32_t cur[4];
#pragma unroll
      for (int k = 0; k < 4; ++k)
        cur[k] = k < len ? __hip_atomic_load(&left[r[k]], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                         : 0u;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        if (k < len && cur[k] > (uint32_t)j) atomicMin(&left[r[k]], (uint32_t)j);
      continue;
    }
    int64_t prev = -1;
    uint32_t bad = 0;
    for (int64_t q = b; q < e; ++q) {
      const int64_t r = rows[q];
      if (r <= prev) bad |= 2u;
      if (r < 0 || r >= j) {
        bad |= 4u;
        break;
      }
      prev = r;
      atomicMin(&left[r], (uint32_t)j);
    }
    if (bad) atomicOr(err, bad);
  }
}

__global__ __launch_bounds__(kBlock) void bscan_lookup_kernel(
    int64_t n, const int64_t* __restrict__ col_ptr, const int64_t* __restrict__ rows,
    int64_t nnz, const uint32_t* __restrict__ left, int32_t* __restrict__ lookup,
    uint8_t* __restrict__ stable, uint8_t* __restrict__ destroyer, int clearing) {
  for (int64_t j = (int64_t)blockIdx.x * kBlock + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * kBlock) {
    const int64_t b = col_ptr[j], e = col_ptr[j + 1];
    uint8_t holds_leftmost = 0;
    if (b >= 0 && e > b && e <= nnz) {  // not zero, not flagged by the scan
      int64_t r = -1;
      for (int64_t q = b; q < e; ++q) {
        r = rows[q];
        if (r < 0 || r >= j) break;  // flagged by the scan
        holds_leftmost |= left[r] == (uint32_t)j ? 1 : 0;
      }
      if (r >= 0 && r < j && left[r] == (uint32_t)j) {  // r: the lowest 1
        lookup[r] = (int32_t)j;
        stable[j] = 1;
        if (clearing) stable[r] = 1;
      }
    }
    destroyer[j] = holds_leftmost;
  }
}

// A workgroup takes kScanRounds x kBlock consecutive columns: it counts its
// unstable columns, reserves their slots with one atomic (one per
// workgroup: returning atomics on one address serialise across the chip),
// then writes them in order, a ballot per wave and round.
constexpr int kScanRounds = 16;

__global__ __launch_bounds__(kBlock) void bscan_unstable_kernel(int64_t n,
                                                                const uint8_t* __restrict__ stable,
                                                                int64_t* __restrict__ unstable,
                                                                unsigned long long* __restrict__ count) {
  __shared__ uint32_t wcount[kBlock / 64];
  __shared__ unsigned long long base;
  const int lane = (int)(threadIdx.x & 63), wave = (int)(threadIdx.x >> 6);
  const int64_t c0 = (int64_t)blockIdx.x * kBlock * kScanRounds;
  uint32_t mine = 0;
  for (int r = 0; r < kScanRounds; ++r) {
    const int64_t j = c0 + (int64_t)r * kBlock + threadIdx.x;
    mine += (j < n && !stable[j]) ? 1u : 0u;
  }
  // workgroup total: wave sums by shuffles, then the waves' sums
  for (int off = 32; off > 0; off >>= 1) mine += __shfl_down(mine, off);
  if (lane == 0) wcount[wave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int w = 0; w < kBlock / 64; ++w) tot += wcount[w];
    base = tot ? atomicAdd(count, tot) : 0ull;
  }
  __syncthreads();
  unsigned long long off = base;
  for (int r = 0; r < kScanRounds; ++r) {
    const int64_t j = c0 + (int64_t)r * kBlock + threadIdx.x;
    const bool un = j < n && !stable[j];
    const unsigned long long m = __ballot(un);
    __syncthreads();  // the previous round's wcount has been read
    if (lane == 0) wcount[wave] = (uint32_t)__popcll(m);
    __syncthreads();
    unsigned long long before = off;
    uint32_t round_total = 0;
    for (int w = 0; w < kBlock / 64; ++w) {
      if (w < wave) before += wcount[w];
      round_total += wcount[w];
    }
    if (un) unstable[before + (uint64_t)__popcll(m & ((1ull << lane) - 1ull))] = j;
    off += round_total;
  }
}

hipError_t launch_boundary_scan(int64_t n, const int64_t* col_ptr, const int64_t* rows, int64_t nnz,
                                uint32_t* left, int32_t* lookup, uint8_t* stable,
                                uint8_t* destroyer, int64_t* unstable, unsigned long long* count,
                                uint32_t* err, bool clearing, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  bscan_init_kernel<<<(int)blocks, kBlock, 0, s>>>(n, left, lookup, stable);
  bscan_leftmost_kernel<<<(int)blocks, kBlock, 0, s>>>(n, col_ptr, rows, nnz, left, stable, err);
  bscan_lookup_kernel<<<(int)blocks, kBlock, 0, s>>>(n, col_ptr, rows, nnz, left, lookup, stable,
                                                    destroyer, clearing ? 1 : 0);
  const int64_t ublocks = (n + (int64_t)kBlock * kScanRounds - 1) / ((int64_t)kBlock * kScanRounds);
  bscan_unstable_kernel<<<(unsigned)ublocks, kBlock, 0, s>>>(n, stable, unstable, count);
  return hipGetLastError();
}

}  // namespace vrph
