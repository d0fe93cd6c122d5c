// Stable LSD radix sort of Column records (8-bit digits), used to put the
// non-apparent columns in coboundary order: diameter descending, index
// ascending (Alg. 18), grouped by cloud.
//
// Per digit pass, four kernels:
//   hist     per tile of kTile records, the digit histogram -> counts[digit][tile]
//   scans    exclusive scan of counts in digit-major order: each digit's row
//            by a workgroup of its own, then the 256 row totals -> offsets
//   scatter  per tile: stable rank of every record among the equal digits of
//            its tile (wave64 match by 8 ballots, cross-wave prefix in LDS),
//            records staged in LDS in digit order, then written out so that
//            consecutive lanes store consecutive addresses.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "vrph_internal.h"

namespace vrph {

constexpr int kSortThreads = 256;
constexpr int kSortItems = 8;
constexpr int kTile = kSortThreads * kSortItems;
constexpr int kRadix = 256;

struct Pass {
  int field;  // 0 cidx, 1 key_hi, 2 cloud
  int shift;
};

__device__ __forceinline__ uint32_t digit_of(const Column& r, Pass p) {
  uint64_t v = p.field == 0 ? r.cidx : (p.field == 1 ? (uint64_t)r.key_hi : (uint64_t)r.cloud);
  return (uint32_t)(v >> p.shift) & 0xFFu;
}

// The record count is `n`, or min(*n_dev, n) when n_dev is given (a count
// produced on the device, so that the sort can be recorded into a graph);
// tiles past the count contribute empty histograms.
__device__ __forceinline__ int64_t record_count(int64_t n, const unsigned long long* n_dev) {
  if (!n_dev) return n;
  const int64_t m = (int64_t)*n_dev;
  return m < n ? m : n;
}

__global__ __launch_bounds__(kSortThreads) void hist_kernel(const Column* __restrict__ a,
                                                            int64_t n_cap, const unsigned long long* n_dev,
                                                            Pass p,
                                                            uint32_t* __restrict__ counts,
                                                            int ntiles) {
  __shared__ uint32_t h[kRadix];
  const int64_t n = record_count(n_cap, n_dev);
  h[threadIdx.x] = 0;
  __syncthreads();
  const int64_t start = (int64_t)blockIdx.x * kTile;
  for (int i = 0; i < kSortItems; ++i) {
    int64_t r = start + (int64_t)i * kSortThreads + threadIdx.x;
    if (r < n) atomicAdd(&h[digit_of(a[r], p)], 1u);
  }
  __syncthreads();
  counts[(int64_t)threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Exclusive scan, in digit-major order, of the counters of the tiles that
// hold records (counts[digit * ntiles + tile], tile < active tiles), in two
// steps: every digit's row is scanned by a workgroup of its own (contiguous
// chunks per thread, then a scan of the chunk sums), which leaves the row's
// total in row_base[digit]; then one workgroup turns the 256 totals into
// the rows' starting offsets, which the scatter adds.
__global__ __launch_bounds__(kRadix) void row_scan_kernel(uint32_t* __restrict__ c, int ntiles,
                                                          int64_t n_cap,
                                                          const unsigned long long* n_dev,
                                                          uint32_t* __restrict__ row_base) {
  __shared__ uint32_t sums[kRadix];
  const int64_t n = record_count(n_cap, n_dev);
  const int act = (int)((n + kTile - 1) / kTile);
  uint32_t* row = c + (int64_t)blockIdx.x * ntiles;
  const int per = (act + kRadix - 1) / kRadix;
  const int b = threadIdx.x * per;
  const int e = b + per < act ? b + per : act;
  uint32_t s = 0;
  for (int i = b; i < e; ++i) s += row[i];
  sums[threadIdx.x] = s;
  __syncthreads();
  for (int o = 1; o < kRadix; o <<= 1) {
    const uint32_t x = threadIdx.x >= (unsigned)o ? sums[threadIdx.x - o] : 0;
    __syncthreads();
    sums[threadIdx.x] += x;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? sums[threadIdx.x - 1] : 0;
  for (int i = b; i < e; ++i) {
    const uint32_t x = row[i];
    row[i] = run;
    run += x;
  }
  if (threadIdx.x == kRadix - 1) row_base[blockIdx.x] = sums[kRadix - 1];
}

__global__ __launch_bounds__(kRadix) void base_scan_kernel(uint32_t* __restrict__ row_base) {
  __shared__ uint32_t t[kRadix];
  t[threadIdx.x] = row_base[threadIdx.x];
  __syncthreads();
  for (int o = 1; o < kRadix; o <<= 1) {
    const uint32_t x = threadIdx.x >= (unsigned)o ? t[threadIdx.x - o] : 0;
    __syncthreads();
    t[threadIdx.x] += x;
    __syncthreads();
  }
  row_base[threadIdx.x] = threadIdx.x ? t[threadIdx.x - 1] : 0;
}

__global__ __launch_bounds__(kSortThreads) void scatter_kernel(const Column* __restrict__ a,
                                                               Column* __restrict__ out,
                                                               int64_t n_cap,
                                                               const unsigned long long* n_dev,
                                                               Pass p,
                                                               const uint32_t* __restrict__ offs,
                                                               const uint32_t* __restrict__ row_base,
                                                               int ntiles) {
  __shared__ Column stage[kTile];
  __shared__ uint32_t wcnt[kSortThreads / 64][kRadix];
  __shared__ uint32_t running[kRadix];
  __shared__ uint32_t excl[kRadix];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t n = record_count(n_cap, n_dev);
  const int64_t start = (int64_t)blockIdx.x * kTile;
  if (start >= n) return;  // uniform across the workgroup
  const unsigned long long below = lane ? ((~0ull) >> (64 - lane)) : 0ull;

  for (int w = 0; w < kSortThreads / 64; ++w) wcnt[w][tid] = 0;
  running[tid] = 0;
  __syncthreads();

  Column rec[kSortItems];
  uint32_t dg[kSortItems], rank[kSortItems];
  bool valid[kSortItems];
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int64_t r = start + (int64_t)i * kSortThreads + tid;
    valid[i] = r < n;
    if (valid[i]) rec[i] = a[r];
    dg[i] = valid[i] ? digit_of(rec[i], p) : 0u;
  }
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    // lanes of this wave holding the same digit
    unsigned long long m = __ballot(valid[i]);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const bool bit = (dg[i] >> b) & 1u;
      const unsigned long long bb = __ballot(bit);
      m &= bit ? bb : ~bb;
    }
    if (valid[i]) {
      const int leader = __ffsll((long long)m) - 1;
      if (lane == leader) wcnt[wave][dg[i]] = (uint32_t)__popcll(m);
    }
    __syncthreads();
    if (valid[i]) {
      uint32_t r = running[dg[i]] + (uint32_t)__popcll(m & below);
      for (int w = 0; w < wave; ++w) r += wcnt[w][dg[i]];
      rank[i] = r;
    }
    __syncthreads();
    uint32_t add = 0;
    for (int w = 0; w < kSortThreads / 64; ++w) {
      add += wcnt[w][tid];
      wcnt[w][tid] = 0;
    }
    running[tid] += add;
    __syncthreads();
  }
  // exclusive scan of the tile's digit totals
  excl[tid] = running[tid];
  __syncthreads();
  for (int o = 1; o < kRadix; o <<= 1) {
    uint32_t x = tid >= o ? excl[tid - o] : 0;
    __syncthreads();
    excl[tid] += x;
    __syncthreads();
  }
  const uint32_t mine = excl[tid] - running[tid];
  __syncthreads();
  excl[tid] = mine;
  __syncthreads();
#pragma unroll
  for (int i = 0; i < kSortItems; ++i)
    if (valid[i]) stage[excl[dg[i]] + rank[i]] = rec[i];
  __syncthreads();
  const int64_t cnt = (n - start) < kTile ? (n - start) : kTile;
#pragma unroll
  for (int i = 0; i < kSortItems; ++i) {
    const int j = i * kSortThreads + tid;
    if (j < cnt) {
      const Column r = stage[j];
      const uint32_t d = digit_of(r, p);
      out[(int64_t)row_base[d] + offs[(int64_t)d * ntiles + blockIdx.x] + (j - excl[d])] = r;
    }
  }
}

// the tile counters, then the 256 row bases
size_t radix_sort_work_bytes(int64_t n) {
  int64_t ntiles = (n + kTile - 1) / kTile;
  if (ntiles < 1) ntiles = 1;
  return ((size_t)ntiles + 1) * kRadix * sizeof(uint32_t);
}

hipError_t radix_sort_columns(Column* a, Column* tmp, int64_t n, int cidx_bits, int cloud_bits,
                              void* work, hipStream_t s, const unsigned long long* n_dev,
                              bool* result_in_tmp) {
  if (result_in_tmp) *result_in_tmp = false;
  if (n <= 1 && !n_dev) return hipSuccess;
  if (n < 1) return hipSuccess;
  const int ntiles = (int)((n + kTile - 1) / kTile);
  uint32_t* counts = static_cast<uint32_t*>(work);
  uint32_t* row_base = counts + (size_t)ntiles * kRadix;
  Pass passes[8 + 4 + 4];
  int np = 0;
  for (int sh = 0; sh < cidx_bits; sh += 8) passes[np++] = {0, sh};
  for (int sh = 0; sh < 32; sh += 8) passes[np++] = {1, sh};
  for (int sh = 0; sh < cloud_bits; sh += 8) passes[np++] = {2, sh};
  Column* src = a;
  Column* dst = tmp;
  for (int i = 0; i < np; ++i) {
    hist_kernel<<<ntiles, kSortThreads, 0, s>>>(src, n, n_dev, passes[i], counts, ntiles);
    row_scan_kernel<<<kRadix, kRadix, 0, s>>>(counts, ntiles, n, n_dev, row_base);
    base_scan_kernel<<<1, kRadix, 0, s>>>(row_base);
    scatter_kernel<<<ntiles, kSortThreads, 0, s>>>(src, dst, n, n_dev, passes[i], counts,
                                                   row_base, ntiles);
    Column* t = src;
    src = dst;
    dst = t;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (src != a) {
    if (result_in_tmp) {
      *result_in_tmp = true;
      return hipSuccess;
    }
    return hipMemcpyAsync(a, src, (size_t)n * sizeof(Column), hipMemcpyDeviceToDevice, s);
  }
  return hipSuccess;
}

}  // namespace vrph
