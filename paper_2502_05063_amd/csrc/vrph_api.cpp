// C ABI of the library (include/vrph.h): argument checks, device workspaces,
// the per-dimension pipeline, result assembly and the batched path.
#include "vrph.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <iterator>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <functional>
#include <map>
#include <memory>
#include <new>
#include <queue>
#include <sstream>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "reduce.h"
#include "vrph_internal.h"


using namespace vrph;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------

static thread_local std::string g_last_error;

static vrph_status fail(vrph_status st, const std::string& msg) {
  g_last_error = msg;
  return st;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? VRPH_ENOMEM : VRPH_EDEVICE,                 \
                  std::string(#expr) + ": " + hipGetErrorString(e_));                     \
  } while (0)

// inside helpers that return a hipError_t
#define HIP_TRY_E(expr)             \
  do {                              \
    hipError_t e_ = (expr);         \
    if (e_ != hipSuccess) return e_; \
  } while (0)

extern "C" const char* vrph_last_error(void) { return g_last_error.c_str(); }

// Entry points that wait for their stream (to hand results back) cannot run
// under a caller's stream capture: they say so instead of breaking it.
static vrph_status check_not_capturing(hipStream_t s, const char* who) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(s, &cs) != hipSuccess) return VRPH_OK;  // the call itself reports
  if (cs != hipStreamCaptureStatusNone)
    return fail(VRPH_ESTATE, std::string(who) + ": called on a stream under capture");
  return VRPH_OK;
}

#define NOT_CAPTURING(s, who)                      \
  do {                                             \
    vrph_status st_ = check_not_capturing(s, who); \
    if (st_ != VRPH_OK) return st_;                \
  } while (0)

// ---------------------------------------------------------------------------
// buffers
// ---------------------------------------------------------------------------

namespace {

// Device buffer owned by a context or a batch plan: grows on demand, freed
// by release() or when its owner is deleted (also on an owner's failed set-up).
struct DevBuf {
  void* p = nullptr;
  size_t cap = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap && p) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipMalloc(&p, want);
    if (e == hipSuccess) cap = want;
    return e;
  }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    cap = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

struct HostPinned {
  void* p = nullptr;
  size_t cap = 0;
  HostPinned() = default;
  HostPinned(const HostPinned&) = delete;
  HostPinned& operator=(const HostPinned&) = delete;
  ~HostPinned() { release(); }
  hipError_t ensure(size_t bytes) {
    if (bytes <= cap && p) return hipSuccess;
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
    size_t want = std::max<size_t>(bytes, 256);
    hipError_t e = hipHostMalloc(&p, want, hipHostMallocDefault);
    if (e == hipSuccess) cap = want;
    return e;
  }
  void release() {
    if (p) (void)hipHostFree(p);
    p = nullptr;
    cap = 0;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

using u128 = unsigned __int128;

// k-major table C(v, k), v <= n, k <= kmax, by Pascal's rule; false if some
// entry reaches 2^63.
bool binomial_table(int n, int kmax, std::vector<uint64_t>& t) {
  t.assign((size_t)(kmax + 1) * (size_t)(n + 1), 0);
  std::vector<u128> prev(kmax + 1, 0), cur(kmax + 1, 0);
  const u128 lim = (u128)1 << 63;
  bool ok = true;
  for (int v = 0; v <= n; ++v) {
    for (int k = 0; k <= kmax; ++k) {
      u128 x = (k == 0) ? 1 : (v == 0 ? 0 : prev[k - 1] + prev[k]);
      if (x >= lim) {
        ok = false;
        x = lim;
      }
      cur[k] = x;
      t[(size_t)k * (n + 1) + v] = (uint64_t)x;
    }
    prev.swap(cur);
  }
  return ok;
}

uint32_t fbits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  return f == 0.0f ? 0u : u;
}

float bitsf(uint32_t u) {
  if (u == kInf) return INFINITY;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

int bits_needed(uint64_t x) {
  int b = 0;
  while (b < 64 && (x >> b) != 0) ++b;
  return b;
}

int host_threads() {
  const unsigned hc = std::thread::hardware_concurrency();
  return (int)std::max(1u, std::min(16u, hc ? hc : 1u));
}

double now_ms() {
  using namespace std::chrono;
  return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

}  // namespace

// ---------------------------------------------------------------------------
// context and results
// ---------------------------------------------------------------------------

// Launch setting of an enumeration kernel: suffixes per work unit (d >= 2)
// and workgroups per compute unit.
// largest work unit (suffixes) the defaults and the autotuner use; large
// units pay off where a threshold skips most prefixes
constexpr int kMaxChunk = 1 << 17;

// clouds from this size on may hand the host their finite edges instead of
// the n x n weights (when their complex is sparse)
constexpr int64_t kEdgeListMinN = 512;

struct Tune {
  int chunk;
  int mult;
};

struct vrph_ctx {
  int device = 0;
  int num_cus = 256;
  hipStream_t stream = nullptr;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  DevBuf D, W, binom, bitmaps, cols, cols_tmp, sort_work, ap, scal, clouds, cstate, h0, deaths;
  DevBuf wr16, rank_bits;  // 16-bit rank matrix and rank -> weight table (LDS kernels)
  DevBuf sink_ctr;         // region counters of the d >= 2 column sink
  DevBuf hset[kMaxDim + 2];  // hashed clearing sets, per dimension
  DevBuf hflag;              // their overflow flags
  uint64_t hslots[kMaxDim + 2] = {};  // slots the hashed sets last needed
  DevBuf ap_ctr, ap_tmp;   // region counters and packed output of the pair sink
  // the unfused order (VRPH_FULL_SORT): sink of every column, its counters
  // and total, the packed columns, the sort's spare buffer and work space
  DevBuf fcols, fctr, fpacked, fspare, fsort_work;
  uint64_t col_cap = 0;    // non-apparent columns the buffers are sized for
  uint64_t pair_cap = 0;   // apparent pairs the buffers are sized for
  HostPinned h_scal, h_cstate;
  HostPinned h_Wn;   // a single cloud's weights on the host (n x n)
  // or, for a large sparse cloud, its finite edges sorted by weight: device
  // records, the sort's spare buffer and work space, the count, host copies
  DevBuf fe_cols, fe_tmp, fe_work, fe_count;
  HostPinned h_fe, h_fe_count;
  RankTable ranks;   // its weight ranks (host reduction, LDS kernels)
  std::vector<uint64_t> h_binom;
  int binom_n = -1, binom_k = -1;
  std::string arch;
  // (dimension, size bucket, kernel variant: 0 global, 1 LDS, 2 the
  // dimension-1 neighbour-list kernel, 3 a batch plan: chunk = workgroup
  // size of the device reduction, mult = edge-kernel workgroups per CU) ->
  // setting
  std::map<std::tuple<int, int, int>, Tune> tuned;
  DevBuf units;                    // unit table of the d >= 2 enumeration
  DevBuf pfx_v, pfx_cum;           // listed prefixes of sparse dimension-2 and 3 enumerations
  DevBuf bscan;                    // scratch of the boundary-matrix scan
  DevBuf h0w;                      // scratch of H0 for large clouds
  DevBuf bflag;                    // edge check of the backward
  // extended persistence of graphs: offsets, sort records, per-graph scratch
  DevBuf g_off, g_lower, g_upper, g_tmp, g_pos, g_adj_off, g_adj, g_stack, g_err;
  std::vector<uint64_t> h_pfx_cum;
  std::vector<uint64_t> h_units;
};

// Work units of the d >= 2 enumeration kernel for tile `chunk`: cum[i] counts
// the units of all prefixes (v_d..v_2) with v_2 > n-1-i; a prefix with v_2 = t
// has C(n-1-t, d-2) choices of (v_d..v_3) and ceil(C(t,2)/chunk) chunks.
static uint64_t enum_units(int n, int d, int chunk, const std::vector<uint64_t>& binom,
                           std::vector<uint64_t>& cum) {
  auto C = [&](int v, int k) -> uint64_t { return binom[(size_t)k * (n + 1) + v]; };
  cum.assign((size_t)n + 1, 0);
  for (int i = 0; i < n; ++i) {
    const int t = n - 1 - i;
    uint64_t u = 0;
    if (t >= 2) {
      const uint64_t suf = (uint64_t)t * (t - 1) / 2;
      u = C(n - 1 - t, d - 2) * ((suf + chunk - 1) / chunk);
    }
    cum[i + 1] = cum[i] + u;
  }
  return cum[n];
}

// Work units over listed dimension-3 prefixes (edges v3 > v2, packed
// v3 << 16 | v2): cum[p] counts the units of the prefixes before p. The
// global-memory kernel enumerates a listed prefix's suffixes over the common
// neighbours of v3 and v2, one unit per prefix.
static uint64_t listed_units(const std::vector<uint32_t>& pv, std::vector<uint64_t>& cum) {
  cum.resize(pv.size() + 1);
  for (size_t p = 0; p <= pv.size(); ++p) cum[p] = p;
  return pv.size();
}

// Autotuning of the enumeration kernels' launch (see VRPH_AUTOTUNE).
static int size_bucket(int n) {
  int b = 1;
  while (b < n) b <<= 1;
  return b;
}

static void load_tuning(vrph_ctx* c) {
  const char* path = std::getenv("VRPH_TUNING_FILE");
  if (!path) return;
  std::ifstream f(path);
  std::string arch;
  int d, b, var, chunk, mult;
  while (f >> arch >> d >> b >> var >> chunk >> mult)
    if (arch == c->arch && d >= 1 && d <= kMaxDim && var >= 0 && var <= 3 &&
        chunk >= 64 && chunk <= (1 << 20) && chunk % 64 == 0 && mult >= 1 && mult <= 1024)
      c->tuned[{d, b, var}] = Tune{chunk, mult};
}

static void save_tuning(vrph_ctx* c, const std::tuple<int, int, int>& key, const Tune& t) {
  const char* path = std::getenv("VRPH_TUNING_FILE");
  if (!path) return;
  std::ofstream f(path, std::ios::app);
  f << c->arch << " " << std::get<0>(key) << " " << std::get<1>(key) << " " << std::get<2>(key)
    << " " << t.chunk << " " << t.mult << "\n";
}

struct vrph_barcode {
  std::vector<vrph_pair> pairs;  // canonical order
  int64_t off[VRPH_MAX_DIM + 3] = {0};
  vrph_stats stats;
};

extern "C" vrph_status vrph_create(int device, vrph_ctx** out) {
  if (!out) return fail(VRPH_EINVAL, "vrph_create: out is NULL");
  *out = nullptr;
  int ndev = 0;
  HIP_TRY(hipGetDeviceCount(&ndev));
  if (device < 0 || device >= ndev) return fail(VRPH_EINVAL, "vrph_create: no such device");
  HIP_TRY(hipSetDevice(device));
  std::unique_ptr<vrph_ctx> c(new (std::nothrow) vrph_ctx());
  if (!c) return fail(VRPH_ENOMEM, "vrph_create: out of host memory");
  c->device = device;
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, device));
  c->num_cus = prop.multiProcessorCount > 0 ? prop.multiProcessorCount : 256;
  c->arch = prop.gcnArchName;
  c->arch = c->arch.substr(0, c->arch.find(':'));
  load_tuning(c.get());
  // the device address of this device's fixed scratch array (allocation-free calls)
  HIP_TRY(noalloc_scratch_setup(device));
  // a blocking stream: ordered against the legacy default stream, which is where
  // torch puts work when the caller passes stream 0
  HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamDefault));
  HIP_TRY(hipEventCreate(&c->ev0));
  HIP_TRY(hipEventCreate(&c->ev1));
  HIP_TRY(hipEventCreate(&c->ev2));
  *out = c.release();
  return VRPH_OK;
}

extern "C" void vrph_destroy(vrph_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  DevBuf* bufs[] = {&c->D,      &c->W,     &c->binom,  &c->bitmaps, &c->cols,
                    &c->cols_tmp, &c->sort_work, &c->ap, &c->scal,  &c->clouds,
                    &c->cstate,  &c->h0,    &c->deaths, &c->units,   &c->wr16,
                    &c->rank_bits, &c->sink_ctr, &c->ap_ctr, &c->ap_tmp, &c->hflag,
                    &c->pfx_v,     &c->pfx_cum,  &c->bscan,  &c->h0w,
                    &c->bflag,     &c->g_off,    &c->g_lower, &c->g_upper, &c->g_tmp,
                    &c->g_pos,     &c->g_adj_off, &c->g_adj, &c->g_stack,  &c->g_err,
                    &c->fcols,     &c->fctr,      &c->fpacked, &c->fspare, &c->fsort_work,
                    &c->fe_cols,   &c->fe_tmp,    &c->fe_work, &c->fe_count};
  for (DevBuf* b : bufs) b->release();
  for (DevBuf& b : c->hset) b.release();
  c->h_scal.release();
  c->h_cstate.release();
  c->h_Wn.release();
  c->h_fe.release();
  c->h_fe_count.release();
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->ev2) (void)hipEventDestroy(c->ev2);
  if (c->stream) (void)hipStreamDestroy(c->stream);
  delete c;
}

extern "C" int64_t vrph_barcode_count(const vrph_barcode* bc, int32_t dim) {
  if (!bc) return 0;
  if (dim < 0) return (int64_t)bc->pairs.size();
  if (dim > VRPH_MAX_DIM) return 0;
  return bc->off[dim + 1] - bc->off[dim];
}

extern "C" const vrph_pair* vrph_barcode_pairs(const vrph_barcode* bc, int32_t dim) {
  if (!bc || bc->pairs.empty()) return nullptr;
  if (dim < 0) return bc->pairs.data();
  if (dim > VRPH_MAX_DIM) return nullptr;
  return bc->pairs.data() + bc->off[dim];
}

extern "C" const vrph_stats* vrph_barcode_stats(const vrph_barcode* bc) {
  return bc ? &bc->stats : nullptr;
}

extern "C" void vrph_barcode_free(vrph_barcode* bc) { delete bc; }

// ---------------------------------------------------------------------------
// pdist
// ---------------------------------------------------------------------------

// One cloud described for the batched kernels. The staging structs are
// pageable stack memory: the copy has consumed them when the call returns.
static vrph_status upload_single_cloud(vrph_ctx* c, int n, float threshold, hipStream_t s) {
  HIP_TRY(c->clouds.ensure(sizeof(Cloud)));
  HIP_TRY(c->cstate.ensure(sizeof(CloudState)));
  HIP_TRY(c->h_cstate.ensure(sizeof(CloudState)));
  Cloud cl;
  cl.x_off = 0;
  cl.w_off = 0;
  cl.e_off = 0;
  cl.bm_off = 0;
  cl.n = n;
  cl.tau_bits = std::isinf(threshold) ? 0x7F800000u : fbits(threshold);
  CloudState cs;
  cs.r_bits = kInf;
  cs.tau_bits = 0;
  cs.err = 0;
  cs.h0_count = 0;
  HIP_TRY(hipMemcpyAsync(c->clouds.p, &cl, sizeof(Cloud), hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(c->cstate.p, &cs, sizeof(CloudState), hipMemcpyHostToDevice, s));
  return VRPH_OK;
}

extern "C" vrph_status vrph_pdist(vrph_ctx* c, const float* X, int64_t n, int32_t m, float* D,
                                  void* hip_stream) {
  if (!c || !X || !D) return fail(VRPH_EINVAL, "vrph_pdist: NULL argument");
  if (n < 1 || n > kMaxN || m < 1) return fail(VRPH_EINVAL, "vrph_pdist: bad n or m");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
  vrph_status st = upload_single_cloud(c, (int)n, INFINITY, s);
  if (st) return st;
  HIP_TRY(launch_batch_pdist(X, m, c->clouds.as<Cloud>(), 1, n, D, s));
  HIP_TRY(hipStreamSynchronize(s));
  return VRPH_OK;
}

// ---------------------------------------------------------------------------
// the single-cloud pipeline
// ---------------------------------------------------------------------------

// Run f(begin, end) over [0, count) split into contiguous ranges on up to
// `threads` host threads (one when the range is small).
template <class F>
static void parallel_ranges(size_t count, int threads, F f) {
  const size_t min_per = 1 << 16;
  size_t t = std::min<size_t>((size_t)std::max(threads, 1), (count + min_per - 1) / min_per);
  if (t <= 1) {
    f((size_t)0, count);
    return;
  }
  std::vector<std::thread> pool;
  for (size_t i = 0; i < t; ++i)
    pool.emplace_back([&, i]() { f(count * i / t, count * (i + 1) / t); });
  for (std::thread& th : pool) th.join();
}

// std::sort of [first, last) on up to `threads` threads: sorted blocks,
// then rounds of pairwise merges.
template <class It, class Cmp>
static void parallel_sort(It first, It last, Cmp cmp, int threads) {
  const size_t n = (size_t)(last - first);
  size_t blocks = std::min<size_t>((size_t)std::max(threads, 1), n / (1 << 16));
  if (blocks <= 1) {
    std::sort(first, last, cmp);
    return;
  }
  std::vector<size_t> cut(blocks + 1);
  for (size_t i = 0; i <= blocks; ++i) cut[i] = n * i / blocks;
  {
    std::vector<std::thread> pool;
    for (size_t i = 0; i < blocks; ++i)
      pool.emplace_back([&, i]() { std::sort(first + cut[i], first + cut[i + 1], cmp); });
    for (std::thread& th : pool) th.join();
  }
  for (size_t width = 1; width < blocks; width *= 2) {
    std::vector<std::thread> pool;
    for (size_t i = 0; i + width < blocks; i += 2 * width) {
      const size_t lo = cut[i], mid = cut[i + width], hi = cut[std::min(i + 2 * width, blocks)];
      pool.emplace_back([=]() { std::inplace_merge(first + lo, first + mid, first + hi, cmp); });
    }
    for (std::thread& th : pool) th.join();
  }
}

// threads: host threads for the edge lookups and the sort (1 where the
// caller already runs one cloud per thread)
// Drops zero persistence (unless keep_zero), sorts canonically (dimension,
// birth, death) and sets the per-dimension offsets.
static void order_pairs(vrph_barcode* bc, bool keep_zero, int threads) {
  std::vector<vrph_pair>& P = bc->pairs;
  if (!keep_zero)
    P.erase(std::remove_if(P.begin(), P.end(),
                           [](const vrph_pair& p) { return !p.essential && p.birth_diam == p.death_diam; }),
            P.end());
  parallel_sort(P.begin(), P.end(), [](const vrph_pair& a, const vrph_pair& b) {
    if (a.dim != b.dim) return a.dim < b.dim;
    if (a.birth != b.birth) return a.birth < b.birth;
    return a.death < b.death;
  }, threads);
  for (int d = 0; d <= VRPH_MAX_DIM + 1; ++d) bc->off[d] = 0;
  for (const vrph_pair& p : P) bc->off[p.dim + 1]++;
  for (int d = 1; d <= VRPH_MAX_DIM + 2; ++d) bc->off[d] += bc->off[d - 1];
}

// Diameter edges of every pair from the host weights, then order_pairs.
static void finish_pairs(vrph_barcode* bc, const HostComplex& H, int max_dim, bool keep_zero,
                         int threads) {
  std::vector<vrph_pair>& P = bc->pairs;
  if (!keep_zero)
    P.erase(std::remove_if(P.begin(), P.end(),
                           [](const vrph_pair& p) { return !p.essential && p.birth_diam == p.death_diam; }),
            P.end());
  parallel_ranges(P.size(), threads, [&](size_t b, size_t e) {
    for (size_t i = b; i < e; ++i) {
      vrph_pair& p = P[i];
      p.birth_edge[0] = p.birth_edge[1] = -1;
      p.death_edge[0] = p.death_edge[1] = -1;
      if (p.dim >= 1) diameter_edge(H, p.birth, p.dim, &p.birth_edge[0], &p.birth_edge[1]);
      if (!p.essential) diameter_edge(H, p.death, p.dim + 1, &p.death_edge[0], &p.death_edge[1]);
    }
  });
  order_pairs(bc, keep_zero, threads);
  (void)max_dim;
}

static vrph_pair make_pair(int dim, uint64_t b, uint32_t bd, uint64_t d, uint32_t dd) {
  vrph_pair p;
  std::memset(&p, 0, sizeof(p));
  p.dim = dim;
  p.essential = d == ~0ull ? 1 : 0;
  p.birth = b;
  p.death = d == ~0ull ? UINT64_MAX : d;
  p.birth_diam = bitsf(bd);
  p.death_diam = p.essential ? INFINITY : bitsf(dd);
  return p;
}

// A sparse distance matrix as given to vrph_barcode_from_sparse (device arrays).
struct SparseInput {
  const int32_t* row;
  const int32_t* col;
  const float* val;
  int64_t nnz;
};

// D: the dense n x n matrix, or, with sp, the context's buffer that the
// sparse entries are written into first (+inf where a pair is not given).
// d_from_pdist: D is pdist's own output (symmetric by construction, so its
// validation skips the symmetry check)
static vrph_status barcode_impl(vrph_ctx* c, const float* D, int n, int max_dim, float threshold,
                                uint32_t flags, hipStream_t s, vrph_barcode** out,
                                const SparseInput* sp = nullptr, bool d_from_pdist = false) {
  const double t_start = now_ms();
  const bool keep_zero = flags & VRPH_KEEP_ZERO_PERSISTENCE;
  const int kmax = max_dim + 2;
  if (c->binom_n != n || c->binom_k != kmax) {
    if (!binomial_table(n, kmax, c->h_binom))
      return fail(VRPH_EOVERFLOW, "C(n, max_dim + 2) >= 2^63: simplex indices do not fit");
    HIP_TRY(c->binom.ensure(c->h_binom.size() * sizeof(uint64_t)));
    HIP_TRY(hipMemcpyAsync(c->binom.p, c->h_binom.data(), c->h_binom.size() * sizeof(uint64_t),
                           hipMemcpyHostToDevice, s));
    c->binom_n = n;
    c->binom_k = kmax;
  }
  HostComplex H;
  H.n = n;
  H.binom = c->h_binom.data();
  H.kmax = kmax;

  // clearing sets: dimension d's columns are C(n, d+1) indices. A bitmap
  // while it takes at most kBitmapBudget bytes, otherwise a hash set (with
  // VRPH_HASHED_CLEARING from dimension 2 on). Dimension 1 is always a
  // bitmap: the H0 kernel marks the forest edges there.
  constexpr uint64_t kBitmapBudget = 8ull << 30;
  std::vector<int64_t> bm_off(max_dim + 3, 0);
  std::vector<char> hashed(max_dim + 3, 0);
  int64_t words = 0;
  for (int d = 1; d <= max_dim + 1; ++d) {
    bm_off[d] = words;
    if (d > std::max(max_dim, 1)) continue;
    const uint64_t bits = H.C(n, d + 1);
    hashed[d] = d >= 2 && ((flags & VRPH_HASHED_CLEARING) || bits / 8 > kBitmapBudget);
    if (!hashed[d]) words += (int64_t)((bits + 31) / 32);
  }
  HIP_TRY(c->bitmaps.ensure((size_t)std::max<int64_t>(words, 1) * 4));
  uint32_t* bm = c->bitmaps.as<uint32_t>();
  HIP_TRY(launch_fill_u32(bm, words, 0u, s));
  HIP_TRY(c->hflag.ensure((kMaxDim + 2) * sizeof(uint32_t)));
  // (re)allocate and empty the hashed set of dimension d with `slots` slots
  auto make_hashed = [&](int d, uint64_t slots) -> hipError_t {
    hipError_t e = c->hset[d].ensure(slots * sizeof(unsigned long long));
    if (e == hipSuccess) e = launch_fill_u32(c->hset[d].as<uint32_t>(), (int64_t)(2 * slots), ~0u, s);
    if (e == hipSuccess) e = launch_fill_u32(c->hflag.as<uint32_t>() + d, 1, 0u, s);
    c->hslots[d] = slots;
    return e;
  };
  auto clear_set = [&](int d) -> ClearSet {
    ClearSet cs{nullptr, nullptr, 0, nullptr};
    if (d < 1 || d > max_dim) return cs;
    if (!hashed[d]) {
      cs.bits = bm + bm_off[d];
    } else {
      cs.keys = c->hset[d].as<unsigned long long>();
      cs.mask = c->hslots[d] - 1;
      cs.overflow = c->hflag.as<uint32_t>() + d;
    }
    return cs;
  };
  for (int d = 2; d <= max_dim; ++d)
    if (hashed[d]) HIP_TRY(make_hashed(d, std::max<uint64_t>(c->hslots[d], 1u << 20)));

  vrph_status st = upload_single_cloud(c, n, threshold, s);
  if (st) return st;
  HIP_TRY(c->W.ensure((size_t)n * n * 4));
  HIP_TRY(c->h0.ensure((size_t)n * sizeof(H0Pair)));
  if (sp)
    HIP_TRY(launch_sparse_matrix(sp->row, sp->col, sp->val, sp->nnz, n, const_cast<float*>(D),
                                 c->cstate.as<CloudState>(), s));
  // A large cloud whose complex is sparse (fewer than half of the vertex
  // pairs within the threshold) sends the host its finite edges sorted by
  // weight instead of the n x n weights, and the host builds its rank table
  // from them in O(edges) (VRPH_DENSE_HOST_WEIGHTS in the environment keeps
  // the matrix, for comparing the two). The weights kernel counts the
  // finite pairs.
  const uint64_t n_pairs = (uint64_t)n * (uint64_t)(n - 1) / 2;
  const bool count_edges =
      max_dim >= 1 && n >= kEdgeListMinN && !std::getenv("VRPH_DENSE_HOST_WEIGHTS");
  if (count_edges) {
    HIP_TRY(c->fe_count.ensure(sizeof(unsigned long long)));
    HIP_TRY(c->h_fe_count.ensure(sizeof(unsigned long long)));
    HIP_TRY(hipMemsetAsync(c->fe_count.p, 0, sizeof(unsigned long long), s));
  }
  HIP_TRY(hipEventRecord(c->ev0, s));
  HIP_TRY(launch_batch_validate_weights(D, c->clouds.as<Cloud>(), 1, n,
                                        !(flags & VRPH_NO_ENCLOSING_RADIUS), c->W.as<uint32_t>(),
                                        c->cstate.as<CloudState>(), s, sp != nullptr,
                                        !d_from_pdist,
                                        count_edges ? c->fe_count.as<unsigned long long>()
                                                    : nullptr));
  CloudState cs;
  // the weights on the host, in a pinned buffer the context keeps (no page
  // faults or zero fill per call, and the copy is a straight DMA)
  uint32_t* hW = nullptr;
  auto copy_weights = [&]() -> hipError_t {
    hipError_t e = c->h_Wn.ensure((size_t)n * n * 4);
    if (e != hipSuccess) return e;
    hW = c->h_Wn.as<uint32_t>();
    return hipMemcpyAsync(hW, c->W.p, (size_t)n * n * 4, hipMemcpyDeviceToHost, s);
  };
  // In edge-list mode the finite edges are listed before H0, whose Boruvka
  // rounds then scan that list instead of the rows of W.
  uint64_t n_finite = 0;
  bool edge_list = false;
  if (count_edges) {
    HIP_TRY(hipMemcpyAsync(c->h_fe_count.p, c->fe_count.p, sizeof(unsigned long long),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::memcpy(&n_finite, c->h_fe_count.p, sizeof(n_finite));
    edge_list = 2 * n_finite < n_pairs;
    if (edge_list) {
      const size_t m = (size_t)std::max<uint64_t>(n_finite, 1);
      HIP_TRY(c->fe_cols.ensure(m * sizeof(Column)));
      HIP_TRY(c->fe_tmp.ensure(m * sizeof(Column)));
      HIP_TRY(c->fe_work.ensure(radix_sort_work_bytes((int64_t)m)));
      HIP_TRY(c->h_fe.ensure(m * sizeof(Column)));
      HIP_TRY(hipMemsetAsync(c->fe_count.p, 0, sizeof(unsigned long long), s));
      HIP_TRY(launch_finite_edges(c->W.as<uint32_t>(), (int)n, c->fe_cols.as<Column>(), n_finite,
                                  c->fe_count.as<unsigned long long>(), s));
    }
  }
  // H0: one workgroup for small clouds; above kH0WideMin points the
  // Boruvka rounds are spread over the chip
  constexpr int kH0WideMin = 512;
  if (n >= kH0WideMin) {
    HIP_TRY(c->h0w.ensure(h0_wide_scratch_bytes(n)));
    HIP_TRY(launch_h0_wide(c->W.as<uint32_t>(), n, c->cstate.as<CloudState>(), c->h0.as<H0Pair>(),
                           bm + bm_off[1], c->h0w.p, s,
                           edge_list ? c->fe_cols.as<Column>() : nullptr,
                           edge_list ? (int64_t)n_finite : 0));
  } else {
    HIP_TRY(launch_batch_h0(c->W.as<uint32_t>(), c->clouds.as<Cloud>(), 1,
                            c->cstate.as<CloudState>(), c->h0.as<H0Pair>(), n, bm + bm_off[1], s));
  }
  HIP_TRY(hipEventRecord(c->ev1, s));
  HIP_TRY(hipMemcpyAsync(c->h_cstate.p, c->cstate.p, sizeof(CloudState), hipMemcpyDeviceToHost, s));
  if (edge_list) {
    // the host's copy, sorted by weight
    bool in_tmp = false;
    HIP_TRY(radix_sort_columns(c->fe_cols.as<Column>(), c->fe_tmp.as<Column>(), (int64_t)n_finite,
                               0, 0, c->fe_work.p, s, nullptr, &in_tmp));
    HIP_TRY(hipMemcpyAsync(c->h_fe.p, in_tmp ? c->fe_tmp.p : c->fe_cols.p,
                           (size_t)n_finite * sizeof(Column), hipMemcpyDeviceToHost, s));
  } else {
    HIP_TRY(copy_weights());
  }
  std::vector<H0Pair> h0(n);
  HIP_TRY(hipMemcpyAsync(h0.data(), c->h0.p, (size_t)n * sizeof(H0Pair), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  std::memcpy(&cs, c->h_cstate.p, sizeof(cs));
  if (cs.err)
    return fail(VRPH_EINVAL, std::string("invalid distance matrix:") +
                                 ((cs.err & 1) ? " non-finite" : "") + ((cs.err & 2) ? " negative" : "") +
                                 ((cs.err & 4) ? " asymmetric" : "") +
                                 ((cs.err & 8) ? " nonzero diagonal" : "") +
                                 ((cs.err & 16) ? " entry index out of range or on the diagonal" : "") +
                                 ((cs.err & 32) ? " repeated pair" : ""));
  RankTable& ranks = c->ranks;  // its storage is reused across calls
  const Column* fe = nullptr;  // the finite edges, sorted by weight (edge-list mode)
  if (edge_list) {
    fe = c->h_fe.as<Column>();
    ranks.build_from_edges((int)n, fe, (size_t)n_finite);
    ranks.attach(H);
  }
  H.W = hW;  // null in edge-list mode: the host reads ranks only
  // Weight ranks: needed by the host reduction and, for small clouds, by the
  // LDS enumeration kernels (16-bit ranks: C(kLdsMaxN, 2) < 0xFFFF).
  std::vector<uint16_t> h_wr16;
  const bool use_lds = max_dim >= 2 && n <= kLdsMaxN && !(flags & VRPH_NO_LDS);
  if (use_lds) {
    ranks.build(n, hW);
    ranks.attach(H);
    const size_t stride = (size_t)lds_stride((int)n);
    h_wr16.assign((size_t)n * stride, 0xFFFF);
    for (size_t a = 0; a < (size_t)n; ++a)
      for (size_t b = 0; b < (size_t)n; ++b) {
        const uint32_t r = ranks.Wr[a * (size_t)n + b];
        h_wr16[a * stride + b] = r == kInf ? (uint16_t)0xFFFF : (uint16_t)r;
      }
    HIP_TRY(c->wr16.ensure(h_wr16.size() * sizeof(uint16_t)));
    HIP_TRY(c->rank_bits.ensure(std::max<size_t>(ranks.bits.size(), 1) * sizeof(uint32_t)));
    HIP_TRY(hipMemcpyAsync(c->wr16.p, h_wr16.data(), h_wr16.size() * sizeof(uint16_t),
                           hipMemcpyHostToDevice, s));
    if (!ranks.bits.empty())
      HIP_TRY(hipMemcpyAsync(c->rank_bits.p, ranks.bits.data(),
                             ranks.bits.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  }

  // Dimensions 2 and 3 over a sparse edge set (at most half the vertex
  // pairs within the threshold): list the prefixes, the vertices v2 >= 2 and
  // the edges (v3 > v2 >= 2) within the threshold, largest v2 first; the
  // global-memory kernel then enumerates their suffixes over common
  // neighbours (see PrefixList).
  // Dimension 1 over a sparse edge set walks neighbour lists too
  // (launch_edges_nb).
  std::vector<uint32_t> pfx2, pfx3;
  bool sparse_edges = false;
  if (count_edges) {
    sparse_edges = edge_list;
  } else if (max_dim >= 1 && n >= 3) {
    // the lower triangle's finite entries, rows interleaved over threads
    std::atomic<uint64_t> valid{0};
    const int nt = n >= 2048 ? host_threads() : 1;
    auto count_rows = [&](int t) {
      uint64_t v = 0;
      for (size_t a = 1 + (size_t)t; a < (size_t)n; a += (size_t)nt)
        for (size_t b = 0; b < a; ++b) v += hW[a * n + b] != kInf;
      valid += v;
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(count_rows, t);
    count_rows(0);
    for (std::thread& th : pool) th.join();
    const uint64_t total = (uint64_t)n * (uint64_t)(n - 1) / 2;
    sparse_edges = 2 * valid.load() < total;
  }
  if (max_dim >= 2 && n >= 3 && !use_lds) {
    if (sparse_edges) {
      for (int v2 = n - 1; v2 >= 2; --v2) pfx2.push_back((uint32_t)v2);
      if (max_dim >= 3 && fe) {
        // the edges (v3 > v2 >= 2), v2 descending and v3 ascending: two
        // stable counting passes over the edge list, by v3 then by v2
        std::vector<uint32_t> tmp, cnt((size_t)n + 1);
        for (size_t k = 0; k < (size_t)n_finite; ++k)
          if ((uint32_t)fe[k].cidx >= 2) ++cnt[(size_t)(fe[k].cidx >> 32) + 1];
        for (size_t v = 1; v <= (size_t)n; ++v) cnt[v] += cnt[v - 1];
        tmp.resize(cnt[(size_t)n]);
        for (size_t k = 0; k < (size_t)n_finite; ++k) {
          const uint32_t v3 = (uint32_t)(fe[k].cidx >> 32), v2 = (uint32_t)fe[k].cidx;
          if (v2 >= 2) tmp[cnt[v3]++] = (v3 << 16) | v2;
        }
        std::fill(cnt.begin(), cnt.end(), 0u);
        for (uint32_t e : tmp) ++cnt[(size_t)(n - 1 - (int)(e & 0xFFFF)) + 1];
        for (size_t v = 1; v <= (size_t)n; ++v) cnt[v] += cnt[v - 1];
        pfx3.resize(tmp.size());
        for (uint32_t e : tmp) pfx3[cnt[(size_t)(n - 1 - (int)(e & 0xFFFF))]++] = e;
      } else if (max_dim >= 3) {
        for (int v2 = n - 2; v2 >= 2; --v2)
          for (int v3 = v2 + 1; v3 < n; ++v3)  // row v2 (W is symmetric): contiguous
            if (hW[(size_t)v2 * n + v3] != kInf) pfx3.push_back(((uint32_t)v3 << 16) | (uint32_t)v2);
      }
      HIP_TRY(c->pfx_v.ensure(std::max<size_t>(pfx2.size() + pfx3.size(), 1) * sizeof(uint32_t)));
      if (!pfx2.empty())
        HIP_TRY(hipMemcpyAsync(c->pfx_v.p, pfx2.data(), pfx2.size() * sizeof(uint32_t),
                               hipMemcpyHostToDevice, s));
      if (!pfx3.empty())
        HIP_TRY(hipMemcpyAsync(c->pfx_v.as<uint32_t>() + pfx2.size(), pfx3.data(),
                               pfx3.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
    }
  }
  // the listed prefixes of dimension d (empty: dense enumeration)
  auto prefixes = [&](int d) -> const std::vector<uint32_t>& {
    static const std::vector<uint32_t> none;
    return d == 2 ? pfx2 : d == 3 ? pfx3 : none;
  };

  std::unique_ptr<vrph_barcode> bc(new (std::nothrow) vrph_barcode());
  if (!bc) return fail(VRPH_ENOMEM, "out of host memory");
  std::memset(&bc->stats, 0, sizeof(bc->stats));
  bc->stats.tau_eff = bitsf(cs.tau_bits);
  bc->stats.max_dim = max_dim;
  float ms = 0;
  HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  bc->stats.gpu_ms[0] = ms;
  bc->stats.candidates[0] = n;
  bc->stats.columns[0] = n;
  for (uint32_t i = 0; i < cs.h0_count && i < (uint32_t)n; ++i) {
    const H0Pair& q = h0[i];
    bc->pairs.push_back(make_pair(0, q.birth, 0u, q.death, q.diam));
  }
  bc->stats.pairs[0] = cs.h0_count;

  HIP_TRY(c->scal.ensure(sizeof(Scalars)));
  HIP_TRY(c->h_scal.ensure(sizeof(Scalars)));
  std::vector<Column> hcols;
  std::vector<ApparentPair> hap;
  std::vector<PairRec> prs;
  std::vector<uint64_t> deaths;
  for (int d = 1; d <= max_dim; ++d) {
    const uint64_t ncand = H.C(n, d + 1);
    // the candidates the enumeration examines: all d-simplex indices, or,
    // over listed prefixes, the suffixes of the listed edges
    const std::vector<uint32_t>& pfx = prefixes(d);
    const uint32_t* const pfx_dev = c->pfx_v.as<uint32_t>() + (d == 3 ? pfx2.size() : 0);
    uint64_t examined = ncand;
    if (!pfx.empty()) {
      examined = 0;
      for (uint32_t pv : pfx) {
        const uint64_t v2 = pv & 0xFFFFu;
        examined += v2 * (v2 - 1) / 2;
      }
    }
    const ClearSet clear_in = clear_set(d);
    ClearSet clear_out = clear_set(d + 1);
    // output capacities grow on demand: the kernel counts past the end
    // without writing, and the dimension runs again with the exact need
    uint64_t cap = c->col_cap;
    if (cap < 4096) cap = std::min<uint64_t>(ncand, 1 << 16) + 1;
    // d >= 2: the kernel fills a ColumnSink in `cols`, which gather_columns
    // packs into `cols_tmp`; d = 1 appends to `cols` directly
    auto ensure_cols = [&]() -> hipError_t {
      hipError_t e = c->cols.ensure((d >= 2 ? sink_records(cap) : cap) * sizeof(Column));
      if (e == hipSuccess) e = c->cols_tmp.ensure(cap * sizeof(Column));
      return e;
    };
    uint64_t ap_cap = 0;
    if (keep_zero) {
      ap_cap = c->pair_cap;
      if (ap_cap < 4096) ap_cap = std::min<uint64_t>(ncand, 1 << 24) + 1;
    }
    // d >= 2: the pairs go to a sink in `ap`, packed into `ap_tmp`; d = 1
    // appends them to `ap` directly
    auto ensure_pairs = [&]() -> hipError_t {
      if (!keep_zero) return hipSuccess;
      hipError_t e = c->ap.ensure((d >= 2 ? sink_records(ap_cap) : std::max<uint64_t>(ap_cap, 1)) *
                                  sizeof(ApparentPair));
      if (e == hipSuccess && d >= 2) e = c->ap_tmp.ensure(ap_cap * sizeof(ApparentPair));
      if (e == hipSuccess && d >= 2)
        e = c->ap_ctr.ensure(kSinkCounters * sizeof(unsigned long long));
      return e;
    };
    Scalars sc;
    Scalars* dsc = c->scal.as<Scalars>();
    HIP_TRY(ensure_cols());
    HIP_TRY(c->sink_ctr.ensure(kSinkCounters * sizeof(unsigned long long)));
    HIP_TRY(ensure_pairs());
    // the launch of dimension d with setting t (suffixes per work unit for
    // d >= 2, workgroups per compute unit); `launched` = the workgroups.
    // Events ev0 / ev2 bracket the kernel alone on the stream.
    uint64_t launched = 0;
    auto launch_dim = [&](const Tune& t) -> hipError_t {
      const unsigned max_groups = (unsigned)c->num_cus * (unsigned)t.mult;
      if (d == 1) {
        HIP_TRY_E(hipEventRecord(c->ev0, s));
        if (sparse_edges) {
          launched = std::min<uint64_t>(max_groups, (uint64_t)n);
          HIP_TRY_E(launch_edges_nb(c->W.as<uint32_t>(), n, clear_in.bits, c->cols.as<Column>(),
                                    cap, keep_zero ? c->ap.as<ApparentPair>() : nullptr, ap_cap,
                                    clear_out, &dsc->columns, (int)launched, s));
        } else {
          launched = max_groups;
          HIP_TRY_E(launch_batch_edges(c->W.as<uint32_t>(), c->clouds.as<Cloud>(), 1,
                                       (int64_t)ncand, clear_in.bits, c->cols.as<Column>(), cap,
                                       keep_zero ? c->ap.as<ApparentPair>() : nullptr, ap_cap,
                                       clear_out, &dsc->columns, (int)max_groups, s));
        }
        return hipEventRecord(c->ev2, s);
      }
      // dimension 3 over a sparse edge set: list the prefixes (edges) instead
      PrefixList pl{nullptr, nullptr, 0};
      uint64_t units = 0;
      if (!pfx.empty()) {
        units = listed_units(pfx, c->h_pfx_cum);
        hipError_t e2 = c->pfx_cum.ensure(c->h_pfx_cum.size() * sizeof(uint64_t));
        if (e2 != hipSuccess) return e2;
        e2 = hipMemcpyAsync(c->pfx_cum.p, c->h_pfx_cum.data(),
                            c->h_pfx_cum.size() * sizeof(uint64_t), hipMemcpyHostToDevice, s);
        if (e2 != hipSuccess) return e2;
        pl = PrefixList{c->pfx_cum.as<uint64_t>(), pfx_dev, (uint32_t)pfx.size()};
      } else {
        units = enum_units(n, d, t.chunk, c->h_binom, c->h_units);
      }
      // LDS kernel: a unit per wave; global-memory kernel: a unit per workgroup
      const uint64_t units_per_group = use_lds ? kLdsBlock / 64 : 1;
      launched = std::min<uint64_t>(
          std::min<uint64_t>((units + units_per_group - 1) / units_per_group, max_groups),
          kMaxGroups);
      hipError_t e = c->units.ensure(c->h_units.size() * sizeof(uint64_t));
      if (e != hipSuccess) return e;
      e = hipMemcpyAsync(c->units.p, c->h_units.data(), c->h_units.size() * sizeof(uint64_t),
                         hipMemcpyHostToDevice, s);
      if (e != hipSuccess) return e;
      HIP_TRY_E(hipMemsetAsync(c->sink_ctr.p, 0, kSinkCounters * sizeof(unsigned long long), s));
      const ColumnSink sink{c->cols.as<Column>(), c->sink_ctr.as<unsigned long long>(),
                            sink_seg(cap), cap};
      PairSink aps{nullptr, nullptr, 0, 0};
      if (keep_zero) {
        HIP_TRY_E(hipMemsetAsync(c->ap_ctr.p, 0, kSinkCounters * sizeof(unsigned long long), s));
        aps = PairSink{c->ap.as<ApparentPair>(), c->ap_ctr.as<unsigned long long>(),
                       sink_seg(ap_cap), ap_cap};
      }
      // the paper's unfused order (VRPH_FULL_SORT), where it applies
      const bool full = (flags & VRPH_FULL_SORT) && use_lds && (d == 2 || d == 3) &&
                        pfx.empty() && !keep_zero && !clear_in.keys && !clear_out.keys;
      uint64_t fcap = 0;
      if (full) {
        fcap = std::max<uint64_t>(examined, 1);  // every candidate at most
        HIP_TRY_E(c->fcols.ensure(sink_records(fcap) * sizeof(Column)));
        HIP_TRY_E(c->fpacked.ensure(fcap * sizeof(Column)));
        HIP_TRY_E(c->fspare.ensure(fcap * sizeof(Column)));
        HIP_TRY_E(c->fctr.ensure((kSinkCounters + 1) * sizeof(unsigned long long)));
        HIP_TRY_E(c->fsort_work.ensure(radix_sort_work_bytes((int64_t)fcap)));
        HIP_TRY_E(hipMemsetAsync(c->fctr.p, 0, (kSinkCounters + 1) * sizeof(unsigned long long), s));
      }
      HIP_TRY_E(hipEventRecord(c->ev0, s));
      if (full) {
        const ColumnSink all{c->fcols.as<Column>(), c->fctr.as<unsigned long long>(),
                             sink_seg(fcap), fcap};
        unsigned long long* const fcount = c->fctr.as<unsigned long long>() + kSinkCounters;
        HIP_TRY_E(launch_enum_filter_lds(d, c->wr16.as<uint16_t>(), c->rank_bits.as<uint32_t>(),
                                         n, c->binom.as<uint64_t>(), t.chunk,
                                         c->units.as<uint64_t>(), units, max_groups, clear_in,
                                         all, dsc, s));
        HIP_TRY_E(launch_gather_columns(all, c->fpacked.as<Column>(), fcap, fcount, s));
        bool in_spare = false;
        HIP_TRY_E(radix_sort_columns(c->fpacked.as<Column>(), c->fspare.as<Column>(),
                                     (int64_t)fcap, bits_needed(ncand), 0, c->fsort_work.p, s,
                                     fcount, &in_spare));
        HIP_TRY_E(launch_apparent_sorted_lds(
            d, c->wr16.as<uint16_t>(), c->rank_bits.as<uint32_t>(), n, c->binom.as<uint64_t>(),
            in_spare ? c->fspare.as<Column>() : c->fpacked.as<Column>(), fcount, fcap,
            (unsigned)c->num_cus * 2, clear_out, sink, dsc, s));
      } else if (use_lds)
        HIP_TRY_E(launch_enum_apparent_lds(
            d, c->wr16.as<uint16_t>(), c->rank_bits.as<uint32_t>(), n, c->binom.as<uint64_t>(),
            t.chunk, c->units.as<uint64_t>(), units, pl, max_groups, clear_in, clear_out, sink,
            aps, dsc, s));
      else
        HIP_TRY_E(launch_enum_apparent(d, c->W.as<uint32_t>(), n, c->binom.as<uint64_t>(),
                                       t.chunk, c->units.as<uint64_t>(), units, pl,
                                       max_groups, clear_in, clear_out, sink, aps, dsc, s));
      HIP_TRY_E(hipEventRecord(c->ev2, s));
      HIP_TRY_E(launch_gather_columns(sink, c->cols_tmp.as<Column>(), cap, &dsc->nonapparent, s));
      if (keep_zero)
        HIP_TRY_E(launch_gather_pairs(aps, c->ap_tmp.as<ApparentPair>(), ap_cap,
                                      &dsc->apparent_written, s));
      // the host table is consumed by the copy before the next launch reuses it
      return hipStreamSynchronize(s);
    };
    const bool lds_dim = use_lds && d >= 2;
    const std::tuple<int, int, int> tkey{d, size_bucket(n),
                                         lds_dim ? 1 : (d == 1 && sparse_edges) ? 2 : 0};
    // LDS kernels: two workgroups of kLdsBlock lanes fill a compute unit.
    // Default work-unit size: the power of two in [64, 2^17] that gives the
    // unit takers of the default grid (waves of the LDS kernel, workgroups of
    // the other) about four units each.
    Tune param{64, lds_dim ? 2 : 8};
    {
      const uint64_t takers = (uint64_t)c->num_cus * (uint64_t)param.mult *
                              (uint64_t)(lds_dim ? kLdsBlock / 64 : 1);
      const uint64_t per = examined / std::max<uint64_t>(4 * takers, 1);
      while (param.chunk < kMaxChunk && (uint64_t)param.chunk * 2 <= per) param.chunk *= 2;
    }
    auto it = c->tuned.find(tkey);
    if (it != c->tuned.end()) {
      param = it->second;
    } else if ((flags & VRPH_AUTOTUNE) && !(flags & VRPH_FULL_SORT)) {
      // time settings on this very input (outputs are rewritten by the run
      // below): for d >= 2 the work-unit size and the workgroups per compute
      // unit, by coordinate search. One launch first sizes the outputs, so
      // that no trial runs with overfull column regions.
      HIP_TRY(hipMemsetAsync(c->scal.p, 0, sizeof(Scalars), s));
      HIP_TRY(launch_dim(param));
      HIP_TRY(hipMemcpyAsync(c->h_scal.p, c->scal.p, sizeof(Scalars), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      std::memcpy(&sc, c->h_scal.p, sizeof(sc));
      if (sc.nonapparent > cap) cap = sc.nonapparent + 1024;
      if (keep_zero && sc.apparent_written > ap_cap) ap_cap = sc.apparent_written + 1024;
      HIP_TRY(ensure_cols());
      HIP_TRY(ensure_pairs());
      float best = -1;
      auto trial = [&](const Tune& t) -> hipError_t {
        HIP_TRY_E(hipMemsetAsync(c->scal.p, 0, sizeof(Scalars), s));
        HIP_TRY_E(launch_dim(t));
        HIP_TRY_E(hipEventSynchronize(c->ev2));
        float ms = 0;
        HIP_TRY_E(hipEventElapsedTime(&ms, c->ev0, c->ev2));
        if (best < 0 || ms < best) {
          best = ms;
          param = t;
        }
        return hipSuccess;
      };
      // two rounds of coordinate search: unit sizes at the current grid,
      // then grids at the current unit size
      // unit sizes that would give far more units than the default are not
      // tried: each unit costs a decode even where its prefix is skipped
      std::vector<uint64_t> scratch;
      const bool listed = !pfx.empty();  // unit size has no effect then
      auto units_for = [&](int chunk) -> uint64_t {
        return listed ? listed_units(pfx, scratch) : enum_units(n, d, chunk, c->h_binom, scratch);
      };
      const uint64_t unit_limit = std::max<uint64_t>(4 * units_for(param.chunk), 1u << 24);
      for (int round = 0; round < 2; ++round) {
        if (d >= 2 && !listed) {
          const int mult = param.mult;
          for (int chunk = 64; chunk <= kMaxChunk; chunk *= 2)
            if (units_for(chunk) <= unit_limit) HIP_TRY(trial(Tune{chunk, mult}));
        }
        const int chunk = param.chunk;
        for (int mult : {1, 2, 4, 8, 16, 32, 64})
          if (!lds_dim || mult <= 4) HIP_TRY(trial(Tune{chunk, mult}));
        if (d < 2) break;
      }
      c->tuned[tkey] = param;
      save_tuning(c, tkey, param);
    }
    // A hashed set of dimension d+1 receives at most one index per column
    // of dimension d (its apparent cofacet or its death); it is kept at four
    // slots per column or more (load <= 1/4).
    auto hashed_out_ok = [&](uint32_t overflow) {
      return !clear_out.keys || (!overflow && c->hslots[d + 1] >= 4 * sc.columns);
    };
    for (int attempt = 0; attempt < 3; ++attempt) {
      HIP_TRY(ensure_cols());
      HIP_TRY(ensure_pairs());
      HIP_TRY(hipMemsetAsync(c->scal.p, 0, sizeof(Scalars), s));
      HIP_TRY(launch_dim(param));
      bc->stats.grid[d] = (int32_t)std::min<uint64_t>(launched, 0x7FFFFFFF);
      HIP_TRY(hipMemcpyAsync(c->h_scal.p, c->scal.p, sizeof(Scalars), hipMemcpyDeviceToHost, s));
      uint32_t hov = 0;
      if (clear_out.keys)
        HIP_TRY(hipMemcpyAsync(&hov, clear_out.overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));
      std::memcpy(&sc, c->h_scal.p, sizeof(sc));
      const bool sets_ok = hashed_out_ok(hov);
      if (sc.nonapparent <= cap && (!keep_zero || sc.apparent_written <= ap_cap) && sets_ok) break;
      cap = std::max<uint64_t>(cap, sc.nonapparent + 1024);
      if (keep_zero) ap_cap = std::max<uint64_t>(ap_cap, sc.apparent_written + 1024);
      if (!sets_ok) {
        uint64_t slots = 1u << 20;
        while (slots < 4 * sc.columns) slots <<= 1;
        HIP_TRY(make_hashed(d + 1, slots));
        clear_out = clear_set(d + 1);
      }
    }
    if (sc.nonapparent > cap || (keep_zero && sc.apparent_written > ap_cap))
      return fail(VRPH_EDEVICE, "column counts changed between two runs of one dimension");
    if (!hashed_out_ok(0))
      return fail(VRPH_EDEVICE, "clearing set of the next dimension overflowed");
    c->col_cap = std::max(c->col_cap, cap);
    if (keep_zero) c->pair_cap = std::max(c->pair_cap, ap_cap);
    const int64_t nna = (int64_t)sc.nonapparent;
    Column* const packed = d >= 2 ? c->cols_tmp.as<Column>() : c->cols.as<Column>();
    Column* const spare = d >= 2 ? c->cols.as<Column>() : c->cols_tmp.as<Column>();
    HIP_TRY(c->sort_work.ensure(radix_sort_work_bytes(nna)));
    HIP_TRY(radix_sort_columns(packed, spare, nna, bits_needed(ncand), 0, c->sort_work.p, s));
    HIP_TRY(hipEventRecord(c->ev1, s));
    hcols.resize(nna);
    if (nna) HIP_TRY(hipMemcpyAsync(hcols.data(), packed, nna * sizeof(Column), hipMemcpyDeviceToHost, s));
    if (keep_zero) {
      hap.resize(sc.apparent_written);
      if (sc.apparent_written)
        HIP_TRY(hipMemcpyAsync(hap.data(), d >= 2 ? c->ap_tmp.p : c->ap.p,
                               sc.apparent_written * sizeof(ApparentPair),
                               hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipStreamSynchronize(s));
    HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev1));
    bc->stats.gpu_ms[d] = ms;
    HIP_TRY(hipEventElapsedTime(&ms, c->ev0, c->ev2));
    bc->stats.apparent_ms[d] = ms;
    bc->stats.cofacets[d] = (int64_t)sc.scan_steps;
    bc->stats.facets[d] = (int64_t)sc.facet_steps;
    // over listed prefixes the kernel counts the suffixes it enumerated
    bc->stats.candidates[d] = !pfx.empty() ? (int64_t)sc.candidates : (int64_t)examined;
    bc->stats.columns[d] = (int64_t)sc.columns;
    bc->stats.apparent[d] = (int64_t)sc.apparent;
    bc->stats.reduced[d] = nna;

    const double h0t = now_ms();
    prs.clear();
    deaths.clear();
    ReduceStats rs;
    if (nna > 0 && !H.Wr) {  // not built yet (no LDS kernel in this call)
      ranks.build(n, hW);
      ranks.attach(H);
    }
    reduce_dimension(H, d, hcols.data(), nna, host_threads(), prs, deaths, rs);
    bc->stats.additions[d] = rs.additions;
    bc->stats.emergent[d] = rs.emergent;
    bc->pairs.reserve(bc->pairs.size() + prs.size() + (keep_zero ? hap.size() : 0));
    for (const PairRec& r : prs) bc->pairs.push_back(make_pair(d, r.birth, r.bdiam, r.death, r.ddiam));
    if (keep_zero) {
      const size_t base = bc->pairs.size();
      bc->pairs.resize(base + hap.size());
      parallel_ranges(hap.size(), host_threads(), [&](size_t b, size_t e) {
        for (size_t i = b; i < e; ++i)
          bc->pairs[base + i] = make_pair(d, hap[i].s, hap[i].diam, hap[i].t, hap[i].diam);
      });
    }
    bc->stats.pairs[d] = (int64_t)prs.size() + (int64_t)sc.apparent;
    bc->stats.host_ms[d] = now_ms() - h0t;
    if ((clear_out.bits || clear_out.keys) && !deaths.empty()) {
      HIP_TRY(c->deaths.ensure(deaths.size() * sizeof(uint64_t)));
      HIP_TRY(hipMemcpyAsync(c->deaths.p, deaths.data(), deaths.size() * sizeof(uint64_t),
                             hipMemcpyHostToDevice, s));
      HIP_TRY(launch_clear_insert(c->deaths.as<uint64_t>(), (int64_t)deaths.size(), clear_out, s));
      uint32_t hov = 0;
      if (clear_out.keys)
        HIP_TRY(hipMemcpyAsync(&hov, clear_out.overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
      HIP_TRY(hipStreamSynchronize(s));  // `deaths` is reused by the next dimension
      if (hov) return fail(VRPH_EDEVICE, "clearing set of the next dimension overflowed");
    }
  }
  finish_pairs(bc.get(), H, max_dim, keep_zero, host_threads());
  bc->stats.total_ms = now_ms() - t_start;
  *out = bc.release();
  return VRPH_OK;
}

constexpr uint32_t kKnownFlags = VRPH_KEEP_ZERO_PERSISTENCE | VRPH_NO_ENCLOSING_RADIUS |
                                 VRPH_AUTOTUNE | VRPH_NO_LDS | VRPH_HASHED_CLEARING |
                                 VRPH_FULL_SORT;

static vrph_status check_common(vrph_ctx* c, int64_t n, int32_t max_dim, float threshold,
                                uint32_t flags, vrph_barcode** out) {
  if (!c || !out) return fail(VRPH_EINVAL, "NULL context or output");
  *out = nullptr;
  if (flags & ~kKnownFlags) return fail(VRPH_EINVAL, "unknown flag bits");
  if (n < 1 || n > kMaxN) return fail(VRPH_EINVAL, "n must be in [1, 16384]");
  if (max_dim < 0 || max_dim > VRPH_MAX_DIM) return fail(VRPH_EINVAL, "max_dim out of range");
  if (std::isnan(threshold) || threshold < 0) return fail(VRPH_EINVAL, "threshold must be >= 0");
  return VRPH_OK;
}

extern "C" vrph_status vrph_barcode_from_dist(vrph_ctx* c, const float* D, int64_t n,
                                              int32_t max_dim, float threshold, uint32_t flags,
                                              void* hip_stream, vrph_barcode** out) {
  vrph_status st = check_common(c, n, max_dim, threshold, flags, out);
  if (st) return st;
  if (!D) return fail(VRPH_EINVAL, "D is NULL");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
  NOT_CAPTURING(s, "vrph_barcode_from_dist");
  return barcode_impl(c, D, (int)n, max_dim, threshold, flags, s, out);
}

extern "C" vrph_status vrph_barcode_from_points(vrph_ctx* c, const float* X, int64_t n,
                                                int32_t m, int32_t max_dim, float threshold,
                                                uint32_t flags, void* hip_stream,
                                                vrph_barcode** out) {
  vrph_status st = check_common(c, n, max_dim, threshold, flags, out);
  if (st) return st;
  if (!X || m < 1) return fail(VRPH_EINVAL, "X is NULL or m < 1");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
  NOT_CAPTURING(s, "vrph_barcode_from_points");
  HIP_TRY(c->D.ensure((size_t)n * n * 4));
  st = upload_single_cloud(c, (int)n, INFINITY, s);
  if (st) return st;
  HIP_TRY(launch_batch_pdist(X, m, c->clouds.as<Cloud>(), 1, n, c->D.as<float>(), s));
  return barcode_impl(c, c->D.as<float>(), (int)n, max_dim, threshold, flags, s, out, nullptr,
                      true);
}

extern "C" vrph_status vrph_barcode_from_sparse(vrph_ctx* c, int64_t n, int64_t nnz,
                                                const int32_t* row, const int32_t* col,
                                                const float* val, int32_t max_dim,
                                                float threshold, uint32_t flags,
                                                void* hip_stream, vrph_barcode** out) {
  vrph_status st = check_common(c, n, max_dim, threshold, flags, out);
  if (st) return st;
  if (nnz < 0 || nnz > n * (n - 1) / 2)
    return fail(VRPH_EINVAL, "nnz must be in [0, n(n-1)/2]");
  if (nnz > 0 && (!row || !col || !val)) return fail(VRPH_EINVAL, "row, col or val is NULL");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
  NOT_CAPTURING(s, "vrph_barcode_from_sparse");
  HIP_TRY(c->D.ensure((size_t)n * n * 4));
  const SparseInput sp{row, col, val, nnz};
  return barcode_impl(c, c->D.as<float>(), (int)n, max_dim, threshold, flags, s, out, &sp);
}

// ---------------------------------------------------------------------------
// backward
// ---------------------------------------------------------------------------

extern "C" vrph_status vrph_backward(vrph_ctx* c, const float* X, int64_t n_total, int32_t m,
                                     const int32_t* edges, int64_t npairs, const float* g_birth,
                                     const float* g_death, float* gX, void* hip_stream) {
  if (!c || !X || !gX || m < 1 || n_total < 0 || npairs < 0)
    return fail(VRPH_EINVAL, "vrph_backward: bad argument");
  if (npairs > 0 && (!edges || !g_birth || !g_death))
    return fail(VRPH_EINVAL, "vrph_backward: NULL pair arrays");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
  NOT_CAPTURING(s, "vrph_backward");
  HIP_TRY(c->bflag.ensure(sizeof(uint32_t)));
  HIP_TRY(launch_backward(X, n_total, m, edges, npairs, g_birth, g_death, gX,
                          c->bflag.as<uint32_t>(), s));
  uint32_t bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, c->bflag.p, sizeof(bad), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (bad)
    return fail(VRPH_EINVAL, "vrph_backward: an edge entry is neither -1 nor a point in [0, n_total)");
  return VRPH_OK;
}

extern "C" vrph_status vrph_backward_noalloc(vrph_ctx* c, const float* X, int64_t n_total,
                                             int32_t m, const int32_t* edges, int64_t npairs,
                                             const float* g_birth, const float* g_death,
                                             float* gX, void* hip_stream) {
  if (!c || !X || !gX || m < 1 || n_total < 0 || npairs < 0)
    return fail(VRPH_EINVAL, "vrph_backward_noalloc: bad argument");
  if (npairs > 0 && (!edges || !g_birth || !g_death))
    return fail(VRPH_EINVAL, "vrph_backward_noalloc: NULL pair arrays");
  uint32_t* bad = noalloc_scratch(c->device);
  if (!bad) return fail(VRPH_ESTATE, "vrph_backward_noalloc: scratch of this device not set up");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
  NOT_CAPTURING(s, "vrph_backward_noalloc");
  HIP_TRY(launch_backward(X, n_total, m, edges, npairs, g_birth, g_death, gX, bad, s));
  uint32_t flag = 0;
  HIP_TRY(hipMemcpyAsync(&flag, bad, sizeof(flag), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (flag)
    return fail(VRPH_EINVAL,
                "vrph_backward_noalloc: an edge entry is neither -1 nor a point in [0, n_total)");
  return VRPH_OK;
}

// ---------------------------------------------------------------------------
// extended persistence of graphs
// ---------------------------------------------------------------------------

// The offsets of a batch of graphs (host arrays of count + 1 entries):
// empty string if valid, else the error; *max_n = the largest graph.
static std::string graph_offsets_error(int32_t count, const int64_t* v_off, const int64_t* e_off,
                                       int* max_n) {
  if (count < 1 || !v_off || !e_off) return "bad argument";
  if (v_off[0] != 0 || e_off[0] != 0) return "offsets must start at 0";
  *max_n = 1;
  for (int g = 0; g < count; ++g) {
    const int64_t n = v_off[g + 1] - v_off[g], m = e_off[g + 1] - e_off[g];
    if (n < 1 || n > kGraphMaxN) return "every graph needs 1 to 4096 vertices";
    if (m < 0) return "edge offsets decrease";
    *max_n = std::max<int>(*max_n, (int)n);
  }
  const int64_t V = v_off[count], E = e_off[count];
  if (V + E >= ((int64_t)1 << 31) || E >= ((int64_t)1 << 31) - 1)
    return "totals must stay below 2^31";
  return "";
}

extern "C" vrph_status vrph_graph_extended(vrph_ctx* c, int32_t count, const int64_t* v_off,
                                           const int64_t* e_off, const float* f,
                                           const int32_t* edges, vrph_ext_bar* bars,
                                           void* hip_stream) {
  if (!c) return fail(VRPH_EINVAL, "vrph_graph_extended: bad argument");
  int max_n = 1;
  const std::string bad = graph_offsets_error(count, v_off, e_off, &max_n);
  if (!bad.empty()) return fail(VRPH_EINVAL, "vrph_graph_extended: " + bad);
  const int64_t V = v_off[count], E = e_off[count];
  if (!f || !bars || (E > 0 && !edges))
    return fail(VRPH_EINVAL, "vrph_graph_extended: NULL array");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
  NOT_CAPTURING(s, "vrph_graph_extended");
  const size_t ne = (size_t)std::max<int64_t>(E, 1);
  HIP_TRY(c->g_off.ensure((size_t)(count + 1) * 2 * sizeof(int64_t)));
  HIP_TRY(c->g_lower.ensure(ne * sizeof(Column)));
  HIP_TRY(c->g_upper.ensure(ne * sizeof(Column)));
  HIP_TRY(c->g_tmp.ensure(ne * sizeof(Column)));
  HIP_TRY(c->sort_work.ensure(radix_sort_work_bytes((int64_t)ne)));
  HIP_TRY(c->g_pos.ensure(ne * 4));
  HIP_TRY(c->g_adj_off.ensure((size_t)(V + count + 1) * 4));
  HIP_TRY(c->g_adj.ensure((size_t)std::max<int64_t>(2 * V, 1) * 4));
  HIP_TRY(c->g_stack.ensure((size_t)std::max<int64_t>(V, 1) * 4));
  HIP_TRY(c->g_err.ensure(sizeof(uint32_t)));
  int64_t* doff = c->g_off.as<int64_t>();
  HIP_TRY(hipMemcpyAsync(doff, v_off, (size_t)(count + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(doff + count + 1, e_off, (size_t)(count + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(launch_graph_ext(doff, doff + count + 1, count, V, E, max_n, f, edges,
                           c->g_lower.as<Column>(), c->g_upper.as<Column>(),
                           c->g_tmp.as<Column>(), c->sort_work.p, c->g_pos.as<uint32_t>(),
                           c->g_adj_off.as<uint32_t>(), c->g_adj.as<uint32_t>(),
                           c->g_stack.as<uint32_t>(), c->g_err.as<uint32_t>(), bars, s));
  uint32_t err = 0;
  HIP_TRY(hipMemcpyAsync(&err, c->g_err.p, sizeof(err), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (err & 7u)
    return fail(VRPH_EINVAL, std::string("vrph_graph_extended:") +
                                 ((err & 1u) ? " an edge endpoint outside its graph" : "") +
                                 ((err & 2u) ? " a loop" : "") +
                                 ((err & 4u) ? " a value that is not finite" : ""));
  if (err) return fail(VRPH_EDEVICE, "vrph_graph_extended: an internal consistency check failed");
  return VRPH_OK;
}

extern "C" vrph_status vrph_graph_extended_backward(vrph_ctx* c, int32_t count,
                                                    const int64_t* v_off, const int64_t* e_off,
                                                    const vrph_ext_bar* bars,
                                                    const float* g_birth, const float* g_death,
                                                    float* g_f, void* hip_stream) {
  if (!c) return fail(VRPH_EINVAL, "vrph_graph_extended_backward: bad argument");
  int max_n = 1;
  const std::string bad = graph_offsets_error(count, v_off, e_off, &max_n);
  if (!bad.empty()) return fail(VRPH_EINVAL, "vrph_graph_extended_backward: " + bad);
  if (!bars || !g_f) return fail(VRPH_EINVAL, "vrph_graph_extended_backward: NULL array");
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
  NOT_CAPTURING(s, "vrph_graph_extended_backward");
  HIP_TRY(c->g_off.ensure((size_t)(count + 1) * 2 * sizeof(int64_t)));
  HIP_TRY(c->g_err.ensure(sizeof(uint32_t)));
  int64_t* doff = c->g_off.as<int64_t>();
  HIP_TRY(hipMemcpyAsync(doff, v_off, (size_t)(count + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(doff + count + 1, e_off, (size_t)(count + 1) * sizeof(int64_t),
                         hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemsetAsync(c->g_err.p, 0, sizeof(uint32_t), s));
  HIP_TRY(launch_graph_ext_grad(doff, doff + count + 1, count, v_off[count] + e_off[count], bars,
                                g_birth, g_death, g_f, c->g_err.as<uint32_t>(), s));
  uint32_t err = 0;
  HIP_TRY(hipMemcpyAsync(&err, c->g_err.p, sizeof(err), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  if (err)
    return fail(VRPH_EINVAL, "vrph_graph_extended_backward: a bar's vertex is not in its graph");
  return VRPH_OK;
}

// ---------------------------------------------------------------------------
// explicit boundary matrices
// ---------------------------------------------------------------------------

extern "C" vrph_status vrph_boundary_pivots(vrph_ctx* c, int64_t ncols, const int64_t* col_ptr,
                                            const int64_t* rows, uint32_t flags, void* hip_stream,
                                            int64_t* low_out, vrph_boundary_stats* stats) {
  if (!c || ncols < 0) return fail(VRPH_EINVAL, "vrph_boundary_pivots: bad argument");
  if (ncols > 0 && (!col_ptr || !low_out))
    return fail(VRPH_EINVAL, "vrph_boundary_pivots: NULL argument");
  if (flags & ~(VRPH_BOUNDARY_NO_CLEARING | VRPH_BOUNDARY_NO_COMPRESSION))
    return fail(VRPH_EINVAL, "vrph_boundary_pivots: unknown flag bits");
  if (ncols >= ((int64_t)1 << 31) - 1)
    return fail(VRPH_EINVAL, "vrph_boundary_pivots: ncols must be below 2^31 - 1");
  vrph_boundary_stats st{};
  st.columns = ncols;
  if (ncols == 0) {
    if (stats) *stats = st;
    return VRPH_OK;
  }
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
  NOT_CAPTURING(s, "vrph_boundary_pivots");
  const size_t n = (size_t)ncols;
  std::vector<int64_t> hptr(n + 1);
  HIP_TRY(hipMemcpyAsync(hptr.data(), col_ptr, 8 * (n + 1), hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const int64_t nnz = hptr[n];
  if (hptr[0] != 0 || nnz < 0)
    return fail(VRPH_EINVAL, "vrph_boundary_pivots: col_ptr must start at 0 and end at nnz >= 0");
  if (nnz > 0 && !rows) return fail(VRPH_EINVAL, "vrph_boundary_pivots: NULL rows");

  // scratch: count (u64), err (u32), left (u32 x n), lookup (i32 x n),
  // unstable (i64 x n), stable (u8 x n), destroyer (u8 x n)
  auto up = [](size_t x) { return (x + 255) & ~(size_t)255; };
  const size_t o_left = 256, o_lookup = o_left + up(4 * n), o_unst = o_lookup + up(4 * n),
               o_stable = o_unst + up(8 * n), o_destr = o_stable + up(n),
               total = o_destr + up(n);
  HIP_TRY(c->bscan.ensure(total));
  char* base = c->bscan.as<char>();
  auto* count = reinterpret_cast<unsigned long long*>(base);
  auto* err = reinterpret_cast<uint32_t*>(base + 8);
  auto* left = reinterpret_cast<uint32_t*>(base + o_left);
  auto* lookup = reinterpret_cast<int32_t*>(base + o_lookup);
  auto* unstable = reinterpret_cast<int64_t*>(base + o_unst);
  auto* stable = reinterpret_cast<uint8_t*>(base + o_stable);
  auto* destroyer = reinterpret_cast<uint8_t*>(base + o_destr);
  const bool clearing = !(flags & VRPH_BOUNDARY_NO_CLEARING);
  // compression relies on the boundary property, as clearing does
  const bool compression = clearing && !(flags & VRPH_BOUNDARY_NO_COMPRESSION);
  HIP_TRY(hipMemsetAsync(base, 0, 16, s));
  HIP_TRY(hipEventRecord(c->ev0, s));
  HIP_TRY(launch_boundary_scan(ncols, col_ptr, rows, nnz, left, lookup, stable, destroyer,
                               unstable, count, err, clearing, s));
  HIP_TRY(hipEventRecord(c->ev1, s));
  uint64_t head[2] = {0, 0};
  HIP_TRY(hipMemcpyAsync(head, base, 16, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  float scan_ms = 0;
  HIP_TRY(hipEventElapsedTime(&scan_ms, c->ev0, c->ev1));
  const uint32_t e = (uint32_t)head[1];
  if (e & 1u) return fail(VRPH_EINVAL, "vrph_boundary_pivots: col_ptr decreasing or past nnz");
  if (e & 2u)
    return fail(VRPH_EINVAL, "vrph_boundary_pivots: rows not strictly increasing in a column");
  if (e & 4u) return fail(VRPH_EINVAL, "vrph_boundary_pivots: a row of column j outside [0, j)");
  const size_t nun = (size_t)head[0];
  if (nun > n) return fail(VRPH_EDEVICE, "vrph_boundary_pivots: unstable count out of range");
  std::vector<int32_t> hlookup(n);
  std::vector<int64_t> hun(nun), hrows((size_t)nnz);
  std::vector<uint8_t> hdestr(compression ? n : 0);
  HIP_TRY(hipMemcpyAsync(hlookup.data(), lookup, 4 * n, hipMemcpyDeviceToHost, s));
  if (compression) HIP_TRY(hipMemcpyAsync(hdestr.data(), destroyer, n, hipMemcpyDeviceToHost, s));
  if (nun) HIP_TRY(hipMemcpyAsync(hun.data(), unstable, 8 * nun, hipMemcpyDeviceToHost, s));
  if (nnz) HIP_TRY(hipMemcpyAsync(hrows.data(), rows, 8 * (size_t)nnz, hipMemcpyDeviceToHost, s));
  HIP_TRY(hipStreamSynchronize(s));
  const double t_host = now_ms();

  // Alg. 2 on the unstable columns (host threads, same result as in order)
  for (size_t r = 0; r < n; ++r) st.scan_pivots += hlookup[r] >= 0;
  std::sort(hun.begin(), hun.end());
  const int64_t* rptr = hptr.data();
  const int64_t* rrows = hrows.data();
  std::vector<int64_t> cptr, crows;
  if (compression) {  // Sec. 4.3.3, Alg. 8-9
    if (!compress_explicit(ncols, hptr.data(), hrows.data(), hlookup.data(), hdestr.data(),
                           hun.data(), (int64_t)nun, host_threads(), cptr, crows,
                           &st.compress_additions, &st.compressed))
      return fail(VRPH_EINVAL, "vrph_boundary_pivots: not a boundary matrix");
    rptr = cptr.data();
    rrows = crows.data();
  }
  if (!reduce_explicit_columns(ncols, rptr, rrows, hlookup.data(), hun.data(), (int64_t)nun,
                               host_threads(), low_out, &st.additions))
    return fail(VRPH_EINVAL, "vrph_boundary_pivots: not a boundary matrix");
  for (size_t j = 0; j < n; ++j) st.zero += hptr[j + 1] == hptr[j];
  st.unstable = (int64_t)nun;
  st.stable = ncols - (int64_t)nun;
  st.scan_ms = scan_ms;
  st.host_ms = now_ms() - t_host;
  if (stats) *stats = st;
  return VRPH_OK;
}

// ---------------------------------------------------------------------------
// batched point clouds
// ---------------------------------------------------------------------------

// starting host-to-device time ratio of a batch's split (one host thread's
// time per unit of estimated cost over the device's, measured on the 64-torus
// batch)
constexpr double kSplitRatio0 = 0.35;

struct vrph_batch {
  vrph_ctx* ctx = nullptr;
  int count = 0, m = 0, max_dim = 0, max_n = 0;
  float threshold = INFINITY;
  uint32_t flags = 0;
  std::vector<Cloud> clouds;
  std::vector<int64_t> sizes;
  int64_t total_points = 0, total_w = 0, total_edges = 0, total_words = 0;
  int max_kmax = 0;
  DevBuf X, D, W, dclouds, cstate, h0, bitmaps, cols, cols_tmp, sort_work, ap, counters;
  HostPinned h_cstate, h_counters, h_W;  // h_W: every cloud's weights, read by the host reduction
  // the forward's device work as two graphs: everything up to the sorted
  // non-apparent columns (front), then the device reduction (back)
  hipGraph_t graph = nullptr, graph_b = nullptr;
  hipGraphExec_t exec = nullptr, exec_b = nullptr;
  hipEvent_t ev[4] = {};
  std::vector<std::vector<uint64_t>> binoms;  // per cloud, k-major (kmax+1) x (n+1)
  std::vector<vrph_barcode> results;
  std::vector<H0Pair> hh0;
  std::vector<Column> hcols;
  std::vector<ApparentPair> hap;
  bool sorted_in_tmp = false;
  int64_t last_columns = 0, last_apparent = 0, last_nonapparent = 0;
  // dimension-1 reduction on the device (unless VRPH_HOST_REDUCTION)
  bool device_reduce = false;
  // Split (unless VRPH_DEVICE_REDUCTION): the clouds the cost model deems
  // heaviest are reduced on host threads while the device reduces the rest.
  // split_ratio: host-thread time per unit of estimated cost over the device
  // time per unit, updated from the times each split forward measures.
  bool split = false;
  double split_ratio = kSplitRatio0;
  // per cloud, the previous forward's dimension-1 columns and additions
  std::vector<int64_t> last_cols, last_add;
  DevBuf dskip;
  HostPinned h_skip;
  std::vector<char> w_on_host;
  // launch settings: the device reduction's workgroup size and the
  // dimension-1 edge kernel's workgroups per compute unit; tuned on the
  // first forward under VRPH_AUTOTUNE (or read from the tuning file)
  int dred_threads = 1024;
  int edge_mult = 8;
  bool tune = false;
  std::vector<DredCloud> hdc;
  DevBuf ddc, ew, eat, egrp, egend, ecnt, epos, tri, tlog, tab_keys, tab_vals, varena, vbits, vtouch,
      col_begin, col_end, out_death, out_ddiam, out_dedge, col_voff, col_vlen, dstats;
  std::vector<unsigned long long> hdeath;
  std::vector<uint32_t> hddiam, hdedge;
  std::vector<DredStats> hdstats;
};

// Buffers of the device reduction, each cloud's region sized from its n:
// the triangle bitmap ceil(C(n, 3) / 32) words; its log of toggled words up
// to half of that (more: the bitmap is cleared whole); the pivot table a
// power of two >= max(1024, E / 4) slots, E = C(n, 2) (a cloud with more
// than half that many non-apparent columns goes to the host); the V arena
// max(65536, E / 2) edges (more: the host); 16384 logged V words (more: V
// is read whole). Bitmaps and counts start at zero and the kernel leaves
// them at zero; epos starts at ~0 (the diagonal stays so).
using Want = std::vector<std::pair<DevBuf*, size_t>>;

static void dred_sizes(vrph_batch* b, Want& want) {
  b->hdc.resize((size_t)b->count);
  int64_t tri = 0, tlog = 0, tab = 0, va = 0, vt = 0;
  for (int i = 0; i < b->count; ++i) {
    const int64_t n = b->clouds[i].n, E = n * (n - 1) / 2;
    DredCloud& d = b->hdc[(size_t)i];
    d.tri_off = tri;
    d.tri_words = std::max<int64_t>((n * (n - 1) * (n - 2) / 6 + 31) / 32, 1);
    d.log_off = tlog;
    d.log_cap = (int32_t)std::max<int64_t>(1024, std::min<int64_t>(d.tri_words / 2, 1 << 20));
    int64_t tc = 1024;
    while (tc < E / 4) tc <<= 1;
    d.tab_off = tab;
    d.tab_cap = (int32_t)tc;
    d.v_off = va;
    d.v_cap = (int32_t)std::max<int64_t>(65536, E / 2);
    d.vt_off = vt;
    d.vt_cap = 16384;
    // test hook: "log,vtouch,arena" capacities (0 keeps the default), to
    // run the overflow paths on small inputs
    if (const char* e = std::getenv("VRPH_DRED_TEST_CAPS")) {
      long lc = 0, vc = 0, ac = 0;
      if (std::sscanf(e, "%ld,%ld,%ld", &lc, &vc, &ac) == 3) {
        if (lc > 0) d.log_cap = (int32_t)std::min<long>(lc, d.log_cap);
        if (vc > 0) d.vt_cap = (int32_t)std::min<long>(vc, d.vt_cap);
        if (ac > 0) d.v_cap = (int32_t)std::min<long>(ac, d.v_cap);
      }
    }
    tri += d.tri_words;
    tlog += d.log_cap;
    tab += d.tab_cap;
    va += d.v_cap;
    vt += d.vt_cap;
  }
  const size_t ne = (size_t)std::max<int64_t>(b->total_edges, 1);
  const size_t cnt = (size_t)b->count;
  const size_t words = (size_t)std::max<int64_t>(b->total_words, 1);
  want.insert(want.end(), {{&b->ddc, cnt * sizeof(DredCloud)}, {&b->ew, ne * 4},
                           {&b->eat, ne * 4}, {&b->egrp, ne * 4}, {&b->egend, ne * 4},
                           {&b->ecnt, ne * 4}, {&b->epos, (size_t)b->total_w * 4},
                           {&b->tri, (size_t)tri * 4}, {&b->tlog, (size_t)tlog * 4},
                           {&b->tab_keys, (size_t)tab * 8}, {&b->tab_vals, (size_t)tab * 4},
                           {&b->varena, (size_t)va * 4}, {&b->vbits, words * 4},
                           {&b->vtouch, (size_t)vt * 4}, {&b->col_begin, cnt * 4},
                           {&b->col_end, cnt * 4}, {&b->out_death, ne * 8},
                           {&b->out_ddiam, ne * 4}, {&b->out_dedge, ne * 4},
                           {&b->col_voff, ne * 4}, {&b->col_vlen, ne * 4},
                           {&b->dstats, cnt * sizeof(DredStats)}});
}

// The device reduction's tables, once allocated: the per-cloud regions, and
// the bitmaps and counts at zero, epos at ~0.
static vrph_status dred_init(vrph_batch* b) {
  const size_t ne = (size_t)std::max<int64_t>(b->total_edges, 1);
  const size_t words = (size_t)std::max<int64_t>(b->total_words, 1);
  HIP_TRY(hipMemcpy(b->ddc.p, b->hdc.data(), (size_t)b->count * sizeof(DredCloud),
                    hipMemcpyHostToDevice));
  HIP_TRY(hipMemset(b->tri.p, 0, b->tri.cap));
  HIP_TRY(hipMemset(b->ecnt.p, 0, ne * 4));
  HIP_TRY(hipMemset(b->vbits.p, 0, words * 4));
  HIP_TRY(hipMemset(b->epos.p, 0xFF, (size_t)b->total_w * 4));
  HIP_TRY(hipDeviceSynchronize());
  return VRPH_OK;
}

extern "C" vrph_status vrph_batch_plan(vrph_ctx* c, const int64_t* sizes, int32_t count,
                                       int32_t m, int32_t max_dim, float threshold,
                                       uint32_t flags, vrph_batch** out) {
  if (!c || !sizes || !out || count < 1 || m < 1)
    return fail(VRPH_EINVAL, "vrph_batch_plan: bad argument");
  *out = nullptr;
  if (max_dim < 0 || max_dim > 1) return fail(VRPH_EINVAL, "vrph_batch_plan: max_dim must be 0 or 1");
  if (flags & ~(VRPH_KEEP_ZERO_PERSISTENCE | VRPH_NO_ENCLOSING_RADIUS | VRPH_HOST_REDUCTION |
                VRPH_AUTOTUNE | VRPH_DEVICE_REDUCTION))
    return fail(VRPH_EINVAL, "vrph_batch_plan: unsupported flag bits");
  if ((flags & VRPH_HOST_REDUCTION) && (flags & VRPH_DEVICE_REDUCTION))
    return fail(VRPH_EINVAL, "vrph_batch_plan: VRPH_HOST_REDUCTION and VRPH_DEVICE_REDUCTION exclude each other");
  if (std::isnan(threshold) || threshold < 0) return fail(VRPH_EINVAL, "threshold must be >= 0");
  HIP_TRY(hipSetDevice(c->device));
  std::unique_ptr<vrph_batch> b(new (std::nothrow) vrph_batch());
  if (!b) return fail(VRPH_ENOMEM, "out of host memory");
  b->ctx = c;
  b->count = count;
  b->m = m;
  b->max_dim = max_dim;
  b->threshold = threshold;
  b->flags = flags;
  b->sizes.assign(sizes, sizes + count);
  b->clouds.resize(count);
  b->binoms.resize(count);
  for (int i = 0; i < count; ++i) {
    const int64_t n = sizes[i];
    if (n < 2 || n > kBatchMaxN) return fail(VRPH_EINVAL, "vrph_batch_plan: cloud size out of [2, 4096]");
    Cloud& cl = b->clouds[i];
    cl.x_off = b->total_points;
    cl.w_off = b->total_w;
    cl.e_off = b->total_edges;
    cl.bm_off = b->total_words;
    cl.n = (int)n;
    cl.tau_bits = std::isinf(threshold) ? 0x7F800000u : fbits(threshold);
    const int64_t ne = n * (n - 1) / 2;
    b->total_points += n;
    b->total_w += n * n;
    b->total_edges += ne;
    b->total_words += (ne + 31) / 32;
    b->max_n = std::max<int>(b->max_n, (int)n);
    if (!binomial_table((int)n, 3, b->binoms[i]))
      return fail(VRPH_EOVERFLOW, "simplex indices do not fit");
  }
  const uint64_t cap = (uint64_t)std::max<int64_t>(b->total_edges, 1);
  const bool keep_zero = flags & VRPH_KEEP_ZERO_PERSISTENCE;
  b->device_reduce = max_dim >= 1 && !(flags & VRPH_HOST_REDUCTION);
  b->split = b->device_reduce && !(flags & VRPH_DEVICE_REDUCTION);
  // every device buffer the plan needs, sized first: a plan larger than the
  // free device memory (or than VRPH_WORKSPACE_CAP bytes, if set) is refused
  // before anything is allocated
  Want want = {{&b->X, (size_t)b->total_points * m * 4},
               {&b->D, (size_t)b->total_w * 4},
               {&b->W, (size_t)b->total_w * 4},
               {&b->dclouds, (size_t)count * sizeof(Cloud)},
               {&b->cstate, (size_t)count * sizeof(CloudState)},
               {&b->h0, (size_t)count * b->max_n * sizeof(H0Pair)},
               {&b->bitmaps, (size_t)std::max<int64_t>(b->total_words, 1) * 4},
               {&b->cols, cap * sizeof(Column)},
               {&b->cols_tmp, cap * sizeof(Column)},
               {&b->sort_work, radix_sort_work_bytes((int64_t)cap)},
               {&b->counters, sizeof(Scalars)}};
  if (keep_zero) want.push_back({&b->ap, cap * sizeof(ApparentPair)});
  if (b->device_reduce) {
    dred_sizes(b.get(), want);
    want.push_back({&b->dskip, (size_t)count * 4});
  }
  size_t need = 0;
  for (const auto& w : want) need += w.second;
  size_t free_b = 0, total_b = 0;
  HIP_TRY(hipMemGetInfo(&free_b, &total_b));
  size_t limit = free_b;
  if (const char* e = std::getenv("VRPH_WORKSPACE_CAP")) {
    const unsigned long long lim = std::strtoull(e, nullptr, 10);
    if (lim > 0) limit = std::min<size_t>(limit, (size_t)lim);
  }
  if (need > limit)
    return fail(VRPH_ENOMEM, "vrph_batch_plan: the plan needs " + std::to_string(need) +
                                 " bytes of device memory, " + std::to_string(limit) +
                                 " are available");
  for (const auto& w : want) HIP_TRY(w.first->ensure(w.second));
  HIP_TRY(b->h_cstate.ensure((size_t)count * sizeof(CloudState)));
  HIP_TRY(b->h_counters.ensure(sizeof(Scalars)));
  if (b->device_reduce) {
    HIP_TRY(b->h_skip.ensure((size_t)count * 4));
    std::memset(b->h_skip.p, 0, (size_t)count * 4);
    HIP_TRY(hipMemcpy(b->dskip.p, b->h_skip.p, (size_t)count * 4, hipMemcpyHostToDevice));
  }
  b->w_on_host.assign((size_t)count, 0);
  b->last_cols.assign((size_t)count, 0);
  b->last_add.assign((size_t)count, 0);
  // the weights on the host: for the host reduction and for the edges of
  // apparent pairs (otherwise allocated only if a cloud falls back to the host)
  if (!b->device_reduce || keep_zero) HIP_TRY(b->h_W.ensure((size_t)b->total_w * 4));
  HIP_TRY(hipMemcpy(b->dclouds.p, b->clouds.data(), (size_t)count * sizeof(Cloud),
                    hipMemcpyHostToDevice));
  if (b->device_reduce) {
    vrph_status st = dred_init(b.get());
    if (st != VRPH_OK) return st;
  }
  // launch settings: a tuning already found for this size bucket, else
  // tuned on the first forward if asked
  {
    const auto it = c->tuned.find({1, size_bucket(b->max_n), 3});
    if (it != c->tuned.end() && (it->second.chunk == 256 || it->second.chunk == 512 ||
                                 it->second.chunk == 1024)) {
      b->dred_threads = it->second.chunk;
      b->edge_mult = it->second.mult;
    } else {
      b->tune = (flags & VRPH_AUTOTUNE) != 0 && max_dim >= 1;
    }
  }
  b->results.resize(count);
  for (hipEvent_t& ev : b->ev) {
    const hipError_t e = hipEventCreate(&ev);
    if (e != hipSuccess) {
      for (hipEvent_t& x : b->ev)
        if (x) (void)hipEventDestroy(x);
      return fail(VRPH_EDEVICE, std::string("hipEventCreate: ") + hipGetErrorString(e));
    }
  }
  *out = b.release();
  return VRPH_OK;
}

extern "C" void vrph_batch_destroy(vrph_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->ctx->device);
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->exec_b) (void)hipGraphExecDestroy(b->exec_b);
  if (b->graph_b) (void)hipGraphDestroy(b->graph_b);
  for (hipEvent_t e : b->ev)
    if (e) (void)hipEventDestroy(e);
  DevBuf* bufs[] = {&b->X,    &b->D,        &b->W,         &b->dclouds, &b->cstate,
                    &b->h0,   &b->bitmaps,  &b->cols,      &b->cols_tmp, &b->sort_work,
                    &b->ap,   &b->counters, &b->ddc, &b->ew, &b->eat, &b->egrp, &b->egend,
                    &b->ecnt, &b->epos,  &b->tri,    &b->tlog,    &b->tab_keys, &b->tab_vals, &b->varena,
                    &b->vbits, &b->vtouch, &b->col_begin, &b->col_end, &b->out_death,
                    &b->out_ddiam, &b->out_dedge, &b->col_voff, &b->col_vlen, &b->dstats, &b->dskip};
  for (DevBuf* d : bufs) d->release();
  b->h_cstate.release();
  b->h_counters.release();
  b->h_W.release();
  b->h_skip.release();
  delete b;
}

// Device work of one forward up to the sorted columns, recorded once into a
// graph and replayed: reset of the per-cloud state with fill kernels (no
// memset nodes), distances, validation + weights, H0, the dimension-1
// enumeration + apparent test over the edges of every cloud, the
// coboundary-order sort with the record count read on the device, and the
// copies of the small results to pinned memory.
static hipError_t batch_record_front(vrph_batch* b, hipStream_t s) {
  const bool keep_zero = b->flags & VRPH_KEEP_ZERO_PERSISTENCE;
  const bool enclosing = !(b->flags & VRPH_NO_ENCLOSING_RADIUS);
  Scalars* sc = b->counters.as<Scalars>();
  hipError_t e;
  if ((e = launch_init_states(b->cstate.as<CloudState>(), b->count, s))) return e;
  if ((e = launch_fill_u32(b->bitmaps.as<uint32_t>(), b->total_words, 0u, s))) return e;
  if ((e = launch_fill_u32(b->counters.as<uint32_t>(), sizeof(Scalars) / 4, 0u, s))) return e;
  if ((e = launch_batch_pdist(b->X.as<float>(), b->m, b->dclouds.as<Cloud>(), b->count,
                              b->total_points, b->D.as<float>(), s)))
    return e;
  // (the clouds' D comes from pdist: symmetric by construction)
  if ((e = launch_batch_validate_weights(b->D.as<float>(), b->dclouds.as<Cloud>(), b->count,
                                         b->total_points, enclosing, b->W.as<uint32_t>(),
                                         b->cstate.as<CloudState>(), s, false, false)))
    return e;
  if ((e = launch_batch_h0(b->W.as<uint32_t>(), b->dclouds.as<Cloud>(), b->count,
                           b->cstate.as<CloudState>(), b->h0.as<H0Pair>(), b->max_n,
                           b->bitmaps.as<uint32_t>(), s)))
    return e;
  if (b->max_dim >= 1) {
    const uint64_t cap = (uint64_t)std::max<int64_t>(b->total_edges, 1);
    int cloud_bits = 0;
    while ((1 << cloud_bits) < b->count) ++cloud_bits;
    // edge positions for the device reduction (cols / cols_tmp as scratch,
    // before the enumeration fills them)
    if (b->device_reduce &&
        (e = launch_dred_prepare(b->W.as<uint32_t>(), b->dclouds.as<Cloud>(), b->count,
                                 b->total_edges, cloud_bits, b->cols.as<Column>(),
                                 b->cols_tmp.as<Column>(), b->sort_work.p, b->ew.as<uint32_t>(),
                                 b->eat.as<uint32_t>(), b->egrp.as<uint32_t>(),
                                 b->egend.as<uint32_t>(), b->epos.as<uint32_t>(), s)))
      return e;
    if ((e = launch_batch_edges(b->W.as<uint32_t>(), b->dclouds.as<Cloud>(), b->count,
                                b->total_edges, b->bitmaps.as<uint32_t>(), b->cols.as<Column>(),
                                cap, keep_zero ? b->ap.as<ApparentPair>() : nullptr,
                                keep_zero ? cap : 0, ClearSet{nullptr, nullptr, 0, nullptr},
                                &sc->columns,
                                b->ctx->num_cus * b->edge_mult, s)))
      return e;
    int max_edges_bits = 0;
    while ((int64_t(1) << max_edges_bits) < (int64_t)b->max_n * (b->max_n - 1) / 2) ++max_edges_bits;
    bool in_tmp = false;
    if ((e = radix_sort_columns(b->cols.as<Column>(), b->cols_tmp.as<Column>(), (int64_t)cap,
                                max_edges_bits, cloud_bits, b->sort_work.p, s, &sc->nonapparent,
                                &in_tmp)))
      return e;
    b->sorted_in_tmp = in_tmp;
  }
  if ((e = hipMemcpyAsync(b->h_cstate.p, b->cstate.p, (size_t)b->count * sizeof(CloudState),
                          hipMemcpyDeviceToHost, s)))
    return e;
  return hipMemcpyAsync(b->h_counters.p, b->counters.p, sizeof(Scalars), hipMemcpyDeviceToHost, s);
}

// The device reduction of dimension 1, recorded into a graph of its own: it
// runs while host threads reduce the clouds flagged in dskip.
static hipError_t batch_record_back(vrph_batch* b, hipStream_t s) {
  if (!b->device_reduce || b->max_dim < 1) return hipSuccess;
  const uint64_t cap = (uint64_t)std::max<int64_t>(b->total_edges, 1);
  Scalars* sc = b->counters.as<Scalars>();
  const bool in_tmp = b->sorted_in_tmp;
  DredArgs a{};
  a.clouds = b->dclouds.as<Cloud>();
  a.dc = b->ddc.as<DredCloud>();
  a.count = b->count;
  a.cols = (in_tmp ? b->cols_tmp : b->cols).as<Column>();
  a.ncols = &sc->nonapparent;
  a.col_begin_w = b->col_begin.as<uint32_t>();
  a.col_end_w = b->col_end.as<uint32_t>();
  a.col_begin = a.col_begin_w;
  a.col_end = a.col_end_w;
  a.epos = b->epos.as<uint32_t>();
  a.eat = b->eat.as<uint32_t>();
  a.egrp = b->egrp.as<uint32_t>();
  a.egend = b->egend.as<uint32_t>();
  a.ew = b->ew.as<uint32_t>();
  a.cnt = b->ecnt.as<uint32_t>();
  a.tri = b->tri.as<uint32_t>();
  a.tlog = b->tlog.as<uint32_t>();
  a.tab_keys = b->tab_keys.as<unsigned long long>();
  a.tab_vals = b->tab_vals.as<uint32_t>();
  a.varena = b->varena.as<uint32_t>();
  a.vbits = b->vbits.as<uint32_t>();
  a.vtouch = b->vtouch.as<uint32_t>();
  a.out_death = b->out_death.as<unsigned long long>();
  a.out_ddiam = b->out_ddiam.as<uint32_t>();
  a.out_dedge = b->out_dedge.as<uint32_t>();
  a.col_voff = b->col_voff.as<uint32_t>();
  a.col_vlen = b->col_vlen.as<uint32_t>();
  a.stats = b->dstats.as<DredStats>();
  a.skip = b->dskip.as<uint32_t>();
  return launch_dred_reduce(a, (int64_t)cap, b->max_n, b->dred_threads, s);
}

// Which clouds host threads reduce while the device reduces the others. The
// clouds come in decreasing estimated cost; the first k go to the host, k minimising the larger of the two sides'
// estimated times: on the host the longest-processing-time schedule of
// those clouds over `threads` threads, each taking `ratio` x its cost; on
// the device the costliest remaining cloud (one workgroup each, all at
// once), or their total over `units` workgroups at a time if that is larger.
// Clouds without columns stay on the device. Ties keep the smaller k.
static int choose_split(const std::vector<double>& cost, const std::vector<int>& order,
                        int threads, double ratio, int units, double* host_est, double* dev_est) {
  const int count = (int)order.size();
  double rest = 0;
  for (int i : order) rest += cost[(size_t)i];
  std::priority_queue<double, std::vector<double>, std::greater<double>> loads;
  for (int t = 0; t < std::max(1, threads); ++t) loads.push(0.0);
  double host = 0, best = -1;
  int best_k = 0;
  for (int k = 0; k <= count; ++k) {
    const double top = k < count ? cost[(size_t)order[(size_t)k]] : 0.0;
    const double dev = std::max(top, rest / std::max(1, units));
    const double t = std::max(host, dev);
    if (best < 0 || t < best) {
      best = t;
      best_k = k;
      *host_est = host;
      *dev_est = dev;
    }
    if (k == count || top == 0) break;
    const double l = loads.top() + ratio * top;
    loads.pop();
    loads.push(l);
    host = std::max(host, l);
    rest -= top;
  }
  return best_k;
}

extern "C" vrph_status vrph_batch_forward(vrph_batch* b, const float* X_packed, void* hip_stream) {
  if (!b || !X_packed) return fail(VRPH_EINVAL, "vrph_batch_forward: NULL argument");
  vrph_ctx* c = b->ctx;
  HIP_TRY(hipSetDevice(c->device));
  hipStream_t s = hip_stream ? (hipStream_t)hip_stream : c->stream;
  NOT_CAPTURING(s, "vrph_batch_forward");
  const double t_start = now_ms();
  const bool dev = b->device_reduce && b->max_dim >= 1;
  HIP_TRY(hipMemcpyAsync(b->X.p, X_packed, (size_t)b->total_points * b->m * 4,
                         hipMemcpyDeviceToDevice, s));
  if (!b->exec && b->tune) {
    // the batch autotuner: the whole device part run eagerly (the same work
    // the graphs record, every cloud reduced on the device) per candidate,
    // timed with HIP events; first the device reduction's workgroup size,
    // then the edge kernel's grid
    if (dev) {
      std::memset(b->h_skip.p, 0, (size_t)b->count * 4);
      HIP_TRY(hipMemcpyAsync(b->dskip.p, b->h_skip.p, (size_t)b->count * 4,
                             hipMemcpyHostToDevice, s));
    }
    auto time_once = [&](int threads, int mult, float* ms) -> hipError_t {
      b->dred_threads = threads;
      b->edge_mult = mult;
      hipError_t e = hipEventRecord(c->ev0, s);
      if (e == hipSuccess) e = batch_record_front(b, s);
      if (e == hipSuccess) e = batch_record_back(b, s);
      if (e == hipSuccess) e = hipEventRecord(c->ev1, s);
      if (e == hipSuccess) e = hipEventSynchronize(c->ev1);
      if (e == hipSuccess) e = hipEventElapsedTime(ms, c->ev0, c->ev1);
      return e;
    };
    int best_t = 1024, best_m = 8;
    float best = 0, ms = 0;
    HIP_TRY(time_once(best_t, best_m, &ms));  // warm-up (code objects, caches)
    HIP_TRY(time_once(best_t, best_m, &best));
    if (b->device_reduce)
      for (int t : {256, 512}) {
        HIP_TRY(time_once(t, best_m, &ms));
        if (ms < best) {
          best = ms;
          best_t = t;
        }
      }
    for (int mlt : {2, 4, 16, 32}) {
      HIP_TRY(time_once(best_t, mlt, &ms));
      if (ms < best) {
        best = ms;
        best_m = mlt;
      }
    }
    b->dred_threads = best_t;
    b->edge_mult = best_m;
    b->tune = false;
    const std::tuple<int, int, int> key{1, size_bucket(b->max_n), 3};
    c->tuned[key] = Tune{best_t, best_m};
    save_tuning(c, key, Tune{best_t, best_m});
  }
  auto capture = [&](hipError_t (*rec)(vrph_batch*, hipStream_t), hipGraph_t* graph,
                     hipGraphExec_t* exec) -> vrph_status {
    HIP_TRY(hipStreamBeginCapture(s, hipStreamCaptureModeThreadLocal));
    hipError_t e = rec(b, s);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(s, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return fail(VRPH_EDEVICE, std::string("graph capture failed: ") +
                                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    *graph = g;
    HIP_TRY(hipGraphInstantiate(exec, g, nullptr, nullptr, 0));
    return VRPH_OK;
  };
  if (!b->exec) {
    vrph_status st = capture(batch_record_front, &b->graph, &b->exec);
    if (st != VRPH_OK) return st;
  }
  if (dev && !b->exec_b) {
    vrph_status st = capture(batch_record_back, &b->graph_b, &b->exec_b);
    if (st != VRPH_OK) return st;
  }
  hipEvent_t* ev = b->ev;
  HIP_TRY(hipEventRecord(ev[0], s));
  HIP_TRY(hipGraphLaunch(b->exec, s));
  HIP_TRY(hipEventRecord(ev[1], s));
  HIP_TRY(hipStreamSynchronize(s));
  float front_ms = 0, back_ms = 0;
  HIP_TRY(hipEventElapsedTime(&front_ms, ev[0], ev[1]));
  Scalars sc;
  std::memcpy(&sc, b->h_counters.p, sizeof(sc));
  const CloudState* cst = b->h_cstate.as<CloudState>();
  for (int i = 0; i < b->count; ++i)
    if (cst[i].err) return fail(VRPH_EINVAL, "invalid distances in cloud " + std::to_string(i));

  // results of the front part
  const bool keep_zero = b->flags & VRPH_KEEP_ZERO_PERSISTENCE;
  const int64_t nna = (int64_t)sc.nonapparent;
  b->hh0.resize((size_t)b->count * b->max_n);
  b->hcols.resize((size_t)nna);
  HIP_TRY(hipMemcpyAsync(b->hh0.data(), b->h0.p, b->hh0.size() * sizeof(H0Pair),
                         hipMemcpyDeviceToHost, s));
  if (nna)
    HIP_TRY(hipMemcpyAsync(b->hcols.data(), b->sorted_in_tmp ? b->cols_tmp.p : b->cols.p,
                           (size_t)nna * sizeof(Column), hipMemcpyDeviceToHost, s));
  if (keep_zero) {
    b->hap.resize(sc.apparent_written);
    if (sc.apparent_written)
      HIP_TRY(hipMemcpyAsync(b->hap.data(), b->ap.p, sc.apparent_written * sizeof(ApparentPair),
                             hipMemcpyDeviceToHost, s));
  }
  HIP_TRY(hipStreamSynchronize(s));

  // per-cloud slices of the sorted columns and of the apparent pairs
  std::vector<int64_t> col_begin(b->count + 1, nna);
  for (int64_t j = nna - 1; j >= 0; --j) col_begin[b->hcols[j].cloud] = j;
  for (int i = b->count - 1; i >= 0; --i)
    if (col_begin[i] > col_begin[i + 1]) col_begin[i] = col_begin[i + 1];
  std::vector<std::vector<uint32_t>> ap_of(keep_zero ? b->count : 0);
  if (keep_zero)
    for (size_t j = 0; j < b->hap.size(); ++j) ap_of[b->hap[j].cloud].push_back((uint32_t)j);

  // clouds in decreasing estimated reduction cost: the non-apparent columns
  // times one plus the additions per column the previous forward made on
  // that cloud (a batch is usually replayed on the same clouds as they
  // move), else times the points / 16; the host hands them out in this
  // order, so that a heavy cloud does not start last and stretch the tail
  std::vector<double> cost((size_t)b->count);
  for (int i = 0; i < b->count; ++i) {
    const double nc = (double)(col_begin[i + 1] - col_begin[i]);
    const int64_t lc = b->last_cols[(size_t)i];
    cost[(size_t)i] = lc > 0 ? nc * (1.0 + (double)b->last_add[(size_t)i] / (double)lc)
                             : nc * b->clouds[i].n / 16.0;
  }
  std::vector<int> order((size_t)b->count);
  for (int i = 0; i < b->count; ++i) order[(size_t)i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int x, int y) { return cost[(size_t)x] > cost[(size_t)y]; });
  const int nthreads = std::max(1, std::min<int>(b->count, std::min<int>(16, (int)std::thread::hardware_concurrency())));
  // the first n_host clouds of `order` are reduced on host threads
  int n_host = b->count;
  double host_est = 0, dev_est = 0;
  if (dev) {
    n_host = b->split ? choose_split(cost, order, nthreads, b->split_ratio, c->num_cus, &host_est,
                                     &dev_est)
                      : 0;
    uint32_t* skip = b->h_skip.as<uint32_t>();
    std::memset(skip, 0, (size_t)b->count * 4);
    for (int q = 0; q < n_host; ++q) skip[order[(size_t)q]] = 1;
    HIP_TRY(hipMemcpyAsync(b->dskip.p, skip, (size_t)b->count * 4, hipMemcpyHostToDevice, s));
  }
  // the weights on the host: all of them for the host reduction and for the
  // edges of apparent pairs, else those of the clouds the host reduces
  std::fill(b->w_on_host.begin(), b->w_on_host.end(), 0);
  auto copy_w = [&](int i) -> hipError_t {
    const Cloud& cl = b->clouds[(size_t)i];
    b->w_on_host[(size_t)i] = 1;
    return hipMemcpyAsync(b->h_W.as<uint32_t>() + cl.w_off, b->W.as<uint32_t>() + cl.w_off,
                          (size_t)cl.n * cl.n * 4, hipMemcpyDeviceToHost, s);
  };
  if (b->max_dim >= 1 && (!dev || keep_zero || n_host > 0)) {
    HIP_TRY(b->h_W.ensure((size_t)b->total_w * 4));
    if (!dev || keep_zero) {
      HIP_TRY(hipMemcpyAsync(b->h_W.p, b->W.p, (size_t)b->total_w * 4, hipMemcpyDeviceToHost, s));
      std::fill(b->w_on_host.begin(), b->w_on_host.end(), 1);
    } else {
      for (int q = 0; q < n_host; ++q) HIP_TRY(copy_w(order[(size_t)q]));
    }
  }
  // the device reduction of the other clouds runs while the host reduces
  HIP_TRY(hipEventRecord(ev[2], s));
  if (dev) {
    HIP_TRY(hipGraphLaunch(b->exec_b, s));
    HIP_TRY(hipEventRecord(ev[3], s));
  }
  HIP_TRY(hipEventSynchronize(ev[2]));

  auto host_reduced = [&](int i) { return !dev || b->h_skip.as<uint32_t>()[i] != 0 || b->hdstats[(size_t)i].err != 0; };
  // one cloud's pairs: H0 from the device, dimension 1 reduced here or by
  // the device, edges from the host weights where they are here
  auto assemble = [&](int i) {
    const Cloud& cl = b->clouds[i];
    HostComplex H;
    H.n = cl.n;
    H.W = b->w_on_host[(size_t)i] ? b->h_W.as<uint32_t>() + cl.w_off : nullptr;
    H.binom = b->binoms[i].data();
    H.kmax = 3;
    vrph_barcode& r = b->results[i];
    r.pairs.clear();
    std::memset(&r.stats, 0, sizeof(r.stats));
    r.stats.max_dim = b->max_dim;
    r.stats.tau_eff = bitsf(cst[i].tau_bits);
    const H0Pair* h0 = b->hh0.data() + (size_t)i * b->max_n;
    for (uint32_t k = 0; k < cst[i].h0_count && k < (uint32_t)cl.n; ++k)
      r.pairs.push_back(make_pair(0, h0[k].birth, 0u, h0[k].death, h0[k].diam));
    r.stats.pairs[0] = cst[i].h0_count;
    if (b->max_dim >= 1) {
      const int64_t cb = col_begin[i], ce = col_begin[i + 1];
      if (!host_reduced(i)) {
        // pairs of the device reduction, with their edges
        for (int64_t j = cb; j < ce; ++j) {
          vrph_pair p = make_pair(1, b->hcols[j].cidx, ~b->hcols[j].key_hi, b->hdeath[j],
                                  b->hddiam[j]);
          int v[2];
          decode_simplex(H, p.birth, 1, v);
          p.birth_edge[0] = v[1];
          p.birth_edge[1] = v[0];
          p.death_edge[0] = p.death_edge[1] = -1;
          if (!p.essential) {
            p.death_edge[0] = (int32_t)(b->hdedge[j] >> 16);
            p.death_edge[1] = (int32_t)(b->hdedge[j] & 0xFFFF);
          }
          r.pairs.push_back(p);
        }
        r.stats.additions[1] = (int64_t)b->hdstats[(size_t)i].additions;
        r.stats.emergent[1] = b->hdstats[(size_t)i].emergent;
        r.stats.device_reduced = 1;
      } else {
        std::vector<PairRec> prs;
        std::vector<uint64_t> deaths;
        ReduceStats rs;
        RankTable ranks;
        if (ce > cb) {
          ranks.build(cl.n, H.W);
          ranks.attach(H);
        }
        reduce_dimension(H, 1, b->hcols.data() + cb, ce - cb, 1, prs, deaths, rs);
        for (const PairRec& q : prs) r.pairs.push_back(make_pair(1, q.birth, q.bdiam, q.death, q.ddiam));
        r.stats.additions[1] = rs.additions;
        r.stats.emergent[1] = rs.emergent;
      }
      if (keep_zero)
        for (uint32_t j : ap_of[i]) {
          const ApparentPair& a = b->hap[j];
          r.pairs.push_back(make_pair(1, a.s, a.diam, a.t, a.diam));
        }
      r.stats.reduced[1] = ce - cb;
    }
    if (H.W) {
      finish_pairs(&r, H, b->max_dim, keep_zero, 1);
    } else {
      // edges without the weights: vertex births have none, an H0 death
      // is its own edge, the dimension-1 pairs carry theirs
      for (vrph_pair& p : r.pairs)
        if (p.dim == 0) {
          p.birth_edge[0] = p.birth_edge[1] = -1;
          p.death_edge[0] = p.death_edge[1] = -1;
          if (!p.essential) {
            int v[2];
            decode_simplex(H, p.death, 1, v);
            p.death_edge[0] = v[1];
            p.death_edge[1] = v[0];
          }
        }
      order_pairs(&r, keep_zero, 1);
    }
  };
  // clouds order[from, to) on the host threads
  auto run_pool = [&](int from, int to) {
    std::atomic<int> next{from};
    auto work = [&]() {
      for (int q; (q = next.fetch_add(1)) < to;) assemble(order[(size_t)q]);
    };
    const int nt = std::max(1, std::min(nthreads, to - from));
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(work);
    work();
    for (std::thread& t : pool) t.join();
  };

  const double th = now_ms();
  run_pool(0, n_host);
  const double host_split_ms = now_ms() - th;
  double tail_ms = 0;
  if (dev) {
    HIP_TRY(hipEventSynchronize(ev[3]));
    HIP_TRY(hipEventElapsedTime(&back_ms, ev[2], ev[3]));
    const double t2 = now_ms();
    b->hdeath.resize((size_t)nna);
    b->hddiam.resize((size_t)nna);
    b->hdedge.resize((size_t)nna);
    b->hdstats.resize((size_t)b->count);
    if (nna) {
      HIP_TRY(hipMemcpyAsync(b->hdeath.data(), b->out_death.p, (size_t)nna * 8,
                             hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(b->hddiam.data(), b->out_ddiam.p, (size_t)nna * 4,
                             hipMemcpyDeviceToHost, s));
      HIP_TRY(hipMemcpyAsync(b->hdedge.data(), b->out_dedge.p, (size_t)nna * 4,
                             hipMemcpyDeviceToHost, s));
    }
    HIP_TRY(hipMemcpyAsync(b->hdstats.data(), b->dstats.p, (size_t)b->count * sizeof(DredStats),
                           hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    // a cloud whose tables overflowed on the device is reduced here
    bool more_w = false;
    for (int q = n_host; q < b->count; ++q) {
      const int i = order[(size_t)q];
      if (b->hdstats[(size_t)i].err != 0 && !b->w_on_host[(size_t)i]) {
        HIP_TRY(b->h_W.ensure((size_t)b->total_w * 4));
        HIP_TRY(copy_w(i));
        more_w = true;
      }
    }
    if (more_w) HIP_TRY(hipStreamSynchronize(s));
    run_pool(n_host, b->count);
    tail_ms = now_ms() - t2;
    // the host-to-device time ratio, from what this forward measured; a
    // forward that left one side without clouds measures nothing, and the
    // ratio then moves back toward its starting value, so that one odd
    // measurement cannot keep every cloud on one side for good
    if (b->split) {
      if (n_host > 0 && n_host < b->count && host_est > 0 && dev_est > 0 && back_ms > 1.0 &&
          host_split_ms > 1.0) {
        const double dev_rate = back_ms / dev_est;
        const double host_rate = host_split_ms / (host_est / b->split_ratio);
        const double r = std::sqrt(b->split_ratio * (host_rate / dev_rate));
        b->split_ratio = std::min(50.0, std::max(0.02, r));
      } else if (n_host == 0 || n_host == b->count) {
        b->split_ratio = std::sqrt(b->split_ratio * kSplitRatio0);
      }
    }
  }
  const double host_ms = host_split_ms + tail_ms;
  for (int i = 0; i < b->count; ++i) {
    b->last_cols[(size_t)i] = b->results[i].stats.reduced[1];
    b->last_add[(size_t)i] = b->results[i].stats.additions[1];
    b->results[i].stats.gpu_ms[0] = front_ms + back_ms;
    b->results[i].stats.host_ms[1] = host_ms;
    b->results[i].stats.grid[1] = b->max_dim >= 1 ? c->num_cus * b->edge_mult : 0;
    b->results[i].stats.total_ms = now_ms() - t_start;
  }
  b->last_columns = (int64_t)sc.columns;
  b->last_apparent = (int64_t)sc.apparent;
  b->last_nonapparent = nna;
  return VRPH_OK;
}

extern "C" vrph_status vrph_batch_result(vrph_batch* b, int32_t cloud, const vrph_barcode** view) {
  if (!b || !view || cloud < 0 || cloud >= b->count)
    return fail(VRPH_EINVAL, "vrph_batch_result: bad argument");
  *view = &b->results[cloud];
  return VRPH_OK;
}
