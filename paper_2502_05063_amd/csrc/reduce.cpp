// Host submatrix reduction (Sec. 5.2.9, 5.5.1) over the columns the GPU
// found non-apparent. Columns of the dimension-d coboundary matrix are
// d-simplices in coboundary order (diameter descending, index ascending);
// rows are (d+1)-simplices in the same order. A row is named by its
// diameter rank and its index; the lowest nonzero of a column (its pivot) is
// its oldest cofacet: the smallest rank, then the largest index.
#include "reduce.h"

#include <algorithm>
#include <iterator>
#include <atomic>
#include <chrono>
#include <memory>
#include <thread>

namespace vrph {

using u128 = unsigned __int128;

void decode_simplex(const HostComplex& H, uint64_t c, int d, int* v) {
  int hi = H.n - 1;
  for (int i = d; i >= 1; --i) {
    int lo = i, h = hi;
    while (lo < h) {
      int mid = (lo + h + 1) >> 1;
      if (H.C(mid, i + 1) <= c)
        lo = mid;
      else
        h = mid - 1;
    }
    v[i] = lo;
    c -= H.C(lo, i + 1);
    hi = lo - 1;
  }
  v[0] = (int)c;
}

void diameter_edge(const HostComplex& H, uint64_t c, int d, int32_t* u, int32_t* w) {
  int v[kMaxDim + 3];
  decode_simplex(H, c, d, v);
  // weights, or their ranks when only those are here: the same order and
  // the same ties
  auto wt = [&](int a, int b) { return H.W ? H.w(a, b) : H.wr(a, b); };
  uint32_t dm = 0;
  for (int i = 1; i <= d; ++i)
    for (int j = 0; j < i; ++j) dm = std::max(dm, wt(v[i], v[j]));
  uint64_t best = 0;
  bool have = false;
  for (int i = 1; i <= d; ++i)
    for (int j = 0; j < i; ++j)
      if (wt(v[i], v[j]) == dm) {
        uint64_t e = H.C(v[i], 2) + (uint64_t)v[j];
        if (!have || e > best) {
          best = e;
          *u = v[i];
          *w = v[j];
          have = true;
        }
      }
}

// index of s + {x} (Eq. 5.6); vertices above x move up one position
static uint64_t cofacet_index(const HostComplex& H, const int* v, int d, int x) {
  uint64_t c = 0;
  int p = d + 1;
  bool placed = false;
  for (int i = d; i >= 0; --i) {
    if (!placed && x > v[i]) {
      c += H.C(x, p + 1);
      --p;
      placed = true;
    }
    c += H.C(v[i], p + 1);
    --p;
  }
  if (!placed) c += (uint64_t)x;
  return c;
}

static uint32_t rank_of(const HostComplex& H, const int* v, int d) {
  uint32_t m = 0;
  for (int i = 1; i <= d; ++i)
    for (int j = 0; j < i; ++j) m = std::max(m, H.wr(v[i], v[j]));
  return m;
}

// max over the vertices of s of the rank of edge (v_i, x); kInf if some edge
// is above tau_eff
static inline uint32_t reach_of(const HostComplex& H, const int* v, int d, int x) {
  uint32_t m = 0;
  for (int i = 0; i <= d; ++i) m = std::max(m, H.wr(v[i], x));
  return m;
}

static inline bool contains(const int* v, int d, int x) {
  for (int i = 0; i <= d; ++i)
    if (v[i] == x) return true;
  return false;
}

// mask = the vertices adjacent within tau_eff to every vertex of s, i.e. the
// x whose cofacet s + {x} is in the complex (the vertices of s are not in
// it: no vertex is its own neighbour)
static void common_neighbors(const HostComplex& H, const int* v, int d, uint64_t* mask) {
  const uint64_t* r0 = H.nb + (size_t)v[0] * (size_t)H.nbw;
  for (int w = 0; w < H.nbw; ++w) mask[w] = r0[w];
  for (int i = 1; i <= d; ++i) {
    const uint64_t* ri = H.nb + (size_t)v[i] * (size_t)H.nbw;
    for (int w = 0; w < H.nbw; ++w) mask[w] &= ri[w];
  }
}

// Calls f(x) for the set bits x of mask from the largest down; stops when f
// returns false.
template <class F>
static void for_each_desc(const uint64_t* mask, int words, F f) {
  for (int w = words - 1; w >= 0; --w)
    for (uint64_t m = mask[w]; m;) {
      const int b = 63 - __builtin_clzll(m);
      m &= ~(1ull << b);
      if (!f(w * 64 + b)) return;
    }
}

// row (r, c) is older than row (r2, c2): smaller diameter, then larger index
static inline bool older(uint32_t r, uint64_t c, uint32_t r2, uint64_t c2) {
  return r < r2 || (r == r2 && c > c2);
}

// low(D_s): the oldest cofacet. The first x from the top whose cofacet keeps
// the diameter is it; otherwise the oldest over all cofacets.
static bool oldest_cofacet(const HostComplex& H, const int* v, int d, uint32_t dr, uint32_t* lr,
                           uint64_t* lc) {
  bool found = false;
  if (H.sparse) {
    uint64_t mask[kMaxN / 64];
    common_neighbors(H, v, d, mask);
    for_each_desc(mask, H.nbw, [&](int x) {
      const uint32_t m = reach_of(H, v, d, x);
      const uint32_t r = std::max(dr, m);
      const uint64_t c = cofacet_index(H, v, d, x);
      if (!found || older(r, c, *lr, *lc)) {
        *lr = r;
        *lc = c;
      }
      found = true;
      return m > dr;
    });
    return found;
  }
  for (int x = H.n - 1; x >= 0; --x) {
    if (contains(v, d, x)) continue;
    const uint32_t m = reach_of(H, v, d, x);
    if (m == kInf) continue;
    const uint32_t r = std::max(dr, m);
    const uint64_t c = cofacet_index(H, v, d, x);
    if (!found || older(r, c, *lr, *lc)) {
      *lr = r;
      *lc = c;
    }
    found = true;
    if (m <= dr) break;
  }
  return found;
}

// reach[x] = max_i rank(v_i, x) for every x: the elementwise max of d+1 rank
// rows. The diagonal is kInf, so reach is kInf at the vertices of s.
static void compute_reach(const HostComplex& H, const int* v, int d, uint32_t* reach) {
  const int n = H.n;
  const uint32_t* r0 = H.Wr + (size_t)v[0] * (size_t)n;
  for (int x = 0; x < n; ++x) reach[x] = r0[x];
  for (int i = 1; i <= d; ++i) {
    const uint32_t* ri = H.Wr + (size_t)v[i] * (size_t)n;
    for (int x = 0; x < n; ++x) reach[x] = std::max(reach[x], ri[x]);
  }
}

// If row t (a (d+1)-simplex of diameter rank rt) is the cofacet of an
// apparent pair (s, t), return s, its vertices in sv and its reach row.
// Def. 5.3.4: s is the youngest facet of t (largest diameter, then smallest
// index: remove the largest vertex u whose removal keeps diam(t)), and t is
// the oldest cofacet of s (no x > u outside s keeps the diameter).
static bool apparent_partner(const HostComplex& H, uint64_t t, uint32_t rt, int d, uint64_t* s,
                             int* sv, uint32_t* reach) {
  int tv[kMaxDim + 3];
  decode_simplex(H, t, d + 1, tv);
  int drop = -1;
  for (int r = d + 1; r >= 0; --r) {  // vertices from the largest down
    uint32_t m = 0;
    for (int i = 1; i <= d + 1; ++i)
      for (int j = 0; j < i; ++j)
        if (i != r && j != r) m = std::max(m, H.wr(tv[i], tv[j]));
    if (m == rt) {
      drop = r;
      break;
    }
  }
  if (drop < 0) return false;
  int k = 0;
  for (int i = 0; i <= d + 1; ++i)
    if (i != drop) sv[k++] = tv[i];
  bool older_cofacet = false;
  if (H.sparse) {  // the caller's coboundary push walks the neighbours itself
    uint64_t mask[kMaxN / 64];
    common_neighbors(H, sv, d, mask);
    const int u = tv[drop];
    for_each_desc(mask, H.nbw, [&](int x) {
      if (x <= u) return false;
      older_cofacet |= reach_of(H, sv, d, x) <= rt;
      return !older_cofacet;
    });
  } else {
    compute_reach(H, sv, d, reach);
    for (int x = tv[drop] + 1; x < H.n; ++x) older_cofacet |= reach[x] <= rt;
  }
  if (older_cofacet) return false;
  uint64_t c = 0;
  for (int i = 0; i <= d; ++i) c += H.C(sv[i], i + 1);
  *s = c;
  return true;
}

struct Simplex {
  uint64_t c;
  uint32_t r;
  bool operator<(const Simplex& o) const { return c < o.c; }
  bool operator==(const Simplex& o) const { return c == o.c; }
};

// A column in the pivot store: its simplex and, for a column reduced here,
// the other columns whose sum with it is its reduced column (the V column of
// the reduction-matrix technique, R = D V, Sec. 5.2.9), stored elsewhere.
// Apparent columns and columns paired at their first pivot need no
// additions: their reduced column is their coboundary (vlen = 0).
struct Partner {
  uint64_t c;
  uint32_t r;     // diameter rank
  uint32_t vlen;  // length of the V column
  const Simplex* v;
};

// Append-only storage of V columns: chunks never move, so a column stored
// by one thread can be read by others once published.
class VArena {
 public:
  const Simplex* put(const Simplex* src, size_t len) {
    Simplex* dst;
    if (len > kChunk / 4) {
      big_.emplace_back(new Simplex[len]);
      dst = big_.back().get();
    } else {
      if (chunks_.empty() || used_ + len > kChunk) {
        chunks_.emplace_back(new Simplex[kChunk]);
        used_ = 0;
      }
      dst = chunks_.back().get() + used_;
      used_ += len;
    }
    std::copy(src, src + len, dst);
    return dst;
  }

 private:
  static constexpr size_t kChunk = 1 << 16;
  std::vector<std::unique_ptr<Simplex[]>> chunks_, big_;
  size_t used_ = 0;
};

// Row keys: a row (rank r, index c) is the integer (r << cbits) | (cmax - c),
// so that a smaller key is an older row and the pivot of a column (its
// oldest row) is its smallest key. cbits covers the largest cofacet index;
// the key is a u64 when the rank fits above it, a u128 otherwise.
template <class K>
struct Keys {
  int cbits;
  K cmax;
  K make(uint32_t r, uint64_t c) const { return ((K)r << cbits) | (cmax - (K)c); }
  uint32_t rank(K k) const { return (uint32_t)(k >> cbits); }
  uint64_t index(K k) const { return (uint64_t)(cmax - (k & cmax)); }
  // a 64-bit key that never decreases as the key grows: the key itself, or
  // its top 64 bits when it is wider (then rank << 32 and the top 32 bits of
  // the index part; cbits >= 32 there since a rank has at most 32 bits)
  uint64_t coarse(K k) const {
    if constexpr (sizeof(K) == 8)
      return (uint64_t)k;
    else
      return (uint64_t)(k >> (cbits - 32));
  }
};

// A vector that grows without zero-filling (default-initialised elements):
// a merge resizes its output and then writes every element.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new ((void*)p) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new ((void*)p) U(std::forward<A>(a)...);
  }
};

// The working column: a monotone min-priority queue of row keys. Rows pushed
// are never older than the current pivot and the pivot only gets younger,
// so the ranks in play only grow. Rows wait in buckets over ranges of ranks
// (2^shift consecutive ranks each, at most kMaxBuckets buckets), where a
// push is an append and a row is never moved; a bitmap marks the buckets
// that hold rows. When the pivot reaches a bucket, its rows are sorted once
// into a run (a radix sort over the key bits that vary within it); rows
// pushed into the pivot's bucket later become runs too (a coboundary is
// enumerated in decreasing index order, so a push is one ascending run per
// rank).
// Runs sit on a stack and the top two are merged while the upper one is at
// least half the size of the one below, so there are few runs and a row is
// merged O(log) times. Equal rows cancel in pairs (Z/2): a run holds each
// row at most once (a sorted batch keeps the rows of odd multiplicity), a
// merge keeps the rows that are in one run but not both, and the pivot is
// the oldest row held by an odd number of runs. Most rows at the pivot's
// rank come in pairs, so the runs stay a few times shorter than the rows
// pushed. Rows beyond the final pivot are appended once and never sorted.
template <class K>
class WorkColumn {
  using KVec = std::vector<K, NoInitAlloc<K>>;

 public:
  // nranks: the number of weight ranks (every row's rank is below it)
  WorkColumn(const Keys<K>& ks, uint32_t nranks) : ks_(ks) {
    while (((uint64_t)nranks >> shift_) >= kMaxBuckets) ++shift_;
    nb_ = (size_t)((uint64_t)nranks >> shift_) + 1;
    b_.resize(nb_);
    used_.assign((nb_ + 63) / 64, 0);
  }

  void clear() {
    for (uint32_t i : touched_) {
      b_[i].clear();
      used_[i >> 6] = 0;
    }
    touched_.clear();
    for (Run& r : runs_) give(std::move(r.v));
    runs_.clear();
    cb_ = 0;
  }

  // the bucket the pivot is in holds the rows at its ranks that are not in a
  // run yet
  void push(K k) {
    const uint32_t i = ks_.rank(k) >> shift_;
    KVec& v = b_[i];
    if (v.empty()) mark(i);
    v.push_back(k);
  }

  void push_many(const K* k, size_t m) {
    for (size_t i = 0; i < m; ++i) push(k[i]);
  }

  // the pivot (smallest key of odd multiplicity), kept in the column; false
  // if the column is zero
  bool pivot(K* out) {
    for (;;) {
      KVec& l = b_[cb_];
      if (!l.empty()) {
        sort_runs(l);
        if (!l.empty()) {
          KVec v = take();
          v.swap(l);
          add_run(std::move(v));
        }
      }
      K top = 0;
      bool any = false;
      for (size_t i = 0; i < runs_.size();) {
        Run& r = runs_[i];
        if (r.pos == r.v.size()) {  // spent
          give(std::move(r.v));
          runs_.erase(runs_.begin() + (std::ptrdiff_t)i);
          continue;
        }
        if (!any || r.v[r.pos] < top) top = r.v[r.pos];
        any = true;
        ++i;
      }
      if (!any) {
        if (!advance()) return false;
        continue;
      }
      // runs hold distinct rows: each run holds top at most once
      size_t k = 0, last = 0;
      for (size_t i = 0; i < runs_.size(); ++i) {
        Run& r = runs_[i];
        if (r.v[r.pos] == top) {
          ++r.pos;
          ++k;
          last = i;
        }
      }
      if (k & 1) {
        --runs_[last].pos;  // one copy stays
        *out = top;
        return true;
      }
    }
  }

 private:
  struct Run {
    KVec v;
    size_t pos = 0;
    size_t left() const { return v.size() - pos; }
  };

  void mark(uint32_t i) {
    uint64_t& w = used_[i >> 6];
    const uint64_t bit = 1ull << (i & 63);
    if (!(w & bit)) {
      w |= bit;
      touched_.push_back(i);
    }
  }

  // the pivot moves on to the next bucket that holds rows
  bool advance() {
    used_[cb_ >> 6] &= ~(1ull << (cb_ & 63));
    size_t i = cb_ + 1;
    if (i >= nb_) return false;
    size_t w = i >> 6;
    uint64_t m = used_[w] & (~0ull << (i & 63));
    while (!m) {
      if (++w == used_.size()) return false;
      m = used_[w];
    }
    cb_ = (uint32_t)(w * 64 + (size_t)__builtin_ctzll(m));
    return true;
  }

  // Sort a batch of rows and keep one copy of each row of odd multiplicity.
  void sort_runs(KVec& l) {
    sort_rows(l);
    l.resize(odd_rows(l.data(), l.size()));
  }

  // keep one copy of each row of odd multiplicity in a sorted sequence
  static size_t odd_rows(K* a, size_t n) {
    size_t o = 0;
    for (size_t i = 0; i < n;) {
      size_t j = i + 1;
      while (j < n && a[j] == a[i]) ++j;
      a[o] = a[i];
      o += (j - i) & 1;
      i = j;
    }
    return o;
  }

  // the rows in exactly one of two runs (each strictly increasing), in
  // order; branch-free while both have rows
  static size_t xor_merge(const K* a, size_t na, const K* b, size_t nb, K* out) {
    size_t i = 0, j = 0, o = 0;
    while (i < na && j < nb) {
      const K x = a[i], y = b[j];
      out[o] = x < y ? x : y;
      o += (size_t)(x != y);
      i += (size_t)(x <= y);
      j += (size_t)(y <= x);
    }
    while (i < na) out[o++] = a[i++];
    while (j < nb) out[o++] = b[j++];
    return o;
  }

  // The rows of a batch arrive as a concatenation of ascending runs, one
  // per push: up to kMergeRuns runs are merged pairwise, more are radix
  // sorted.
  void sort_rows(KVec& l) {
    constexpr int kMergeRuns = 8;
    size_t bounds[kMergeRuns + 1];
    int runs = 1;
    bounds[0] = 0;
    for (size_t i = 1; i < l.size(); ++i)
      if (l[i] < l[i - 1]) {
        if (runs == kMergeRuns) {
          radix_sort(l);
          return;
        }
        bounds[runs++] = i;
      }
    if (runs == 1) return;
    bounds[runs] = l.size();
    KVec t = take();
    t.resize(l.size());
    KVec* src = &l;
    KVec* dst = &t;
    while (runs > 1) {
      int out = 0;
      for (int r = 0; r < runs; r += 2) {
        // runs r and r + 1 (a last odd run is copied: m = e)
        const size_t b = bounds[r], m = bounds[r + 1], e = r + 1 < runs ? bounds[r + 2] : m;
        std::merge(src->begin() + (std::ptrdiff_t)b, src->begin() + (std::ptrdiff_t)m,
                   src->begin() + (std::ptrdiff_t)m, src->begin() + (std::ptrdiff_t)e,
                   dst->begin() + (std::ptrdiff_t)b);
        bounds[out++] = b;
      }
      bounds[out] = l.size();
      runs = out;
      std::swap(src, dst);
    }
    if (src != &l) l.swap(*src);
    give(std::move(t));
  }

  // LSD radix sort, 8 bits a pass, over the bytes in which the keys of the
  // batch differ (within a bucket only the index part and the low rank bits
  // vary); small batches and keys that differ above bit 63 go to std::sort
  void radix_sort(KVec& l) {
    const size_t n = l.size();
    K diff = 0;
    for (size_t i = 1; i < n; ++i) diff |= l[i] ^ l[0];
    if (n < 64 || (diff >> 32 >> 32) != 0) {
      std::sort(l.begin(), l.end());
      return;
    }
    const uint64_t dv = (uint64_t)diff;
    KVec t = take();
    t.resize(n);
    KVec* src = &l;
    KVec* dst = &t;
    for (int sh = 0; sh < 64; sh += 8) {
      if (((dv >> sh) & 0xFF) == 0) continue;
      uint32_t cnt[256] = {};
      for (size_t i = 0; i < n; ++i) ++cnt[((uint64_t)(*src)[i] >> sh) & 0xFF];
      uint32_t sum = 0;
      for (int b = 0; b < 256; ++b) {
        const uint32_t c = cnt[b];
        cnt[b] = sum;
        sum += c;
      }
      K* out = dst->data();
      for (size_t i = 0; i < n; ++i) {
        const K x = (*src)[i];
        out[cnt[((uint64_t)x >> sh) & 0xFF]++] = x;
      }
      std::swap(src, dst);
    }
    if (src != &l) l.swap(*src);
    give(std::move(t));
  }

  KVec take() {
    if (spare_.empty()) return {};
    KVec v = std::move(spare_.back());
    spare_.pop_back();
    return v;
  }
  void give(KVec&& v) {
    v.clear();
    spare_.push_back(std::move(v));
  }

  void add_run(KVec&& v) {
    runs_.push_back(Run{std::move(v), 0});
    while (runs_.size() >= 2 && runs_.back().left() * 2 >= runs_[runs_.size() - 2].left()) {
      Run& a = runs_[runs_.size() - 2];
      Run& b = runs_.back();
      KVec m = take();
      m.resize(a.left() + b.left());
      m.resize(xor_merge(a.v.data() + a.pos, a.left(), b.v.data() + b.pos, b.left(), m.data()));
      give(std::move(a.v));
      give(std::move(b.v));
      runs_.pop_back();
      runs_.back() = Run{std::move(m), 0};
    }
  }

  static constexpr uint64_t kMaxBuckets = 1024;
  Keys<K> ks_;
  int shift_ = 0;
  size_t nb_ = 0;
  std::vector<KVec> b_;
  std::vector<uint64_t> used_;     // buckets holding rows (or once did, this column)
  std::vector<uint32_t> touched_;  // buckets marked since the last clear
  std::vector<Run> runs_;
  std::vector<KVec> spare_;
  uint32_t cb_ = 0;  // the bucket the pivot is in
};

// Push the cofacets of simplex v (index c, diameter rank dr) that are not
// older than the row `limit`; `reach` is its reach row, computed here unless
// the caller has it; kb is scratch for 2n keys. Used to add a reduced column R_k whose pivot is
// `limit`: R_k is zero below its pivot, so the parts of its summands below
// the pivot cancel and are not pushed. Cofacet s + {x} has index (Alg. 14)
// high + C(x, j+2) + low with j+1 the number of vertices below x: vertices
// above x contribute C(v_i, i+2) to `high` (they moved up one position),
// those below C(v_i, i+1) to `low`. Between two vertices of s these sums are
// constant, so the keys of a stretch of x are computed in one pass; pushes
// then go out in decreasing index order.
template <class K>
static void push_coboundary(const HostComplex& H, const Keys<K>& ks, const int* v, uint64_t c,
                            uint32_t dr, int d, K limit, WorkColumn<K>& w, uint32_t* reach,
                            bool have_reach, K* kb) {
  const int n = H.n;
  if (H.sparse) {
    // only the common neighbours have cofacets in the complex; the index
    // sums move past a vertex of s when x drops below it
    uint64_t mask[kMaxN / 64];
    common_neighbors(H, v, d, mask);
    uint64_t high = 0, low = c;
    int pos = d;
    size_t m = 0;  // kept rows, selected without branches into kb
    for_each_desc(mask, H.nbw, [&](int x) {
      while (pos >= 0 && v[pos] > x) {
        high += H.C(v[pos], pos + 2);
        low -= H.C(v[pos], pos + 1);
        --pos;
      }
      const K k = ks.make(std::max(dr, reach_of(H, v, d, x)), high + H.C(x, pos + 2) + low);
      kb[m] = k;
      m += (size_t)(k >= limit);
      return true;
    });
    w.push_many(kb, m);
    return;
  }
  if (!have_reach) compute_reach(H, v, d, reach);
  uint64_t high = 0, low = c;
  int hi = n;  // the stretch is [lo, hi)
  for (int pos = d; pos >= -1; --pos) {
    const int lo = pos >= 0 ? v[pos] + 1 : 0;
    const uint64_t base = high + low;
    const uint64_t* row = H.binom + (size_t)(pos + 2) * (size_t)(n + 1);
    for (int x = lo; x < hi; ++x) kb[x] = ks.make(std::max(dr, reach[x]), base + row[x]);
    if (pos >= 0) {
      high += H.C(v[pos], pos + 2);
      low -= H.C(v[pos], pos + 1);
      hi = v[pos];
    }
  }
  // push in decreasing index order; the rows are selected without branches
  // (whether a row is kept depends on the data) into the second half of kb
  K* sel = kb + n;
  size_t m = 0;
  for (int x = n - 1; x >= 0; --x) {
    const K k = kb[x];
    sel[m] = k;
    m += (size_t)((reach[x] != kInf) & (k >= limit));
  }
  w.push_many(sel, m);
}

// Row index -> column of this dimension's reduced pivots, shared by the
// reduction threads: open addressing with linear probing at load <= 1/2 (a
// row index is < 2^63, so ~0 and ~1 are free to mark an empty slot and one
// being filled). An inserter claims an empty slot, writes the value, then
// publishes the key (release); a reader that meets a slot being filled waits
// for it. Entries are never removed.
class PivotTable {
 public:
  explicit PivotTable(size_t n) {
    size_t cap = 16;
    int bits = 4;
    while (cap < 2 * n + 2) {
      cap <<= 1;
      ++bits;
    }
    keys_.reset(new std::atomic<uint64_t>[cap]);
    for (size_t i = 0; i < cap; ++i) keys_[i].store(kEmpty, std::memory_order_relaxed);
    vals_.reset(new Partner[cap]);
    mask_ = cap - 1;
    shift_ = 64 - bits;
  }
  bool find(uint64_t k, Partner* out) const {
    for (size_t i = slot(k);; i = (i + 1) & mask_) {
      uint64_t s = keys_[i].load(std::memory_order_acquire);
      while (s == kBusy) {
        std::this_thread::yield();
        s = keys_[i].load(std::memory_order_acquire);
      }
      if (s == k) {
        *out = vals_[i];
        return true;
      }
      if (s == kEmpty) return false;
    }
  }
  // start loading the slot of row k (a lookup in a large table misses the
  // caches)
  void prefetch(uint64_t k) const {
    const size_t i = slot(k);
    __builtin_prefetch(&keys_[i]);
    __builtin_prefetch(&vals_[i]);
  }
  void insert(uint64_t k, const Partner& p) {
    for (size_t i = slot(k);; i = (i + 1) & mask_) {
      uint64_t e = kEmpty;
      if (keys_[i].load(std::memory_order_relaxed) == kEmpty &&
          keys_[i].compare_exchange_strong(e, kBusy, std::memory_order_acq_rel)) {
        vals_[i] = p;
        keys_[i].store(k, std::memory_order_release);
        return;
      }
    }
  }

 private:
  static constexpr uint64_t kEmpty = ~0ull, kBusy = ~0ull - 1;
  size_t slot(uint64_t k) const { return (size_t)((k * 0x9E3779B97F4A7C15ull) >> shift_); }
  std::unique_ptr<std::atomic<uint64_t>[]> keys_;
  std::unique_ptr<Partner[]> vals_;
  size_t mask_ = 0;
  int shift_ = 0;
};

// The part of a column's reduction that does not depend on other columns.
// While the pivot of a column is the cofacet of an apparent pair, Alg. 2
// adds that apparent column: the pivot store of the other non-apparent
// columns is never consulted for such a row, because the cofacet of an
// apparent pair is the pivot of its own column only (pivots are unique).
// So each column can follow its chain of apparent pivots on its own, in
// parallel, until it reaches a row that is not an apparent cofacet; the
// sequential pass then only continues the columns whose row is already
// taken. The sequence of additions is exactly the sequential one.
struct PreReduced {
  uint64_t lc;      // pivot after the apparent chain (row index)
  uint32_t lr;      // its rank
  uint32_t dr;      // diameter rank of the column
  uint32_t voff;    // apparent columns added: chain_v[j / kChunk][voff, voff + vcount)
  uint32_t vcount;
  bool nonzero;
};

constexpr int64_t kChunk = 256;

template <class K>
static void pre_reduce(const HostComplex& H, const Keys<K>& ks, int d, const Column* cols,
                       int64_t ncols, int threads, std::vector<PreReduced>& out,
                       std::vector<std::vector<Simplex>>& chain_v, int64_t* additions) {
  out.resize((size_t)ncols);
  chain_v.assign((size_t)((ncols + kChunk - 1) / kChunk), {});
  std::atomic<int64_t> next{0}, adds{0};
  auto worker = [&]() {
    int v[kMaxDim + 3], sv[kMaxDim + 3];
    WorkColumn<K> work(ks, H.nranks);
    std::vector<uint32_t> reach((size_t)H.n), areach((size_t)H.n);
    std::vector<K> kb(2 * (size_t)H.n);
    int64_t local_adds = 0;
    for (;;) {
      const int64_t j0 = next.fetch_add(kChunk);
      if (j0 >= ncols) break;
      const int64_t j1 = std::min<int64_t>(ncols, j0 + kChunk);
      std::vector<Simplex>& cv = chain_v[(size_t)(j0 / kChunk)];
      for (int64_t j = j0; j < j1; ++j) {
        PreReduced& f = out[(size_t)j];
        const uint64_t c = cols[j].cidx;
        decode_simplex(H, c, d, v);
        f.dr = rank_of(H, v, d);
        f.voff = (uint32_t)cv.size();
        f.vcount = 0;
        f.nonzero = oldest_cofacet(H, v, d, f.dr, &f.lr, &f.lc);
        uint64_t s;
        if (!f.nonzero || !apparent_partner(H, f.lc, f.lr, d, &s, sv, areach.data())) continue;
        K low = ks.make(f.lr, f.lc);
        work.clear();
        push_coboundary(H, ks, v, c, f.dr, d, low, work, reach.data(), false, kb.data());
        for (;;) {
          push_coboundary(H, ks, sv, s, f.lr, d, low, work, areach.data(), true, kb.data());
          cv.push_back(Simplex{s, f.lr});
          ++f.vcount;
          ++local_adds;
          if (!work.pivot(&low)) {
            f.nonzero = false;
            break;
          }
          f.lr = ks.rank(low);
          f.lc = ks.index(low);
          if (!apparent_partner(H, f.lc, f.lr, d, &s, sv, areach.data())) break;
        }
      }
    }
    adds += local_adds;
  };
  threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, ncols / 1024));
  std::vector<std::thread> pool;
  for (int i = 1; i < threads; ++i) pool.emplace_back(worker);
  worker();
  for (std::thread& t : pool) t.join();
  *additions += adds.load();
}

// The columns that the apparent chains leave with a pivot taken by another
// column are reduced on `threads` threads at once, with the same result as
// the column-by-column pass of Alg. 2. Column j adds R_k whenever its pivot
// is the pivot of an earlier column k; it may stop at a pivot l only once no
// earlier column can still end at l. A column's pivot only gets younger
// while it is reduced (its key only grows), so an earlier column whose
// current pivot key is above l's can no longer end at l, and a finished one
// has its pivot in the table. Each thread publishes the column it holds and
// that column's current pivot key (coarsened to 64 bits, which only makes
// the test more cautious). Columns are taken in order, under a lock that
// also publishes the new column, so every earlier column that is not
// finished is held by a thread. Column j waits while an earlier held
// column's key is <= l's, then looks l up again (a finished column's pivot
// is in the table before its thread takes another column). The earliest
// unfinished column never waits, so the pass always progresses; the
// additions each column makes are exactly those of the sequential pass. A
// finished column's V column is stored before its pivot is published, so a
// column found in the table can be added at once.
// The bookkeeping costs a few hundred nanoseconds per column and waits are
// common among columns of equal diameter, so the pass runs in blocks: a
// block goes to all threads only when the columns of the block before took
// more than kParallelNs each on one thread (long columns: many additions,
// or large coboundaries), and wide blocks continue while their columns stay
// that long and the threads' busy time (their time outside waits) is at
// least kMinSpeedup times the block's wall time.
template <class K>
static void reduce_keys(const HostComplex& H, const Keys<K>& ks, int d, const Column* cols,
                        int64_t ncols, int threads, std::vector<PairRec>& pairs,
                        std::vector<uint64_t>& deaths, ReduceStats& stats, bool always_wide) {
  PivotTable pivots((size_t)ncols);
  std::vector<PreReduced> pre;
  std::vector<std::vector<Simplex>> chain_v;
  pre_reduce(H, ks, d, cols, ncols, threads, pre, chain_v, &stats.additions);

  // column j's pair goes to pairs[first + j]
  const size_t first = pairs.size();
  pairs.resize(first + (size_t)ncols);

  threads = std::max(threads, 1);
  // per thread: the column it holds (-1: none) and that column's current
  // pivot key, coarsened
  std::unique_ptr<std::atomic<int64_t>[]> held_col(new std::atomic<int64_t>[threads]);
  std::unique_ptr<std::atomic<uint64_t>[]> held_key(new std::atomic<uint64_t>[threads]);
  for (int t = 0; t < threads; ++t) {
    held_col[t].store(-1, std::memory_order_relaxed);
    held_key[t].store(0, std::memory_order_relaxed);
  }
  std::atomic_flag take_lock = ATOMIC_FLAG_INIT;
  int64_t next = 0, end = 0;
  int nthr = 1;  // threads of the current block
  std::atomic<int64_t> adds{0}, emergent{0}, busy_ns{0};
  // waits that last: a few yields, then short sleeps, so that waiting
  // threads leave the cores to the columns they wait for
  auto backoff = [](int& spins) {
    if (++spins < 64)
      std::this_thread::yield();
    else
      std::this_thread::sleep_for(std::chrono::microseconds(20));
  };

  // per-thread scratch, kept across blocks
  struct Scratch {
    WorkColumn<K> work;
    std::vector<Simplex> vj, red;
    VArena arena;
    std::vector<uint32_t> reach, areach;
    std::vector<K> kb;
    Scratch(const Keys<K>& k, const HostComplex& H)
        : work(k, H.nranks), reach((size_t)H.n), areach((size_t)H.n), kb(2 * (size_t)H.n) {}
  };
  std::vector<std::unique_ptr<Scratch>> scratch((size_t)threads);
  auto worker = [&](int self) {
    const auto w0 = std::chrono::steady_clock::now();
    double waited = 0;
    if (!scratch[(size_t)self]) scratch[(size_t)self].reset(new Scratch(ks, H));
    Scratch& sc = *scratch[(size_t)self];
    WorkColumn<K>& work = sc.work;
    std::vector<Simplex>& vj = sc.vj;
    std::vector<Simplex>& red = sc.red;
    std::vector<uint32_t>& reach = sc.reach;
    std::vector<uint32_t>& areach = sc.areach;
    std::vector<K>& kb = sc.kb;
    int sv[kMaxDim + 3], pv[kMaxDim + 3];
    int64_t local_adds = 0, local_emergent = 0;
    // returns once no earlier column held by another thread can still end
    // at row l (key coarsened to lq)
    auto settle = [&](int64_t j, uint64_t lq) {
      for (int t = 0; t < nthr; ++t) {
        if (t == self) continue;
        std::chrono::steady_clock::time_point s0;
        for (int spins = 0;; backoff(spins)) {
          const int64_t k = held_col[t].load(std::memory_order_acquire);
          if (k < 0 || k >= j || held_key[t].load(std::memory_order_acquire) > lq) {
            if (spins > 0)
              waited += std::chrono::duration<double, std::nano>(
                            std::chrono::steady_clock::now() - s0).count();
            break;
          }
          if (spins == 0) s0 = std::chrono::steady_clock::now();
        }
      }
    };
    for (;;) {
      int64_t j;
      if (nthr == 1) {  // alone: nothing to publish
        if (next >= end) break;
        j = next++;
        // the table slots of a column a few ahead: most columns need only
        // a lookup and an insert, each a cache miss in a large table
        constexpr int64_t kAhead = 8;
        if (j + kAhead < end && pre[(size_t)(j + kAhead)].nonzero)
          pivots.prefetch(pre[(size_t)(j + kAhead)].lc);
      } else {
        for (int spins = 0; take_lock.test_and_set(std::memory_order_acquire); backoff(spins)) {
        }
        if (next >= end) {
          take_lock.clear(std::memory_order_release);
          break;
        }
        j = next++;
        held_key[self].store(ks.coarse(ks.make(pre[(size_t)j].lr, pre[(size_t)j].lc)),
                             std::memory_order_release);
        held_col[self].store(j, std::memory_order_release);
        take_lock.clear(std::memory_order_release);
      }
      const uint64_t c = cols[j].cidx;
      const PreReduced& f = pre[(size_t)j];
      const Simplex* chain = chain_v[(size_t)(j / kChunk)].data() + f.voff;
      const uint32_t dr = f.dr;
      uint32_t lr = f.lr;
      uint64_t lc = f.lc;
      bool nonzero = f.nonzero;
      vj.assign(chain, chain + f.vcount);
      Partner p{};
      bool have_p = false;
      if (nonzero) {
        have_p = pivots.find(lc, &p);
        if (!have_p) {
          settle(j, ks.coarse(ks.make(lr, lc)));
          have_p = pivots.find(lc, &p);
        }
      }
      if (have_p) {
        // Alg. 2 on column j, continued: while its pivot is the pivot of an
        // earlier column k, add R_k = D_k + sum_{i in V_k} D_i (the pivot
        // then moves up). Lookups are two-layer (Fig. 5.10): pairs found by
        // this reduction first, then the apparent pairs, recognised from
        // Def. 5.3.4 instead of a stored array. The working column restarts
        // from the column and the apparent columns its chain added.
        bool pv_known = false;  // pv holds the vertices of p.c
        K low = ks.make(lr, lc);
        work.clear();
        decode_simplex(H, c, d, sv);
        push_coboundary(H, ks, sv, c, dr, d, low, work, reach.data(), false, kb.data());
        for (uint32_t i = 0; i < f.vcount; ++i) {
          decode_simplex(H, chain[i].c, d, sv);
          push_coboundary(H, ks, sv, chain[i].c, chain[i].r, d, low, work, reach.data(), false,
                          kb.data());
        }
        for (;;) {
          if (!pv_known) decode_simplex(H, p.c, d, pv);
          if (pv_known)  // its reach row came with the lookup
            push_coboundary(H, ks, pv, p.c, p.r, d, low, work, areach.data(), true, kb.data());
          else
            push_coboundary(H, ks, pv, p.c, p.r, d, low, work, reach.data(), false, kb.data());
          vj.push_back(Simplex{p.c, p.r});
          for (uint32_t i = 0; i < p.vlen; ++i) {
            const Simplex& r = p.v[i];
            decode_simplex(H, r.c, d, sv);
            push_coboundary(H, ks, sv, r.c, r.r, d, low, work, reach.data(), false, kb.data());
            vj.push_back(r);
          }
          ++local_adds;
          if (!work.pivot(&low)) {
            nonzero = false;
            break;
          }
          lr = ks.rank(low);
          lc = ks.index(low);
          held_key[self].store(ks.coarse(low), std::memory_order_release);
          if (pivots.find(lc, &p)) {
            pv_known = false;
          } else if (apparent_partner(H, lc, lr, d, &p.c, pv, areach.data())) {
            p.r = lr;
            p.vlen = 0;
            pv_known = true;
          } else {
            settle(j, ks.coarse(low));
            if (pivots.find(lc, &p))
              pv_known = false;
            else
              break;
          }
        }
      } else if (nonzero && f.vcount == 0) {
        ++local_emergent;
      }
      if (nonzero) {
        Partner mine{c, dr, 0, nullptr};
        if (!vj.empty()) {
          // V over Z/2: a column added twice cancels
          std::sort(vj.begin(), vj.end());
          red.clear();
          for (size_t a = 0; a < vj.size();) {
            size_t b = a;
            while (b < vj.size() && vj[b] == vj[a]) ++b;
            if ((b - a) & 1) red.push_back(vj[a]);
            a = b;
          }
          mine.vlen = (uint32_t)red.size();
          mine.v = sc.arena.put(red.data(), red.size());
        }
        pivots.insert(lc, mine);
        pairs[first + (size_t)j] = PairRec{c, lc, H.rank_bits[dr], H.rank_bits[lr]};
      } else {
        pairs[first + (size_t)j] = PairRec{c, ~0ull, H.rank_bits[dr], kInf};
      }
    }
    held_col[self].store(-1, std::memory_order_release);
    busy_ns += (int64_t)(std::chrono::duration<double, std::nano>(
                             std::chrono::steady_clock::now() - w0).count() - waited);
    adds += local_adds;
    emergent += local_emergent;
  };
  constexpr double kParallelNs = 2000.0, kMinSpeedup = 2.0;
  constexpr int64_t kProbeBlock = 256, kMaxNarrowBlock = 8192, kParallelBlock = 8192;
  constexpr int kCooldown = 16;  // one-thread blocks after a wide one that did not pay
  bool wide = always_wide && threads > 1;
  int cooldown = 0;
  int64_t narrow_block = kProbeBlock;  // grows while the columns stay short
  while (next < ncols) {
    const int64_t j0 = next;
    end = std::min<int64_t>(ncols, j0 + (wide ? kParallelBlock : narrow_block));
    nthr = wide ? (int)std::min<int64_t>(threads, end - j0) : 1;
    busy_ns = 0;
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> pool;
    for (int t = 1; t < nthr; ++t) pool.emplace_back(worker, t);
    worker(0);
    for (std::thread& t : pool) t.join();
    const double wall =
        std::chrono::duration<double, std::nano>(std::chrono::steady_clock::now() - t0).count();
    const double per_col = (double)busy_ns.load() / (double)(end - j0);
    if (always_wide) {
      wide = threads > 1;
    } else if (wide) {
      if ((double)busy_ns.load() < kMinSpeedup * wall) {
        wide = false;
        cooldown = kCooldown;
      } else {
        wide = per_col > kParallelNs;
      }
      narrow_block = kProbeBlock;
    } else {
      narrow_block = per_col < 0.25 * kParallelNs ? std::min(2 * narrow_block, kMaxNarrowBlock)
                                                  : kProbeBlock;
      if (cooldown > 0)
        --cooldown;
      else
        wide = threads > 1 && per_col > kParallelNs;
    }
  }
  stats.additions += adds.load();
  stats.emergent += emergent.load();

  for (size_t i = first; i < pairs.size(); ++i)
    if (pairs[i].death != ~0ull) deaths.push_back(pairs[i].death);
}

// Explicit matrices: the same blocks and the same stopping rule as
// reduce_keys, mirrored (Alg. 2 works left to right and a pivot is a
// column's lowest row, which only falls as columns are added).
bool reduce_explicit_columns(int64_t n, const int64_t* ptr, const int64_t* rows,
                             const int32_t* lookup, const int64_t* unstable, int64_t nun,
                             int threads, int64_t* low, int64_t* additions, bool always_wide) {
  std::unique_ptr<std::atomic<int64_t>[]> pivot_of(new std::atomic<int64_t>[(size_t)n]);
  for (int64_t r = 0; r < n; ++r) {
    pivot_of[r].store(lookup[r], std::memory_order_relaxed);
    low[r] = -1;
  }
  for (int64_t r = 0; r < n; ++r)
    if (lookup[r] >= 0) low[lookup[r]] = r;
  if (nun == 0) return true;
  // reduced unstable columns, by position in `unstable`; red_of[j] is that
  // position for column j (written before j's pivot is published)
  std::vector<std::vector<int64_t>> red((size_t)nun);
  std::vector<int32_t> red_of((size_t)n, -1);
  for (int64_t u = 0; u < nun; ++u) red_of[(size_t)unstable[u]] = (int32_t)u;

  threads = std::max(threads, 1);
  std::unique_ptr<std::atomic<int64_t>[]> held_col(new std::atomic<int64_t>[threads]);
  std::unique_ptr<std::atomic<int64_t>[]> held_low(new std::atomic<int64_t>[threads]);
  for (int t = 0; t < threads; ++t) {
    held_col[t].store(-1, std::memory_order_relaxed);
    held_low[t].store(-1, std::memory_order_relaxed);
  }
  std::atomic_flag take_lock = ATOMIC_FLAG_INIT;
  int64_t next = 0, end = 0;
  int nthr = 1;
  std::atomic<int64_t> adds{0}, busy_ns{0};
  std::atomic<bool> bad{false};
  auto backoff = [](int& spins) {
    if (++spins < 64)
      std::this_thread::yield();
    else
      std::this_thread::sleep_for(std::chrono::microseconds(20));
  };
  auto worker = [&](int self) {
    const auto w0 = std::chrono::steady_clock::now();
    double waited = 0;
    std::vector<int64_t> work, tmp;
    int64_t local_adds = 0;
    // returns once no earlier column held by another thread can still end
    // at row l (its lowest row is already below l)
    auto settle = [&](int64_t j, int64_t l) {
      for (int t = 0; t < nthr; ++t) {
        if (t == self) continue;
        std::chrono::steady_clock::time_point s0;
        for (int spins = 0;; backoff(spins)) {
          const int64_t k = held_col[t].load(std::memory_order_acquire);
          if (k < 0 || k >= j || held_low[t].load(std::memory_order_acquire) < l) {
            if (spins > 0)
              waited += std::chrono::duration<double, std::nano>(
                            std::chrono::steady_clock::now() - s0).count();
            break;
          }
          if (spins == 0) s0 = std::chrono::steady_clock::now();
        }
      }
    };
    for (;;) {
      int64_t u;
      if (nthr == 1) {
        if (next >= end) break;
        u = next++;
      } else {
        for (int spins = 0; take_lock.test_and_set(std::memory_order_acquire); backoff(spins)) {
        }
        if (next >= end) {
          take_lock.clear(std::memory_order_release);
          break;
        }
        u = next++;
        const int64_t jj = unstable[u];
        held_low[self].store(ptr[jj + 1] > ptr[jj] ? rows[ptr[jj + 1] - 1] : -1,
                             std::memory_order_release);
        held_col[self].store(jj, std::memory_order_release);
        take_lock.clear(std::memory_order_release);
      }
      const int64_t j = unstable[u];
      work.assign(rows + ptr[j], rows + ptr[j + 1]);
      while (!work.empty()) {
        const int64_t l = work.back();
        int64_t k = pivot_of[l].load(std::memory_order_acquire);
        if (k < 0) {
          settle(j, l);
          k = pivot_of[l].load(std::memory_order_acquire);
          if (k < 0) {  // j's pivot
            low[j] = l;
            red[(size_t)u] = work;
            pivot_of[l].store(j, std::memory_order_release);
            break;
          }
        }
        if (k >= j) {
          bad.store(true);
          break;
        }
        const int64_t *kb, *ke;
        if (red_of[(size_t)k] >= 0) {
          const std::vector<int64_t>& rk = red[(size_t)red_of[(size_t)k]];
          kb = rk.data();
          ke = kb + rk.size();
        } else {  // a pivot the scan fixed: its column as it is
          kb = rows + ptr[k];
          ke = rows + ptr[k + 1];
        }
        tmp.clear();
        std::set_symmetric_difference(work.begin(), work.end(), kb, ke, std::back_inserter(tmp));
        work.swap(tmp);
        ++local_adds;
        if (nthr > 1)
          held_low[self].store(work.empty() ? -1 : work.back(), std::memory_order_release);
      }
    }
    held_col[self].store(-1, std::memory_order_release);
    busy_ns += (int64_t)(std::chrono::duration<double, std::nano>(
                             std::chrono::steady_clock::now() - w0).count() - waited);
    adds += local_adds;
  };
  constexpr double kParallelNs = 2000.0, kMinSpeedup = 2.0;
  constexpr int64_t kProbeBlock = 256, kMaxNarrowBlock = 8192, kParallelBlock = 8192;
  constexpr int kCooldown = 16;
  bool wide = always_wide && threads > 1;
  int cooldown = 0;
  int64_t narrow_block = kProbeBlock;
  while (next < nun) {
    const int64_t u0 = next;
    end = std::min<int64_t>(nun, u0 + (wide ? kParallelBlock : narrow_block));
    nthr = wide ? (int)std::min<int64_t>(threads, end - u0) : 1;
    busy_ns = 0;
    const auto t0 = std::chrono::steady_clock::now();
    std::vector<std::thread> pool;
    for (int t = 1; t < nthr; ++t) pool.emplace_back(worker, t);
    worker(0);
    for (std::thread& t : pool) t.join();
    if (bad.load()) return false;
    const double wall =
        std::chrono::duration<double, std::nano>(std::chrono::steady_clock::now() - t0).count();
    const double per_col = (double)busy_ns.load() / (double)(end - u0);
    if (always_wide) {
      wide = threads > 1;
    } else if (wide) {
      if ((double)busy_ns.load() < kMinSpeedup * wall) {
        wide = false;
        cooldown = kCooldown;
      } else {
        wide = per_col > kParallelNs;
      }
      narrow_block = kProbeBlock;
    } else {
      narrow_block = per_col < 0.25 * kParallelNs ? std::min(2 * narrow_block, kMaxNarrowBlock)
                                                  : kProbeBlock;
      if (cooldown > 0)
        --cooldown;
      else
        wide = threads > 1 && per_col > kParallelNs;
    }
  }
  *additions += adds.load();
  return true;
}

bool compress_explicit(int64_t n, const int64_t* ptr, const int64_t* rows, const int32_t* lookup,
                       const uint8_t* destroyer, const int64_t* unstable, int64_t nun,
                       int threads, std::vector<int64_t>& cptr, std::vector<int64_t>& crows,
                       int64_t* additions, int64_t* dropped) {
  // compressed pivot columns of the scan, and whether one is a single entry
  std::vector<int64_t> sarena, sbeg((size_t)n, -1);
  std::vector<int32_t> slen((size_t)n, 0);
  std::vector<uint8_t> single((size_t)n, 0);
  // Alg. 8 on one column c (source rows [b, e), increasing) into `out`
  // (increasing): rows are taken from the lowest up, so what an addition
  // brings in (rows above the one it removes) is still to be looked at.
  auto compress = [&](int64_t c, const int64_t* b, const int64_t* e, std::vector<int64_t>& out,
                      std::vector<int64_t>& work, std::vector<int64_t>& tmp, int64_t& adds,
                      int64_t& drops) -> bool {
    work.assign(b, e);
    out.clear();
    while (!work.empty()) {
      const int64_t r = work.back();
      work.pop_back();
      if (destroyer[r]) {  // column r keeps a pivot (Lemma 4.2.5): row r is zero (Lemma 4.2.4)
        ++drops;
        continue;
      }
      const int64_t p = lookup[r];
      if (p >= 0 && p < c) {
        if (single[(size_t)p]) {  // adding column p, a single 1 at row r, removes it
          ++drops;
          continue;
        }
        // add compressed column p; its lowest 1, at r, cancels the one removed
        const int64_t* pb = sarena.data() + sbeg[(size_t)p];
        const int64_t* pe = pb + slen[(size_t)p];
        if (pe[-1] != r) return false;  // the scan's pivot was compressed away: not a boundary matrix
        tmp.clear();
        std::set_symmetric_difference(work.begin(), work.end(), pb, pe - 1, std::back_inserter(tmp));
        work.swap(tmp);
        ++adds;
        continue;
      }
      out.push_back(r);
    }
    std::reverse(out.begin(), out.end());
    return true;
  };

  int64_t adds = 0, drops = 0;
  {
    // the scan's pivot columns, in increasing order: a column only adds
    // compressed pivot columns to its left
    std::vector<int64_t> piv;
    for (int64_t r = 0; r < n; ++r)
      if (lookup[r] >= 0) piv.push_back(lookup[r]);
    std::sort(piv.begin(), piv.end());
    std::vector<int64_t> out, work, tmp;
    for (int64_t p : piv) {
      if (!compress(p, rows + ptr[p], rows + ptr[p + 1], out, work, tmp, adds, drops)) return false;
      sbeg[(size_t)p] = (int64_t)sarena.size();
      slen[(size_t)p] = (int32_t)out.size();
      single[(size_t)p] = out.size() == 1;
      sarena.insert(sarena.end(), out.begin(), out.end());
    }
  }
  // the unstable columns are independent of each other: ranges of them on
  // the host threads, each into an arena of its own
  threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, (nun + 4095) / 4096));
  std::vector<std::vector<int64_t>> arena((size_t)threads);
  std::vector<int64_t> ubeg((size_t)nun), ulen((size_t)nun);
  std::vector<int64_t> t_adds((size_t)threads, 0), t_drops((size_t)threads, 0);
  std::vector<char> t_ok((size_t)threads, 1);
  auto run = [&](int t) {
    const int64_t u0 = nun * t / threads, u1 = nun * (t + 1) / threads;
    std::vector<int64_t> out, work, tmp;
    for (int64_t u = u0; u < u1; ++u) {
      const int64_t j = unstable[u];
      if (!compress(j, rows + ptr[j], rows + ptr[j + 1], out, work, tmp, t_adds[(size_t)t],
                    t_drops[(size_t)t])) {
        t_ok[(size_t)t] = 0;
        return;
      }
      ubeg[(size_t)u] = (int64_t)arena[(size_t)t].size();
      ulen[(size_t)u] = (int64_t)out.size();
      arena[(size_t)t].insert(arena[(size_t)t].end(), out.begin(), out.end());
    }
  };
  {
    std::vector<std::thread> pool;
    for (int t = 1; t < threads; ++t) pool.emplace_back(run, t);
    run(0);
    for (std::thread& th : pool) th.join();
  }
  for (int t = 0; t < threads; ++t) {
    if (!t_ok[(size_t)t]) return false;
    adds += t_adds[(size_t)t];
    drops += t_drops[(size_t)t];
  }
  // the compressed matrix: pivot and unstable columns, every other column zero
  std::vector<int64_t> len((size_t)n, 0);
  for (int64_t j = 0; j < n; ++j) len[(size_t)j] = slen[(size_t)j];
  for (int64_t u = 0; u < nun; ++u) len[(size_t)unstable[u]] = ulen[(size_t)u];
  cptr.assign((size_t)n + 1, 0);
  for (int64_t j = 0; j < n; ++j) cptr[(size_t)j + 1] = cptr[(size_t)j] + len[(size_t)j];
  crows.resize((size_t)cptr[(size_t)n]);
  for (int64_t j = 0; j < n; ++j)
    if (sbeg[(size_t)j] >= 0)
      std::copy(sarena.begin() + sbeg[(size_t)j], sarena.begin() + sbeg[(size_t)j] + slen[(size_t)j],
                crows.begin() + cptr[(size_t)j]);
  for (int t = 0; t < threads; ++t) {
    const int64_t u0 = nun * t / threads, u1 = nun * (t + 1) / threads;
    for (int64_t u = u0; u < u1; ++u)
      std::copy(arena[(size_t)t].begin() + ubeg[(size_t)u],
                arena[(size_t)t].begin() + ubeg[(size_t)u] + ulen[(size_t)u],
                crows.begin() + cptr[(size_t)unstable[u]]);
  }
  *additions += adds;
  *dropped += drops;
  return true;
}

void reduce_dimension(const HostComplex& H, int d, const Column* cols, int64_t ncols,
                      int threads, std::vector<PairRec>& pairs, std::vector<uint64_t>& deaths,
                      ReduceStats& stats, bool always_wide) {
  if (ncols == 0) return;
  // bits of the largest cofacet index C(n, d+2) - 1 and of the largest rank
  const uint64_t top = H.C(H.n, d + 2);
  const uint64_t largest = top ? top - 1 : 0;
  int cbits = 1, rbits = 1;
  while (cbits < 64 && (largest >> cbits)) ++cbits;
  while (rbits < 32 && ((uint64_t)(H.nranks ? H.nranks - 1 : 0) >> rbits)) ++rbits;
  const u128 cmax = cbits == 64 ? (u128)~0ull : (((u128)1 << cbits) - 1);
  if (rbits + cbits <= 64)
    reduce_keys<uint64_t>(H, Keys<uint64_t>{cbits, (uint64_t)cmax}, d, cols, ncols, threads,
                          pairs, deaths, stats, always_wide);
  else
    reduce_keys<u128>(H, Keys<u128>{cbits, cmax}, d, cols, ncols, threads, pairs, deaths, stats,
                      always_wide);
}

// Dense ranks of the finite weights: the finite upper-triangle entries are
// sorted by weight (a least-significant-digit radix sort on the 32-bit
// pattern, which orders non-negative floats), and equal weights share a rank.
void RankTable::build(int n, const uint32_t* W) {
  const size_t nn = (size_t)n * (size_t)n;
  tracked_n = 0;  // every entry is rewritten here
  bits.clear();
  // the n x n fill and the scan of the lower triangle run on several
  // threads for large clouds (row blocks; the edges are concatenated in row
  // order, as one thread would list them)
  const int nt = n >= 2048 ? (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency())) : 1;
  std::vector<std::vector<uint64_t>> part((size_t)nt);  // weight << 32 | position a*n + b
  Wr.resize(nn);
  auto scan = [&](int t) {
    const int a0 = (int)((int64_t)n * t / nt), a1 = (int)((int64_t)n * (t + 1) / nt);
    std::fill(Wr.begin() + (std::ptrdiff_t)((size_t)a0 * n), Wr.begin() + (std::ptrdiff_t)((size_t)a1 * n),
              kInf);
    for (int a = std::max(a0, 1); a < a1; ++a)
      for (int b = 0; b < a; ++b) {
        const uint32_t w = W[(size_t)a * n + b];
        if (w != kInf) part[(size_t)t].push_back(((uint64_t)w << 32) | (uint32_t)((size_t)a * n + b));
      }
  };
  {
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(scan, t);
    scan(0);
    for (std::thread& th : pool) th.join();
  }
  std::vector<uint64_t> e, tmp;
  size_t total = 0;
  for (const auto& v : part) total += v.size();
  e.reserve(total);
  for (const auto& v : part) e.insert(e.end(), v.begin(), v.end());
  tmp.resize(e.size());
  for (int shift = 32; shift < 64; shift += 11) {
    size_t cnt[2049] = {0};
    for (uint64_t x : e) ++cnt[((x >> shift) & 2047) + 1];
    bool trivial = false;
    for (int k = 1; k <= 2048; ++k)
      if (cnt[k] == e.size()) trivial = true;
    if (trivial) continue;
    for (int k = 1; k <= 2048; ++k) cnt[k] += cnt[k - 1];
    for (uint64_t x : e) tmp[cnt[(x >> shift) & 2047]++] = x;
    e.swap(tmp);
  }
  nbw = (n + 63) / 64;
  nb.assign((size_t)n * (size_t)nbw, 0);
  for (size_t k = 0; k < e.size(); ++k) {
    const uint32_t w = (uint32_t)(e[k] >> 32);
    if (bits.empty() || bits.back() != w) bits.push_back(w);
    const uint32_t pos = (uint32_t)e[k];
    const uint32_t a = pos / (uint32_t)n, b = pos % (uint32_t)n;
    Wr[(size_t)a * n + b] = Wr[(size_t)b * n + a] = (uint32_t)(bits.size() - 1);
    nb[(size_t)a * nbw + (b >> 6)] |= 1ull << (b & 63);
    nb[(size_t)b * nbw + (a >> 6)] |= 1ull << (a & 63);
  }
  sparse = (uint64_t)e.size() * 4 < (uint64_t)n * (uint64_t)(n - 1) / 2;
}

void RankTable::build_from_edges(int n, const Column* e, size_t m) {
  const size_t nn = (size_t)n * (size_t)n;
  if (tracked_n == n && Wr.size() == nn) {
    // undo the previous build's entries; every neighbour bit it set belongs
    // to one of them, so their words go back to zero whole
    for (uint64_t p : last) {
      const size_t a = (size_t)(p >> 32), b = (size_t)(uint32_t)p;
      Wr[a * n + b] = Wr[b * n + a] = kInf;
      nb[a * (size_t)nbw + (b >> 6)] = 0;
      nb[b * (size_t)nbw + (a >> 6)] = 0;
    }
  } else {
    Wr.resize(nn);
    const int nt = n >= 2048 ? (int)std::max(1u, std::min(16u, std::thread::hardware_concurrency())) : 1;
    auto fill = [&](int t) {
      const size_t r0 = (size_t)n * (size_t)t / (size_t)nt, r1 = (size_t)n * (size_t)(t + 1) / (size_t)nt;
      std::fill(Wr.begin() + (std::ptrdiff_t)(r0 * n), Wr.begin() + (std::ptrdiff_t)(r1 * n), kInf);
    };
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t) pool.emplace_back(fill, t);
    fill(0);
    for (std::thread& th : pool) th.join();
    nbw = (n + 63) / 64;
    nb.assign((size_t)n * (size_t)nbw, 0);
  }
  bits.clear();
  last.resize(m);
  for (size_t k = 0; k < m; ++k) {
    const uint32_t w = e[k].key_hi;
    if (bits.empty() || bits.back() != w) bits.push_back(w);
    const uint32_t r = (uint32_t)(bits.size() - 1);
    const size_t a = (size_t)(e[k].cidx >> 32), b = (size_t)(uint32_t)e[k].cidx;
    Wr[a * n + b] = Wr[b * n + a] = r;
    nb[a * (size_t)nbw + (b >> 6)] |= 1ull << (b & 63);
    nb[b * (size_t)nbw + (a >> 6)] |= 1ull << (a & 63);
    last[k] = e[k].cidx;
  }
  sparse = (uint64_t)m * 4 < (uint64_t)n * (uint64_t)(n - 1) / 2;
  tracked_n = n;
}

}  // namespace vrph
