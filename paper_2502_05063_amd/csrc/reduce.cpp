// Host submatrix reduction (Sec. 5.2.9, 5.5.1) over the columns the GPU
// found non-apparent. Columns of the dimension-d coboundary matrix are
// d-simplices in coboundary order (diameter descending, index ascending);
// rows are (d+1)-simplices in the same order. A row is represented by a
// 128-bit key (~diameter, index): increasing key = increasing row index, so
// the lowest nonzero of a column (its pivot, the oldest cofacet) is the
// largest key.
#include "reduce.h"

#include <algorithm>
#include <atomic>
#include <thread>
#include <unordered_map>

namespace vrph {

using u128 = unsigned __int128;

// Row keys. A diameter is a non-negative float, so its bit pattern has a
// zero sign bit and fits in 31 bits; when 31 + (bits of the largest cofacet
// index) <= 64 the key is a u64 ((2^31-1 - diameter) above the index),
// otherwise a u128 with the diameter in the high word.
template <class K>
struct Keys;

template <>
struct Keys<uint64_t> {
  int cbits;
  uint64_t make(uint32_t diam, uint64_t c) const {
    return ((uint64_t)(0x7FFFFFFFu - diam) << cbits) | c;
  }
  uint64_t index(uint64_t k) const { return k & ((cbits == 64) ? ~0ull : ((1ull << cbits) - 1)); }
  uint32_t diam(uint64_t k) const { return 0x7FFFFFFFu - (uint32_t)(k >> cbits); }
  static int high_bit(uint64_t x) { return 63 - __builtin_clzll(x); }
  static constexpr int kBits = 64;
};

template <>
struct Keys<u128> {
  int cbits;
  u128 make(uint32_t diam, uint64_t c) const { return ((u128)(uint32_t)~diam << 64) | (u128)c; }
  uint64_t index(u128 k) const { return (uint64_t)k; }
  uint32_t diam(u128 k) const { return ~(uint32_t)(k >> 64); }
  static int high_bit(u128 x) {
    const uint64_t hi = (uint64_t)(x >> 64), lo = (uint64_t)x;
    return hi ? 127 - __builtin_clzll(hi) : 63 - __builtin_clzll(lo);
  }
  static constexpr int kBits = 128;
};

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

static uint32_t diameter_of(const HostComplex& H, const int* v, int d) {
  uint32_t m = 0;
  for (int i = 1; i <= d; ++i)
    for (int j = 0; j < i; ++j) m = std::max(m, H.w(v[i], v[j]));
  return m;
}

void diameter_edge(const HostComplex& H, uint64_t c, int d, int32_t* u, int32_t* w) {
  int v[kMaxDim + 3];
  decode_simplex(H, c, d, v);
  uint32_t dm = diameter_of(H, v, d);
  uint64_t best = 0;
  bool have = false;
  for (int i = 1; i <= d; ++i)
    for (int j = 0; j < i; ++j)
      if (H.w(v[i], v[j]) == dm) {
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

// max over the vertices of s of W(v_i, x); kInf if some edge is above tau_eff
static inline uint32_t reach(const HostComplex& H, const int* v, int d, int x) {
  uint32_t m = 0;
  for (int i = 0; i <= d; ++i) m = std::max(m, H.w(v[i], x));
  return m;
}

static inline bool contains(const int* v, int d, int x) {
  for (int i = 0; i <= d; ++i)
    if (v[i] == x) return true;
  return false;
}

// low(D_s): the oldest cofacet = smallest diameter, then largest index. The
// first x from the top whose cofacet keeps the diameter is it; otherwise the
// largest key over all cofacets.
template <class K>
static bool oldest_cofacet(const HostComplex& H, const Keys<K>& ks, const int* v, int d,
                           uint32_t diam, K* low) {
  bool found = false;
  for (int x = H.n - 1; x >= 0; --x) {
    if (contains(v, d, x)) continue;
    uint32_t m = reach(H, v, d, x);
    if (m == kInf) continue;
    K k = ks.make(std::max(diam, m), cofacet_index(H, v, d, x));
    if (!found || k > *low) *low = k;
    found = true;
    if (m <= diam) break;
  }
  return found;
}

// If row t (a (d+1)-simplex) is the cofacet of an apparent pair (s, t),
// return s. Def. 5.3.4: s is the youngest facet of t (largest diameter, then
// smallest index: remove the largest vertex u whose removal keeps diam(t)),
// and t is the oldest cofacet of s (no x > u outside s keeps the diameter).
static bool apparent_partner(const HostComplex& H, uint64_t t, uint32_t dt, int d, uint64_t* s,
                             int* sv) {
  int tv[kMaxDim + 3];
  decode_simplex(H, t, d + 1, tv);
  int drop = -1;
  for (int r = d + 1; r >= 0; --r) {  // vertices from the largest down
    uint32_t m = 0;
    for (int i = 1; i <= d + 1; ++i)
      for (int j = 0; j < i; ++j)
        if (i != r && j != r) m = std::max(m, H.w(tv[i], tv[j]));
    if (m == dt) {
      drop = r;
      break;
    }
  }
  if (drop < 0) return false;
  int k = 0;
  for (int i = 0; i <= d + 1; ++i)
    if (i != drop) sv[k++] = tv[i];
  const int u = tv[drop];
  for (int x = H.n - 1; x > u; --x) {
    if (contains(sv, d, x)) continue;
    if (reach(H, sv, d, x) <= dt) return false;
  }
  uint64_t c = 0;
  for (int i = 0; i <= d; ++i) c += H.C(sv[i], i + 1);
  *s = c;
  return true;
}

// A column in the pivot store: its simplex and, for a column reduced here,
// the other columns whose sum with it is its reduced column (the V column of
// the reduction-matrix technique, R = D V, Sec. 5.2.9). Apparent columns and
// columns paired at their first pivot need no additions: their reduced column
// is their coboundary (v = -1).
struct Partner {
  uint64_t c;
  uint32_t diam;
  int32_t v;  // index into the stored V columns, -1 for none
};

struct Simplex {
  uint64_t c;
  uint32_t diam;
  bool operator<(const Simplex& o) const { return c < o.c; }
  bool operator==(const Simplex& o) const { return c == o.c; }
};

// The working column: a monotone max-priority queue of row keys (a radix
// heap). Every key pushed is <= the current pivot and pivots only decrease,
// so a key lives in the bucket of the highest bit where it differs from the
// last extracted maximum; bucket 0 holds copies of that maximum, and since
// equal keys cancel in pairs over Z/2 the maximum survives iff bucket 0 has
// odd size.
template <class K>
class WorkColumn {
 public:
  void clear() {
    for (auto& b : b_) b.clear();
    last_ = ~(K)0;
  }
  void push(K k) { b_[bucket(k)].push_back(k); }
  // the pivot (largest key of odd multiplicity), kept; false if zero
  bool pivot(K* k) {
    for (;;) {
      if (b_[0].empty() && !refill()) return false;
      if (b_[0].size() & 1) {
        b_[0].resize(1);
        *k = last_;
        return true;
      }
      b_[0].clear();
    }
  }

 private:
  int bucket(K k) const { return k == last_ ? 0 : Keys<K>::high_bit(k ^ last_) + 1; }
  bool refill() {
    int i = 1;
    while (i <= Keys<K>::kBits && b_[i].empty()) ++i;
    if (i > Keys<K>::kBits) return false;
    std::vector<K>& src = b_[i];
    K m = src[0];
    for (K x : src) m = x > m ? x : m;
    last_ = m;
    std::vector<K> moved;
    moved.swap(src);
    for (K x : moved) b_[bucket(x)].push_back(x);
    moved.clear();
    moved.swap(src);  // keep the capacity
    return true;
  }
  std::vector<K> b_[Keys<K>::kBits + 1];
  K last_ = ~(K)0;
};

// Push the cofacets of one column with row key <= limit. Used to add a
// reduced column R_k whose pivot is `limit`: R_k is zero below its pivot, so
// the parts of its summands below the pivot cancel and are not pushed.
// Cofacets s + {x} come in decreasing index order as x goes down (Alg. 14);
// the index is kept incrementally: vertices of s above x contribute
// C(v_i, i+2) (they moved up one position), those below C(v_i, i+1), and x
// itself C(x, j+1) with j the number of vertices below it.
template <class K>
static void push_coboundary(const HostComplex& H, const Keys<K>& ks, uint64_t c, uint32_t diam,
                            int d, K limit, WorkColumn<K>& w, uint32_t* reach_buf) {
  int v[kMaxDim + 3];
  decode_simplex(H, c, d, v);
  // reach_buf[x] = max_i W(v_i, x): elementwise max of d+1 weight rows
  const size_t n = (size_t)H.n;
  const uint32_t* r0 = H.W + (size_t)v[0] * n;
  for (size_t x = 0; x < n; ++x) reach_buf[x] = r0[x];
  for (int i = 1; i <= d; ++i) {
    const uint32_t* ri = H.W + (size_t)v[i] * n;
    for (size_t x = 0; x < n; ++x) reach_buf[x] = std::max(reach_buf[x], ri[x]);
  }
  uint64_t high = 0, low = c;
  int pos = d;  // vertices v[pos+1..d] are above x
  for (int x = H.n - 1; x >= 0; --x) {
    if (pos >= 0 && x == v[pos]) {
      high += H.C(v[pos], pos + 2);
      low -= H.C(v[pos], pos + 1);
      --pos;
      continue;
    }
    const uint32_t m = reach_buf[x];
    if (m == kInf) continue;
    const K k = ks.make(std::max(diam, m), high + H.C(x, pos + 2) + low);
    if (k <= limit) w.push(k);
  }
}

// What a column needs before the sequential pass, independent of every other
// column: its first pivot low(D_j) and, if that row is the cofacet of an
// apparent pair, the apparent column.
template <class K>
struct FirstPivot {
  K low;
  uint64_t apparent;  // the apparent column owning `low`, if has_apparent
  bool nonzero;
  bool has_apparent;
};

template <class K>
static void first_pivots(const HostComplex& H, const Keys<K>& ks, int d, const Column* cols,
                         int64_t ncols, int threads, std::vector<FirstPivot<K>>& out) {
  out.resize((size_t)ncols);
  std::atomic<int64_t> next{0};
  auto work = [&]() {
    int v[kMaxDim + 3], sv[kMaxDim + 3];
    for (;;) {
      const int64_t j0 = next.fetch_add(256);
      if (j0 >= ncols) return;
      const int64_t j1 = std::min<int64_t>(ncols, j0 + 256);
      for (int64_t j = j0; j < j1; ++j) {
        FirstPivot<K>& f = out[(size_t)j];
        decode_simplex(H, cols[j].cidx, d, v);
        f.nonzero = oldest_cofacet(H, ks, v, d, ~cols[j].key_hi, &f.low);
        f.has_apparent =
            f.nonzero && apparent_partner(H, ks.index(f.low), ks.diam(f.low), d, &f.apparent, sv);
      }
    }
  };
  threads = (int)std::max<int64_t>(1, std::min<int64_t>(threads, ncols / 1024));
  std::vector<std::thread> pool;
  for (int i = 1; i < threads; ++i) pool.emplace_back(work);
  work();
  for (std::thread& t : pool) t.join();
}

template <class K>
static void reduce_keys(const HostComplex& H, const Keys<K>& ks, int d, const Column* cols,
                        int64_t ncols, int threads, std::vector<PairRec>& pairs,
                        std::vector<uint64_t>& deaths, ReduceStats& stats) {
  std::unordered_map<uint64_t, Partner> pivots;  // row index -> column, this dimension
  pivots.reserve((size_t)ncols * 2 + 16);
  std::vector<std::vector<Simplex>> vstore;       // V columns of the reduced columns
  WorkColumn<K> work;
  std::vector<Simplex> vj;
  std::vector<uint32_t> reach_buf((size_t)H.n);
  int pv[kMaxDim + 3];
  std::vector<FirstPivot<K>> first;
  first_pivots(H, ks, d, cols, ncols, threads, first);

  // two-layer lookup (Fig. 5.10): pairs found by this reduction first, then
  // the apparent pairs, recognised from Def. 5.3.4 instead of a stored array
  auto lookup = [&](K row, Partner* p) -> bool {
    auto it = pivots.find(ks.index(row));
    if (it != pivots.end()) {
      *p = it->second;
      return true;
    }
    uint64_t s;
    if (apparent_partner(H, ks.index(row), ks.diam(row), d, &s, pv)) {
      *p = Partner{s, ks.diam(row), -1};
      return true;
    }
    return false;
  };

  for (int64_t j = 0; j < ncols; ++j) {
    const uint64_t c = cols[j].cidx;
    const uint32_t diam = ~cols[j].key_hi;
    const FirstPivot<K>& f = first[(size_t)j];
    K low = f.low;
    Partner p;
    bool nonzero = f.nonzero;
    bool taken = false;
    if (nonzero) {
      if (f.has_apparent) {
        p = Partner{f.apparent, ks.diam(low), -1};
        taken = true;
      } else {
        auto it = pivots.find(ks.index(low));
        if (it != pivots.end()) {
          p = it->second;
          taken = true;
        }
      }
    }
    vj.clear();
    if (taken) {
      // Alg. 2 on column j: while its pivot is the pivot of an earlier column
      // k, add R_k = D_k + sum_{i in V_k} D_i (the pivot then moves up)
      work.clear();
      push_coboundary(H, ks, c, diam, d, low, work, reach_buf.data());
      for (;;) {
        push_coboundary(H, ks, p.c, p.diam, d, low, work, reach_buf.data());
        vj.push_back(Simplex{p.c, p.diam});
        if (p.v >= 0)
          for (const Simplex& q : vstore[p.v]) {
            push_coboundary(H, ks, q.c, q.diam, d, low, work, reach_buf.data());
            vj.push_back(q);
          }
        ++stats.additions;
        if (!work.pivot(&low)) {
          nonzero = false;
          break;
        }
        if (!lookup(low, &p)) break;
      }
    } else if (nonzero) {
      ++stats.emergent;
    }
    if (nonzero) {
      int32_t vi = -1;
      if (!vj.empty()) {
        // V over Z/2: a column added twice cancels
        std::sort(vj.begin(), vj.end());
        std::vector<Simplex> red;
        for (size_t a = 0; a < vj.size();) {
          size_t b = a;
          while (b < vj.size() && vj[b] == vj[a]) ++b;
          if ((b - a) & 1) red.push_back(vj[a]);
          a = b;
        }
        vi = (int32_t)vstore.size();
        vstore.push_back(std::move(red));
      }
      pivots.emplace(ks.index(low), Partner{c, diam, vi});
      pairs.push_back(PairRec{c, ks.index(low), diam, ks.diam(low)});
      deaths.push_back(ks.index(low));
    } else {
      pairs.push_back(PairRec{c, ~0ull, diam, kInf});
    }
  }
}

void reduce_dimension(const HostComplex& H, int d, const Column* cols, int64_t ncols,
                      int threads, std::vector<PairRec>& pairs, std::vector<uint64_t>& deaths,
                      ReduceStats& stats) {
  // bits of the largest cofacet index, C(n, d+2) - 1
  const uint64_t top = H.C(H.n, d + 2);
  const uint64_t largest = top ? top - 1 : 0;
  int cbits = 1;
  while (cbits < 64 && (largest >> cbits)) ++cbits;
  if (31 + cbits <= 64)
    reduce_keys<uint64_t>(H, Keys<uint64_t>{cbits}, d, cols, ncols, threads, pairs, deaths,
                          stats);
  else
    reduce_keys<u128>(H, Keys<u128>{64}, d, cols, ncols, threads, pairs, deaths, stats);
}

}  // namespace vrph
