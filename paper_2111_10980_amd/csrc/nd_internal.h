// Internal definitions shared by the library's HIP translation units.
// Device layout (all in HBM, all indices 0-based):
//   relabeled graph G'   rp[n+1] int64, col[2m] int32 (rows ascending),
//                        up[n] int64 = first position in row v holding a
//                        neighbour > v; the out-neighbours of v under the
//                        orientation are col[up[v] .. rp[v+1]).
//   r-clique table T     seg[n+1] uint64: the last-level table of first
//                        vertex v occupies slots [seg[v], seg[v+1]);
//                        slots[] 16-byte {key, cnt, stamp}; v1[] int32 per
//                        slot.  The slot position is the r-clique's index.
//                        Segments are hashed (open addressing), except for
//                        r = 3 plans of the s = r+1 path, where a root with
//                        an adjacency bitmap keeps its triangles in the rank
//                        order of the bitmap's bits (exactly full).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nd {

constexpr uint32_t kLive = 0xFFFFFFFFu;      // stamp of an unpeeled r-clique
constexpr uint64_t kOcc = 1ull << 63;        // key bit marking an occupied slot
constexpr int kWave = 64;
constexpr int kMaxS = 8;
constexpr int kMaxBitmapWords = 8;           // 8 x 64 = 512 out-neighbours per root

struct alignas(16) Slot {
  uint64_t key;    // kOcc | low 63 bits of the packed (v2, v3, ...); 0 = empty
  uint32_t cnt;    // s-clique count, decremented while peeling
  uint32_t stamp;  // round in which the r-clique was peeled, or kLive
};
static_assert(sizeof(Slot) == 16, "slot must be 16 bytes");

struct GraphView {
  int32_t n;
  const int64_t *__restrict__ rp;
  const int32_t *__restrict__ col;
  const int64_t *__restrict__ up;
};

struct TableView {
  int bits;                            // bits per vertex field of a key
  const uint64_t *__restrict__ seg;    // n+1
  Slot *__restrict__ slots;
  int32_t *__restrict__ v1;            // first vertex of each occupied slot
  uint64_t *__restrict__ khi;          // second key word per slot, or null (keys fit 63 bits)
  // Three levels (aseg non-null; Section 4.1, l = 3): the middle level is
  // v1's out-row of the oriented CSR, searched for v2; the arc at position e
  // owns the last-level table [aseg[e], aseg[e+1]), keyed by v3..vr.
  const uint64_t *__restrict__ aseg;   // per arc position (2m+1), or null: two levels
  int32_t *__restrict__ v2;            // second vertex of each occupied slot (three levels)
  GraphView arcs;                      // the oriented CSR (three levels)
};

// Key of a sorted r-tuple (v1 < ... < vR) within its last-level table: the
// fields v2..vR (two levels) or v3..vR (three levels), `bits` each, packed
// from bit 0 up into at most 126 bits.  Its low 63 bits plus the occupied bit
// form the slot's key word; its high 63 bits are the second word, zero
// unless the fields need more than 63 bits (then the table keeps them in
// TableView::khi).
struct Key {
  uint64_t lo, hi;
};

// Device-side error flags (bit set in a device word, read by the host).
enum : uint32_t {
  kErrGraph = 1u,
  kErrLookup = 2u,
  kErrOverflow = 4u,
  kErrTable = 8u,
  kErrBucket = 16u,  // a level advance found no live r-clique, or an empty bucket
  kErrRuntime = 32u, // host side: a HIP call of the peel loop failed
  kErrCapacity = 64u, // host side: a round needs more records or trace than the workspace holds
};

// ----------------------------------------------------------------- helpers

// splitmix64 output mixer (Steele, Lea, Flood, "Fast splittable pseudorandom
// number generators", OOPSLA 2014): a bijective 64-bit finaliser.
__device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x ^= x >> 30;
  x *= 0xbf58476d1ce4e5b9ull;
  x ^= x >> 27;
  x *= 0x94d049bb133111ebull;
  x ^= x >> 31;
  return x;
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t lanes_below() {
  return (1ull << lane_id()) - 1ull;
}

// true if x occurs in the sorted range a[lo, hi)
__device__ __forceinline__ bool sorted_contains(const int32_t *__restrict__ a, int64_t lo,
                                                int64_t hi, int32_t x) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    int32_t v = a[mid];
    if (v == x) return true;
    if (v < x) lo = mid + 1;
    else hi = mid;
  }
  return false;
}

// Edge test through the orientation: the lower-ranked endpoint's
// out-neighbour list is short (bounded by the orientation's out-degree).
__device__ __forceinline__ bool adjacent(const GraphView &g, int32_t x, int32_t y) {
  int32_t a = x < y ? x : y;
  int32_t b = x < y ? y : x;
  if (a == b) return false;
  return sorted_contains(g.col, g.up[a], g.rp[a + 1], b);
}

// Position of the arc between x and y in the lower-ranked endpoint's
// out-neighbour list, or -1 when they are not adjacent.
__device__ __forceinline__ int64_t arc_pos(const GraphView &g, int32_t x, int32_t y) {
  const int32_t a = x < y ? x : y;
  const int32_t b = x < y ? y : x;
  if (a == b) return -1;
  int64_t lo = g.up[a], hi = g.rp[a + 1];
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int32_t v = g.col[mid];
    if (v == b) return mid;
    if (v < b) lo = mid + 1;
    else hi = mid;
  }
  return -1;
}

// first: index of the first key field (1: two levels, 2: three levels, R >= 4)
template <int R>
__device__ __forceinline__ Key make_key(const int32_t *v, int bits, int first = 1) {
  uint64_t lo = 0, hi = 0;
  if constexpr (R <= 3) {  // at most two fields of <= 31 bits: one word
#pragma unroll
    for (int i = 1; i < R; i++) lo |= (uint64_t)(uint32_t)v[i] << (bits * (i - 1));
    return Key{lo | kOcc, 0ull};
  }
#pragma unroll
  for (int i = 1; i < R; i++) {
    if (i < first) continue;
    const int o = bits * (i - first);
    const uint64_t f = (uint32_t)v[i];
    if (o < 63) {
      lo |= f << o;
      if (o + bits > 63) hi |= f >> (63 - o);  // the field straddles the two words
    } else {
      hi |= f << (o - 63);
    }
  }
  return Key{(lo & (kOcc - 1)) | kOcc, hi};
}

__device__ __forceinline__ int key_first(const TableView &T) { return T.aseg ? 2 : 1; }

// The key of a sorted r-tuple in table T.
template <int R>
__device__ __forceinline__ Key rkey(const TableView &T, const int32_t *v) {
  return make_key<R>(v, T.bits, R >= 4 ? key_first(T) : 1);
}

// v2..vR of the r-clique in slot p (v[0] is the caller's).
template <int R>
__device__ __forceinline__ void decode_key(const TableView &T, uint64_t p, uint64_t key_lo,
                                           int32_t *v) {
  const int bits = T.bits;  // <= 31
  const uint64_t mask = (1ull << bits) - 1ull;
  if constexpr (R <= 3) {  // one word
#pragma unroll
    for (int i = 1; i < R; i++) v[i] = (int32_t)((key_lo >> (bits * (i - 1))) & mask);
    return;
  }
  const uint64_t lo = key_lo & (kOcc - 1);
  const uint64_t hi = T.khi ? T.khi[p] : 0ull;
  const int first = key_first(T);
  if (first == 2) v[1] = T.v2[p];
#pragma unroll
  for (int i = 1; i < R; i++) {
    if (i < first) continue;
    const int o = bits * (i - first);
    uint64_t f;
    if (o >= 63) {
      f = hi >> (o - 63);
    } else {
      f = lo >> o;
      if (o + bits > 63) f |= hi << (63 - o);
    }
    v[i] = (int32_t)(f & mask);
  }
}

__device__ __forceinline__ uint64_t home_slot(const Key &key, uint64_t cap) {
  // fastrange: maps the high 32 hash bits onto [0, cap) without a division
  return ((mix64(key.lo ^ (key.hi * 0x9E3779B97F4A7C15ull)) >> 32) * cap) >> 32;
}

// Does slot i (whose key word is `lo`) hold `key`?  The second word is
// tested at run time for every r: compiled out for r < 4, the listing
// kernels of the count phase took 16 more registers per lane (the probe
// loops were laid out differently) and spilled at 8 bitmap words.
template <bool kR4>
__device__ __forceinline__ bool key_eq(const TableView &T, uint64_t i, uint64_t lo,
                                       const Key &key) {
  return lo == key.lo && (!T.khi || T.khi[i] == key.hi);
}

// The last-level table of an r-clique with first vertices v1 < v2:
// [base, base + cap).  cap = 0 when there is none (no such r-clique).
// kR4 = false: the caller's r is below 4, so its table has two levels and
// one-word keys, and the code for the others is compiled out.
template <bool kR4>
__device__ __forceinline__ void last_level(const TableView &T, int32_t v1, int32_t v2,
                                           uint64_t &base, uint64_t &cap) {
  if (!kR4 || !T.aseg) {
    base = T.seg[v1];
    cap = T.seg[v1 + 1] - base;
    return;
  }
  const int64_t e = arc_pos(T.arcs, v1, v2);
  base = e >= 0 ? T.aseg[e] : 0;
  cap = e >= 0 ? T.aseg[e + 1] - base : 0;
}

// Positions of N arcs (a[q] < b[q]) in the rows of a[q], searched in
// lock-step so their loads overlap; -1 when absent or not wanted.
template <int N>
__device__ __forceinline__ void arc_pos_n(const GraphView &g, const int32_t (&a)[N],
                                          const int32_t (&b)[N], const bool (&want)[N],
                                          int64_t (&e)[N]) {
  int64_t base[N], len[N];
#pragma unroll
  for (int q = 0; q < N; q++) {
    base[q] = want[q] ? g.up[a[q]] : 0;
    len[q] = want[q] ? g.rp[a[q] + 1] - base[q] : 0;
  }
  // invariant: b[q], when present, lies in [base, base + len)
  bool more = true;
  while (more) {
    more = false;
#pragma unroll
    for (int q = 0; q < N; q++) {
      if (len[q] > 1) {
        const int64_t half = len[q] >> 1;
        if (g.col[base[q] + half] <= b[q]) base[q] += half;
        len[q] -= half;
        more = more || len[q] > 1;
      }
    }
  }
#pragma unroll
  for (int q = 0; q < N; q++) e[q] = len[q] == 1 && g.col[base[q]] == b[q] ? base[q] : -1;
}

// Linear probe of the last-level table of the r-clique starting v1 < v2.
// Returns the slot index, or -1 when absent; *out receives the slot.
template <bool kR4>
__device__ __forceinline__ int64_t table_find(const TableView &T, int32_t v1, int32_t v2,
                                              const Key &key, Slot *out) {
  uint64_t base, cap;
  last_level<kR4>(T, v1, v2, base, cap);
  if (cap == 0) return -1;
  uint64_t i = home_slot(key, cap);
  for (uint64_t probe = 0; probe < cap; probe++) {
    Slot s = T.slots[base + i];
    if (key_eq<kR4>(T, base + i, s.key, key)) {
      *out = s;
      return (int64_t)(base + i);
    }
    if (s.key == 0) return -1;
    if (++i == cap) i = 0;
  }
  return -1;
}

// Every r-clique is inserted once (the listing meets each exactly once), so
// claiming an empty slot is enough.  With two-word keys a slot whose first
// word equals this key's holds another r-clique (or one whose second word is
// still being written): probing goes on.
template <bool kR4>
__device__ __forceinline__ int64_t table_insert(const TableView &T, int32_t v1, int32_t v2,
                                               const Key &key) {
  uint64_t base, cap;
  last_level<kR4>(T, v1, v2, base, cap);
  if (cap == 0) return -1;
  uint64_t i = home_slot(key, cap);
  for (uint64_t probe = 0; probe < cap; probe++) {
    unsigned long long *kp = (unsigned long long *)&T.slots[base + i].key;
    unsigned long long prev = atomicCAS(kp, 0ull, (unsigned long long)key.lo);
    const bool wide = kR4 && T.khi;
    if (prev == 0ull || (prev == key.lo && !wide)) {
      if (wide) T.khi[base + i] = key.hi;
      if (kR4 && T.v2) T.v2[base + i] = v2;
      T.v1[base + i] = v1;
      return (int64_t)(base + i);
    }
    if (++i == cap) i = 0;
  }
  return -1;
}

// K lower bounds in the same sorted range, advanced in lock-step so their
// loads are independent (one dependent step per halving, not K).
template <int K>
__device__ __forceinline__ void lower_bounds(const int32_t *__restrict__ a, int64_t lo0, int64_t hi0,
                                             const int32_t (&y)[K], int64_t (&out)[K]) {
  int64_t base[K], n = hi0 - lo0;
#pragma unroll
  for (int q = 0; q < K; q++) base[q] = lo0;
  if (n <= 0) {
#pragma unroll
    for (int q = 0; q < K; q++) out[q] = lo0;
    return;
  }
  // invariant: the answer lies in [base, base + n]; every read index is
  // base + half < base + n <= hi0
  while (n > 1) {
    const int64_t half = n >> 1;
#pragma unroll
    for (int q = 0; q < K; q++) base[q] = a[base[q] + half] < y[q] ? base[q] + half : base[q];
    n -= half;
  }
#pragma unroll
  for (int q = 0; q < K; q++) out[q] = base[q] + (a[base[q]] < y[q] ? 1 : 0);
}

// N independent table lookups issued together: the home slots of all keys
// are loaded before any collision chain is followed.  want[q] = false skips
// lookup q (pos[q] = -1).
template <int N, bool kR4>
__device__ __forceinline__ void table_find_n(const TableView &T, const int32_t (&v1)[N],
                                             const int32_t (&v2)[N], const Key (&key)[N],
                                             const bool (&want)[N], int64_t (&pos)[N],
                                             Slot (&out)[N]) {
  uint64_t base[N], cap[N], i[N];
  int64_t e[N];
  const bool arcs = kR4 && T.aseg;
  if (arcs) arc_pos_n<N>(T.arcs, v1, v2, want, e);
#pragma unroll
  for (int q = 0; q < N; q++) {
    pos[q] = -1;
    base[q] = 0;
    cap[q] = 0;
    i[q] = 0;
    if (want[q]) {
      if (arcs) {
        base[q] = e[q] >= 0 ? T.aseg[e[q]] : 0;
        cap[q] = e[q] >= 0 ? T.aseg[e[q] + 1] - base[q] : 0;
      } else {
        base[q] = T.seg[v1[q]];
        cap[q] = T.seg[v1[q] + 1] - base[q];
      }
      if (cap[q]) i[q] = home_slot(key[q], cap[q]);
    }
  }
#pragma unroll
  for (int q = 0; q < N; q++)
    if (want[q] && cap[q]) out[q] = T.slots[base[q] + i[q]];
#pragma unroll
  for (int q = 0; q < N; q++) {
    if (!want[q] || !cap[q]) continue;
    for (uint64_t probe = 0; probe < cap[q]; probe++) {
      if (key_eq<kR4>(T, base[q] + i[q], out[q].key, key[q])) {
        pos[q] = (int64_t)(base[q] + i[q]);
        break;
      }
      if (out[q].key == 0) break;
      if (++i[q] == cap[q]) i[q] = 0;
      out[q] = T.slots[base[q] + i[q]];
    }
  }
}

// Wave-aggregated append: every active lane calls it; lanes with want=true
// get consecutive positions in buf reserved with one atomic per wave.
__device__ __forceinline__ void wave_append(bool want, uint32_t val, uint32_t *buf,
                                            uint32_t *counter) {
  uint64_t m = __ballot(want);
  if (m == 0) return;
  int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomicAdd(counter, (uint32_t)__popcll(m));
  base = __shfl(base, leader);
  if (want) buf[base + (uint32_t)__popcll(m & lanes_below())] = val;
}

// Per-wave staging of appends in LDS.  One wave owns `buf` (kCap entries);
// `count` is wave-uniform.  Entries are flushed to the global list with a
// single atomic when fewer than 64 free entries remain, so a round with
// A appended r-cliques costs about A / (kCap - 64) global atomics instead of
// one per appending wave call (same-address atomics serialise across XCDs).
struct NoFlushHook {
  __device__ __forceinline__ void operator()(uint32_t) const {}
};

template <int kCap, class Hook = NoFlushHook>
struct WaveAppender {
  uint32_t *buf;   // LDS, kCap entries, private to this wave
  uint32_t count;  // wave-uniform
  uint32_t *out;
  uint32_t *counter;
  Hook hook;       // called once per value as it is written out

  __device__ __forceinline__ void flush() {
    if (count == 0) return;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    uint32_t base = 0;
    if (lane_id() == 0) base = atomicAdd(counter, count);
    base = __shfl(base, 0);
    for (uint32_t i = (uint32_t)lane_id(); i < count; i += kWave) {
      const uint32_t v = buf[i];
      out[base + i] = v;
      hook(v);
    }
    __builtin_amdgcn_wave_barrier();
    count = 0;
  }
  // every lane of the wave calls this together
  __device__ __forceinline__ void push(bool want, uint32_t val) {
    const uint64_t m = __ballot(want);
    if (m == 0) return;
    if (want) buf[count + (uint32_t)__popcll(m & lanes_below())] = val;
    count += (uint32_t)__popcll(m);
    if (count > (uint32_t)(kCap - kWave)) flush();
  }
};

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    uint32_t o = __shfl_xor(v, off);
    v = o < v ? o : v;
  }
  return v;
}

// Inclusive prefix sum across the wave.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  int lane = lane_id();
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t o = __shfl_up(v, off);
    if (lane >= off) v += o;
  }
  return v;
}

// ---------------------------------------------------- r-subsets of s-sets

constexpr int binom(int n, int k) {
  if (k < 0 || k > n) return 0;
  int r = 1;
  for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
  return r;
}

// All R-subsets of {0..S-1}, lexicographic, as bit masks.
template <int S, int R>
struct Combos {
  static constexpr int N = binom(S, R);
  uint8_t mask[N > 0 ? N : 1];
  uint8_t idx[N > 0 ? N : 1][R > 0 ? R : 1];
  constexpr Combos() : mask{}, idx{} {
    int c[R > 0 ? R : 1] = {};
    for (int i = 0; i < R; i++) c[i] = i;
    for (int q = 0; q < N; q++) {
      uint8_t m = 0;
      for (int i = 0; i < R; i++) {
        idx[q][i] = (uint8_t)c[i];
        m = (uint8_t)(m | (1u << c[i]));
      }
      mask[q] = m;
      int i = R - 1;
      while (i >= 0 && c[i] == S - R + i) i--;
      if (i < 0) break;
      c[i]++;
      for (int j = i + 1; j < R; j++) c[j] = c[j - 1] + 1;
    }
  }
};

// ------------------------------------------------------- host-side launch

struct Counters {
  uint64_t n_s;          // s-cliques listed by the count phase
  uint64_t decrements;
  uint64_t discoveries;
  uint64_t atomics;      // returning atomic decrements issued (subset of decrements)
  uint32_t err;          // kErr* bits
  uint32_t next_size;    // appends to the next frontier in this round
  uint32_t class_size[8];
  uint32_t low_size;     // size of the level-window list (appends continue after it)
};



// Device-resident state of the peel loop (Algorithm 2's bucket structure B,
// the level k, the round number and the frontier).  Small control kernels
// advance it and every round kernel reads its parameters from it, so the
// host can queue rounds back to back and only read it now and then.
constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kWindowLevels = 16;      // first window: levels k+1..k+16
constexpr uint32_t kMaxWindowLevels = 1u << 16;

// Top of a window opened at level k with wl levels (clamped below the
// largest count the partition can test).
__host__ __device__ inline uint32_t window_top(uint32_t k, uint32_t wl) {
  const uint64_t t = (uint64_t)k + wl;
  return t < 0xFFFFFFFEull ? (uint32_t)t : 0xFFFFFFFEu;
}

struct RoundCtl {
  // parameters of the current round, set by k_round_begin
  const uint32_t *F;   // frontier A_t
  uint32_t *Fnext;     // r-cliques whose count reaches k (next frontier)
  uint32_t *Low;       // r-cliques whose count enters the window (k, kw]
  // list storage: two buffers each, the live one picked by sel*
  uint32_t *bufF[2], *bufW[2], *bufH[2];
  uint32_t *trace_size;  // per round: |A_t|
  uint32_t *trace_k;     // per round: k
  uint64_t n_r, finished;
  uint64_t total, cap;     // record slots allocated this round / capacity
  uint64_t total2;         // second record list (member records)
  uint64_t total3, cap3;   // third list (out-arcs of members) / capacity
  uint64_t need;           // capacity asked for when a round halted (halt 1: total, 4: total3)
  uint64_t max_total, max_total3;  // largest record / out-arc totals of a finished round
  uint64_t contract_every;  // r = 2 graph contraction: peeled edges between contractions (0 off)
  uint64_t peeled_since;    // edges peeled since the last contraction
  uint32_t contract_due;    // set when peeled_since reaches contract_every
  uint32_t contractions;    // contraction passes done
  uint32_t t, k, kw, nF;   // round, level, window top, |A_t|
  uint32_t wlev;           // levels the next window opened from the high list spans
  uint64_t wscan;          // window-list entries scanned by advances inside the current window
  uint32_t nA;             // |A_t| of the round under way (set by begin, kept by end)
  uint32_t nW, nH;         // window list and high list sizes
  uint32_t selF, selW, selH;
  uint32_t done;           // every r-clique peeled
  uint32_t halt;           // 1: records, 2: trace, 4: arcs; kernels skip until cleared
  uint32_t err;            // kErr* bits
  uint32_t mw, mh;         // live minima of the window / high list (advance)
  uint32_t cF, cW, cH;     // partition output sizes (advance)
  uint32_t advances;
  uint32_t trace_cap;
  uint32_t ndone;          // blocks of the advance kernel finished (the last one resets it)
};

// Statistics accumulated by many waves go to kStatLines counter lines (one
// 128-byte line each, picked by block index) and are summed once at the
// end: a single global counter hit by every wave serialises in one L2
// channel across all XCDs.
constexpr int kStatLines = 1024;
constexpr int kStatStride = 16;  // u64 per line
enum : int { kStatDec = 0, kStatDisc = 1, kStatNs = 2, kStatAtom = 3 };

__device__ __forceinline__ void stat_add(unsigned long long *stats, int which, uint64_t v) {
  const uint64_t t = wave_sum_u64(v);
  if (lane_id() == 0 && t)
    atomicAdd(&stats[(blockIdx.x & (kStatLines - 1)) * kStatStride + which],
              (unsigned long long)t);
}

}  // namespace nd
