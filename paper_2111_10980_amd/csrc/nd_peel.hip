// Bucketing and peeling (paper Algorithm 2 main loop, Update, Update-Func;
// Section 2 "Parallel Bucketing"; Section 4.5 "Obtaining the Set of
// Updated r-cliques").
//
// Round t at level k peels the frontier A_t (every live r-clique whose count
// is <= k).  Before the round's peel kernel runs, every member of A_t is
// stamped with t, so inside the kernel a stamp answers Update-Func's two
// questions exactly: stamp < t means "peeled in an earlier round" (the
// s-clique is already gone), stamp == t means "in A".
//
// Update-Func subtracts 1/a from each unpeeled r-subset, a being the number
// of peeled r-subsets of the s-clique.  Here exactly one of those a subsets,
// the one with the smallest table index (the owner), subtracts 1; the other
// a-1 do nothing.  The total is the same and all counts stay 32-bit integers.
//
// The set U of updated r-cliques is never materialised.  The only members of
// U the bucket structure needs are those that reach the current level, and
// the atomic decrement's return value identifies each of them exactly once
// (old == k+1).  They are appended to the next frontier with one atomic per
// wave (the role of the paper's per-thread list buffer).  When a round
// leaves no frontier, the level advances to the minimum live count, found by
// a reduction over a compacted list of live r-cliques.
#include "nd_host.h"

namespace nd {

namespace {

int64_t grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  return b < cap ? b : cap;
}

struct PeelArgs {
  GraphView g;
  TableView T;
  uint32_t t, k;
  uint32_t *Fnext;
  Counters *ctr;
  unsigned long long *stats;  // kStatLines x kStatStride
  uint32_t kw;                // top of the level window (> k), or 0: no window
  uint32_t *Low;              // r-cliques whose count fell to kw (window list)
};

struct LaneStats {
  uint64_t dec = 0, disc = 0;
  uint32_t err = 0;
};

constexpr int kAppendCap = 512;  // LDS entries per wave for next-frontier appends
using Appender = WaveAppender<kAppendCap>;

// Update-Func for one s-clique S (sorted) found from the peeled r-clique at
// slot p, whose vertices occupy the positions in rmask.  Called by every
// lane of the wave in lock-step (active=false lanes only join the appends).
template <int R, int S, bool kConvergent>
__device__ __forceinline__ void update_func(const PeelArgs &a, const int32_t (&Sv)[S],
                                            uint32_t rmask, uint32_t p, bool active,
                                            LaneStats &ls, Appender *ap) {
  constexpr Combos<S, R> cb{};
  constexpr int N = cb.N;
  int32_t v1[N];
  uint64_t key[N];
  bool want[N];
#pragma unroll
  for (int q = 0; q < N; q++) {
    int32_t Rv[R];
#pragma unroll
    for (int i = 0; i < R; i++) Rv[i] = Sv[cb.idx[q][i]];
    v1[q] = Rv[0];
    key[q] = make_key<R>(Rv, a.T.bits);
    want[q] = active && cb.mask[q] != rmask;
  }
  int64_t pos[N];
  Slot sl[N];
  table_find_n<N>(a.T, v1, key, want, pos, sl);
  bool alive = active;
  uint32_t owner = p;
  bool live[N];
#pragma unroll
  for (int q = 0; q < N; q++) {
    live[q] = false;
    if (!want[q]) continue;
    if (pos[q] < 0) {
      ls.err |= kErrLookup;
      alive = false;
    } else if (sl[q].stamp < a.t) {
      alive = false;  // S was destroyed in an earlier round
    } else if (sl[q].stamp == a.t) {
      owner = (uint32_t)pos[q] < owner ? (uint32_t)pos[q] : owner;
    } else {
      live[q] = true;
    }
  }
  if (active) ls.disc++;
  const bool mine = alive && owner == p;
#pragma unroll
  for (int q = 0; q < N; q++) {
    bool want_append = false, want_low = false;
    if (mine && live[q]) {
      uint32_t old = __hip_atomic_fetch_add(&a.T.slots[pos[q]].cnt, 0xFFFFFFFFu, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
      ls.dec++;
      want_append = old == a.k + 1;              // reaches this round's level
      want_low = a.kw > a.k && old == a.kw + 1;  // enters the level window
    }
    if constexpr (kConvergent) {
      ap[0].push(want_append, (uint32_t)pos[q]);
      ap[1].push(want_low, (uint32_t)pos[q]);
    } else {
      if (want_append) a.Fnext[atomicAdd(&a.ctr->next_size, 1u)] = (uint32_t)pos[q];
      if (want_low) a.Low[atomicAdd(&a.ctr->low_size, 1u)] = (uint32_t)pos[q];
    }
  }
}

// Extension of the peeled R by a clique Q of size S-R inside
// I = common neighbourhood of R: Q[0] is given, later members are
// out-neighbours of the previous one that are adjacent to all of R and Q.
template <int L, int R, int S>
__device__ void extend_q(const PeelArgs &a, const int32_t (&Rv)[R], int32_t (&Q)[S - R],
                         uint32_t p, LaneStats &ls) {
  const int32_t x = Q[L - 1];
  for (int64_t e = a.g.up[x]; e < a.g.rp[x + 1]; e++) {
    const int32_t y = a.g.col[e];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < R; j++) ok = ok && adjacent(a.g, Rv[j], y);
#pragma unroll
    for (int j = 0; j < L - 1; j++) ok = ok && adjacent(a.g, Q[j], y);
    if (!ok) continue;
    Q[L] = y;
    if constexpr (L + 1 == S - R) {
      int32_t Sv[S];
      uint32_t rmask = 0;
      int i = 0, j = 0;
#pragma unroll
      for (int o = 0; o < S; o++) {
        if (j >= S - R || (i < R && Rv[i] < Q[j])) {
          Sv[o] = Rv[i++];
          rmask |= 1u << o;
        } else {
          Sv[o] = Q[j++];
        }
      }
      update_func<R, S, false>(a, Sv, rmask, p, true, ls, nullptr);
    } else {
      extend_q<L + 1, R, S>(a, Rv, Q, p, ls);
    }
  }
}

// One wave per peeled r-clique (Algorithm 2, Update).
template <int R, int S>
__global__ __launch_bounds__(256) void k_peel(PeelArgs a, const uint32_t *__restrict__ F,
                                              uint32_t nF) {
  const int wpb = blockDim.x / kWave;
  const int lane = lane_id();
  LaneStats ls;
  __shared__ uint32_t abuf[256 / kWave][2][kAppendCap];
  Appender ap[2] = {{abuf[threadIdx.x / kWave][0], 0u, a.Fnext, &a.ctr->next_size},
                    {abuf[threadIdx.x / kWave][1], 0u, a.Low, &a.ctr->low_size}};
  for (int64_t it = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; it < nF;
       it += (int64_t)gridDim.x * wpb) {
    const uint32_t p = F[it];
    const Slot sl = a.T.slots[p];
    if (sl.cnt == 0) continue;  // every s-clique of R is already gone
    int32_t Rv[R];
    Rv[0] = a.T.v1[p];
    decode_key<R>(sl.key, a.T.bits, Rv);
    // drive the intersection from the member of R with the smallest degree
    int drv = 0;
    int64_t best = a.g.rp[Rv[0] + 1] - a.g.rp[Rv[0]];
#pragma unroll
    for (int i = 1; i < R; i++) {
      int64_t d = a.g.rp[Rv[i] + 1] - a.g.rp[Rv[i]];
      if (d < best) {
        best = d;
        drv = i;
      }
    }
    const int64_t lo = a.g.rp[Rv[drv]];
    for (int64_t base = 0; base < best; base += kWave) {
      const int64_t idx = base + lane;
      bool in = idx < best;
      int32_t x = in ? a.g.col[lo + idx] : 0;
#pragma unroll
      for (int i = 0; i < R; i++)
        if (i != drv) in = in && adjacent(a.g, x, Rv[i]);
      if constexpr (S - R == 1) {
        int32_t Sv[S];
        uint32_t rmask = 0;
        int at = 0;
#pragma unroll
        for (int i = 0; i < R; i++) at += Rv[i] < x ? 1 : 0;
#pragma unroll
        for (int o = 0, i = 0; o < S; o++) {
          if (o == at) {
            Sv[o] = x;
          } else {
            Sv[o] = Rv[i++];
            rmask |= 1u << o;
          }
        }
        update_func<R, S, true>(a, Sv, rmask, p, in, ls, ap);
      } else {
        if (in) {
          int32_t Q[S - R];
          Q[0] = x;
          extend_q<1, R, S>(a, Rv, Q, p, ls);
        }
      }
    }
  }
  ap[0].flush();
  ap[1].flush();
  stat_add(a.stats, kStatDec, ls.dec);
  stat_add(a.stats, kStatDisc, ls.disc);
  if (ls.err) atomicOr(&a.ctr->err, ls.err);
}

// ------------------------------------------------------------ s = r + 1
// The common neighbourhood I(R) of R = {v1 < ... < vr} is split by the
// orientation (see the index builder): x > v1 are the set bits of the AND
// of the rows of v2..vr in v1's adjacency bitmap; x < v1 are the members
// of every apex list of the arcs (v1, vi).

__device__ __forceinline__ int64_t lower_pos(const int32_t *__restrict__ a, int64_t lo, int64_t hi,
                                             int32_t y) {
  while (lo < hi) {
    int64_t mid = (lo + hi) >> 1;
    if (a[mid] < y) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

// r = 3 liveness bitmaps.  A triangle's bits in its root's alive bitmap are
// cleared after the round that peels it, so the AND of two alive rows lists
// only candidates whose two triangles through v1 were not peeled earlier.
__global__ void k_clear_alive(GraphView g, TableView T, FastView fx,
                              const uint32_t *__restrict__ F, uint32_t nF) {
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < nF;
       it += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = F[it];
    int32_t Rv[3];
    Rv[0] = T.v1[p];
    decode_key<3>(T.slots[p].key, T.bits, Rv);
    const int64_t o = g.up[Rv[0]];
    const int d = (int)(g.rp[Rv[0] + 1] - o);
    if (d > 512) continue;
    const int64_t i = lower_pos(g.col, o, o + d, Rv[1]) - o;
    const int64_t j = lower_pos(g.col, o, o + d, Rv[2]) - o;
    if (i >= d || j >= d) continue;
    const int wd = (d + 63) >> 6;
    unsigned long long *rows = (unsigned long long *)(fx.alive + fx.bm_off[Rv[0]]);
    atomicAnd(&rows[i * wd + (j >> 6)], ~(1ull << (j & 63)));
    atomicAnd(&rows[j * wd + (i >> 6)], ~(1ull << (i & 63)));
  }
}

// count(R) = |I(R)|, computed per r-clique without atomics.
template <int R>
__global__ __launch_bounds__(256) void k_count_direct(GraphView g, TableView T, FastView fx,
                                                      const uint32_t *__restrict__ occ,
                                                      uint64_t n_r, uint32_t *err) {
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < (int64_t)n_r;
       it += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = occ[it];
    const Slot sl = T.slots[p];
    int32_t Rv[R];
    Rv[0] = T.v1[p];
    decode_key<R>(sl.key, T.bits, Rv);
    const int32_t v1 = Rv[0];
    const int64_t o = g.up[v1];
    const int d = (int)(g.rp[v1 + 1] - o);
    int64_t e[R];
    bool found = true;
    {
      int32_t ys[R - 1];
      int64_t at[R - 1];
#pragma unroll
      for (int i = 1; i < R; i++) ys[i - 1] = Rv[i];
      lower_bounds<R - 1>(g.col, o, o + d, ys, at);
#pragma unroll
      for (int i = 1; i < R; i++) {
        e[i] = at[i - 1];
        found = found && e[i] < o + d && g.col[e[i]] == Rv[i];
      }
    }
    if (!found) {
      atomicOr(err, kErrLookup);
      continue;
    }
    uint32_t c = 0;
    if (d <= 512) {
      const int wd = (d + 63) >> 6;
      const uint64_t *rows = fx.bm + fx.bm_off[v1];
      for (int w = 0; w < wd; w++) {
        uint64_t x = ~0ull;
#pragma unroll
        for (int i = 1; i < R; i++) x &= rows[(e[i] - o) * wd + w];
        c += (uint32_t)__popcll(x);
      }
    } else {
      for (int64_t j = o; j < o + d; j++) {
        const int32_t y = g.col[j];
        bool ok = true;
#pragma unroll
        for (int i = 1; i < R; i++) ok = ok && adjacent(g, y, Rv[i]);
        c += ok ? 1u : 0u;
      }
    }
    int drv = 1;
    uint64_t best = fx.lptr[e[1] + 1] - fx.lptr[e[1]];
#pragma unroll
    for (int i = 2; i < R; i++) {
      uint64_t len = fx.lptr[e[i] + 1] - fx.lptr[e[i]];
      if (len < best) {
        best = len;
        drv = i;
      }
    }
    if (R == 2) {
      c += (uint32_t)best;
    } else {
      for (uint64_t j = fx.lptr[e[drv]]; j < fx.lptr[e[drv] + 1]; j++) {
        const int32_t x = fx.lval[j];
        bool ok = true;
#pragma unroll
        for (int i = 1; i < R; i++)
          if (i != drv) ok = ok && sorted_contains(fx.lval, fx.lptr[e[i]], fx.lptr[e[i] + 1], x);
        c += ok ? 1u : 0u;
      }
    }
    T.slots[p].cnt = c;
  }
}

template <int R>
__device__ __forceinline__ void peel_candidate(const PeelArgs &a, const int32_t (&Rv)[R],
                                               int32_t x, bool in, uint32_t p, LaneStats &ls,
                                               Appender *ap) {
  constexpr int S = R + 1;
  int32_t Sv[S];
  uint32_t rmask = 0;
  int at = 0;
#pragma unroll
  for (int i = 0; i < R; i++) at += Rv[i] < x ? 1 : 0;
#pragma unroll
  for (int o = 0, i = 0; o < S; o++) {
    if (o == at) {
      Sv[o] = x;
    } else {
      Sv[o] = Rv[i++];
      rmask |= 1u << o;
    }
  }
  update_func<R, S, true>(a, Sv, rmask, p, in, ls, ap);
}

constexpr int kListCap = 1024;  // LDS entries per wave for a staged apex list

__device__ __forceinline__ bool lds_contains(const int32_t *a, int n, int32_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int32_t v = a[mid];
    if (v == x) return true;
    if (v < x) lo = mid + 1;
    else hi = mid;
  }
  return false;
}

// ---------------------------------------------- split round (expand/apply)
// A round of the s = r+1 peel in three passes over the frontier:
//   bound   thread per r-clique: decode it (slot, first vertex, local
//           indices) and bound its candidates: popcount of the AND of the
//           alive rows + length of the shortest apex list;
//   expand  wave per r-clique: write one record (frontier index, x) per
//           candidate at the prefix-summed offset, x = -1 where the apex
//           membership test fails;
//   apply   thread per record: Update-Func for s-clique R + x, every probe
//           and decrement of a thread independent of the others.
// The apply pass carries almost all memory operations of the round with a
// dependency chain of about five accesses per thread.

template <int R>
__device__ __forceinline__ bool front_positions(const PeelArgs &a, uint64_t lc,
                                                const int32_t (&Rv)[R], int64_t o, int d,
                                                int64_t (&e)[R]) {
  if (lc >> 63) {
#pragma unroll
    for (int i = 1; i < R; i++) e[i] = o + (int64_t)((lc >> (9 * (i - 1))) & 511u);
    return true;
  }
  int32_t ys[R - 1];
  int64_t at[R - 1];
#pragma unroll
  for (int i = 1; i < R; i++) ys[i - 1] = Rv[i];
  lower_bounds<R - 1>(a.g.col, o, o + d, ys, at);
  bool found = true;
#pragma unroll
  for (int i = 1; i < R; i++) {
    e[i] = at[i - 1];
    found = found && e[i] < o + d && a.g.col[e[i]] == Rv[i];
  }
  return found;
}

template <int R>
__global__ __launch_bounds__(256) void k_expand_bound(PeelArgs a, FastView fx,
                                                      const uint64_t *__restrict__ loc,
                                                      const uint32_t *__restrict__ F, uint32_t nF,
                                                      uint64_t *ub, int32_t *fv) {
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nF;
       f += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = F[f];
    const Slot sl = a.T.slots[p];
    int32_t Rv[R];
    Rv[0] = a.T.v1[p];
    decode_key<R>(sl.key, a.T.bits, Rv);
#pragma unroll
    for (int i = 0; i < R; i++) fv[f * R + i] = Rv[i];
    uint64_t bound = 0;
    if (sl.cnt != 0) {  // otherwise every s-clique of R is already gone
      const int64_t o = a.g.up[Rv[0]];
      const int d = (int)(a.g.rp[Rv[0] + 1] - o);
      int64_t e[R];
      if (front_positions<R>(a, loc[p], Rv, o, d, e)) {
        uint64_t total1 = 0;
        if (d <= 512) {
          const int wd = (d + 63) >> 6;
          const uint64_t *rows = (R == 3 ? fx.alive : fx.bm) + fx.bm_off[Rv[0]];
          for (int w = 0; w < wd; w++) {
            uint64_t x = ~0ull;
#pragma unroll
            for (int i = 1; i < R; i++) x &= rows[(e[i] - o) * wd + w];
            total1 += (uint64_t)__popcll(x);
          }
        } else {
          total1 = (uint64_t)d;
        }
        uint64_t len2 = fx.lptr[e[1] + 1] - fx.lptr[e[1]];
#pragma unroll
        for (int i = 2; i < R; i++) {
          const uint64_t len = fx.lptr[e[i] + 1] - fx.lptr[e[i]];
          len2 = len < len2 ? len : len2;
        }
        bound = total1 + len2;
      } else {
        atomicOr(&a.ctr->err, kErrLookup);
      }
    }
    ub[f] = bound;
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_expand(PeelArgs a, FastView fx,
                                                const uint64_t *__restrict__ loc,
                                                const uint32_t *__restrict__ F, uint32_t nF,
                                                const uint64_t *__restrict__ off,
                                                const int32_t *__restrict__ fv, int2 *rec) {
  const int wpb = blockDim.x / kWave;
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  __shared__ int32_t lbuf[256 / kWave][R == 3 ? kListCap : 1];
  for (int64_t f = (int64_t)blockIdx.x * wpb + wv; f < nF; f += (int64_t)gridDim.x * wpb) {
    const uint64_t b = off[f];
    const uint64_t total = off[f + 1] - b;
    if (total == 0) continue;
    const uint32_t p = F[f];
    int32_t Rv[R];
#pragma unroll
    for (int i = 0; i < R; i++) Rv[i] = fv[f * R + i];
    const int32_t v1 = Rv[0];
    const int64_t o = a.g.up[v1];
    const int d = (int)(a.g.rp[v1 + 1] - o);
    int64_t e[R];
    front_positions<R>(a, loc[p], Rv, o, d, e);  // found: the bound pass checked it
    const bool has_bm = d <= 512;
    uint32_t total1, iw[8];
    uint64_t cw = 0;
    if (has_bm) {
      const int wd = (d + 63) >> 6;
      const uint64_t *rows = (R == 3 ? fx.alive : fx.bm) + fx.bm_off[v1];
      if (lane < wd) {
        cw = ~0ull;
#pragma unroll
        for (int i = 1; i < R; i++) cw &= rows[(e[i] - o) * wd + lane];
      }
      const uint32_t incl = wave_incl_scan((uint32_t)__popcll(cw));
      total1 = __shfl(incl, kWave - 1);
#pragma unroll
      for (int q = 0; q < 8; q++) iw[q] = __shfl(incl, q);
    } else {
      total1 = (uint32_t)d;
#pragma unroll
      for (int q = 0; q < 8; q++) iw[q] = 0;
    }
    int drv = 1;
    uint64_t len2 = fx.lptr[e[1] + 1] - fx.lptr[e[1]];
#pragma unroll
    for (int i = 2; i < R; i++) {
      const uint64_t len = fx.lptr[e[i] + 1] - fx.lptr[e[i]];
      if (len < len2) {
        len2 = len;
        drv = i;
      }
    }
    const uint64_t lb = fx.lptr[e[drv]];
    int staged_len = -1;
    uint64_t ob = 0, oe = 0;
    if constexpr (R == 3) {
      const int other = drv == 1 ? 2 : 1;
      ob = fx.lptr[e[other]];
      oe = fx.lptr[e[other] + 1];
      if (len2 > 0 && oe - ob <= (uint64_t)kListCap) {
        staged_len = (int)(oe - ob);
        for (int i = lane; i < staged_len; i += kWave) lbuf[wv][i] = fx.lval[ob + i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
    for (uint64_t base = 0; base < total; base += kWave) {
      const uint64_t k = base + lane;
      bool in = k < total;
      int32_t x = 0;
      const uint32_t kk = k < total1 ? (uint32_t)k : 0u;
      int w = 0;
      uint32_t before = 0;
#pragma unroll
      for (int q = 0; q < 7; q++) {
        if (iw[q] <= kk) {
          w = q + 1;
          before = iw[q];
        }
      }
      const uint64_t wordw = __shfl(cw, w);
      if (in && k < total1) {
        if (has_bm) {
          uint64_t m = wordw;
          for (uint32_t q = 0; q < kk - before; q++) m &= m - 1;
          x = a.g.col[o + w * 64 + (__ffsll((unsigned long long)m) - 1)];
        } else {
          x = a.g.col[o + (int64_t)k];
#pragma unroll
          for (int i = 1; i < R; i++) in = in && adjacent(a.g, x, Rv[i]);
        }
      } else if (in) {
        x = fx.lval[lb + (k - total1)];
        if constexpr (R == 3) {
          in = staged_len >= 0 ? lds_contains(lbuf[wv], staged_len, x)
                               : sorted_contains(fx.lval, ob, oe, x);
        } else {
#pragma unroll
          for (int i = 1; i < R; i++)
            if (i != drv)
              in = in && sorted_contains(fx.lval, fx.lptr[e[i]], fx.lptr[e[i] + 1], x);
        }
      }
      if (k < total) rec[b + k] = make_int2((int)f, in ? x : -1);
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_apply(PeelArgs a, const int2 *__restrict__ rec,
                                               uint64_t total, const uint32_t *__restrict__ F,
                                               const int32_t *__restrict__ fv) {
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  LaneStats ls;
  __shared__ uint32_t abuf[256 / kWave][2][kAppendCap];
  Appender ap[2] = {{abuf[wv][0], 0u, a.Fnext, &a.ctr->next_size},
                    {abuf[wv][1], 0u, a.Low, &a.ctr->low_size}};
  // wave-uniform trip count: every lane reaches every append
  for (uint64_t base = ((uint64_t)blockIdx.x * blockDim.x) + (uint64_t)wv * kWave; base < total;
       base += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = base + lane;
    bool in = i < total;
    int2 rc = make_int2(0, -1);
    if (in) rc = rec[i];
    in = in && rc.y >= 0;
    int32_t Rv[R];
    uint32_t p = 0;
    if (in) {
      p = F[rc.x];
#pragma unroll
      for (int q = 0; q < R; q++) Rv[q] = fv[(int64_t)rc.x * R + q];
    } else {
#pragma unroll
      for (int q = 0; q < R; q++) Rv[q] = q;
    }
    peel_candidate<R>(a, Rv, in ? rc.y : R, in, p, ls, ap);
  }
  ap[0].flush();
  ap[1].flush();
  stat_add(a.stats, kStatDec, ls.dec);
  stat_add(a.stats, kStatDisc, ls.disc);
  if (ls.err) atomicOr(&a.ctr->err, ls.err);
}

// Direct count, one wave per r-clique (r >= 3): the part x > v1 is a
// popcount of the AND of v1's bitmap rows; the part x < v1 is the
// intersection of the apex lists, the shortest one split across the lanes
// and the other (r = 3) staged in LDS.
template <int R>
__global__ __launch_bounds__(256) void k_count_wave(PeelArgs a, FastView fx,
                                                    const uint64_t *__restrict__ loc,
                                                    const uint32_t *__restrict__ occ, uint64_t n_r) {
  const int wpb = blockDim.x / kWave;
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  __shared__ int32_t lbuf[256 / kWave][R == 3 ? kListCap : 1];
  for (int64_t it = (int64_t)blockIdx.x * wpb + wv; it < (int64_t)n_r;
       it += (int64_t)gridDim.x * wpb) {
    const uint32_t p = occ[it];
    const Slot sl = a.T.slots[p];
    int32_t Rv[R];
    Rv[0] = a.T.v1[p];
    decode_key<R>(sl.key, a.T.bits, Rv);
    const int64_t o = a.g.up[Rv[0]];
    const int d = (int)(a.g.rp[Rv[0] + 1] - o);
    int64_t e[R];
    if (!front_positions<R>(a, loc[p], Rv, o, d, e)) {  // wave-uniform
      if (lane == 0) atomicOr(&a.ctr->err, kErrLookup);
      continue;
    }
    uint32_t c = 0;
    if (d <= 512) {
      const int wd = (d + 63) >> 6;
      const uint64_t *rows = fx.bm + fx.bm_off[Rv[0]];
      if (lane < wd) {
        uint64_t x = ~0ull;
#pragma unroll
        for (int i = 1; i < R; i++) x &= rows[(e[i] - o) * wd + lane];
        c = (uint32_t)__popcll(x);
      }
    } else {
      for (int64_t j = o + lane; j < o + d; j += kWave) {
        const int32_t y = a.g.col[j];
        bool ok = true;
#pragma unroll
        for (int i = 1; i < R; i++) ok = ok && adjacent(a.g, y, Rv[i]);
        c += ok ? 1u : 0u;
      }
    }
    int drv = 1;
    uint64_t len2 = fx.lptr[e[1] + 1] - fx.lptr[e[1]];
#pragma unroll
    for (int i = 2; i < R; i++) {
      const uint64_t len = fx.lptr[e[i] + 1] - fx.lptr[e[i]];
      if (len < len2) {
        len2 = len;
        drv = i;
      }
    }
    const uint64_t lb = fx.lptr[e[drv]];
    int staged_len = -1;
    uint64_t ob = 0, oe = 0;
    if constexpr (R == 3) {
      const int other = drv == 1 ? 2 : 1;
      ob = fx.lptr[e[other]];
      oe = fx.lptr[e[other] + 1];
      if (len2 > 0 && oe - ob <= (uint64_t)kListCap) {
        staged_len = (int)(oe - ob);
        for (int i = lane; i < staged_len; i += kWave) lbuf[wv][i] = fx.lval[ob + i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
    for (uint64_t j = lane; j < len2; j += kWave) {
      const int32_t x = fx.lval[lb + j];
      bool in = true;
      if constexpr (R == 3) {
        in = staged_len >= 0 ? lds_contains(lbuf[wv], staged_len, x)
                             : sorted_contains(fx.lval, ob, oe, x);
      } else {
#pragma unroll
        for (int i = 1; i < R; i++)
          if (i != drv) in = in && sorted_contains(fx.lval, fx.lptr[e[i]], fx.lptr[e[i] + 1], x);
      }
      c += in ? 1u : 0u;
    }
    const uint64_t total = wave_sum_u64(c);
    if (lane == 0) a.T.slots[p].cnt = (uint32_t)total;
    __builtin_amdgcn_wave_barrier();
  }
}

// Local indices of v2..vr in N+(v1) for every occupied slot of a bitmap
// root (9 bits each, bit 63 marks them valid).
template <int R>
__global__ void k_make_loc(GraphView g, TableView T, uint64_t n_slots, uint64_t *loc) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < (int64_t)n_slots;
       p += (int64_t)gridDim.x * blockDim.x) {
    const Slot sl = T.slots[p];
    uint64_t v = 0;
    if (sl.key != 0) {
      int32_t Rv[R];
      Rv[0] = T.v1[p];
      decode_key<R>(sl.key, T.bits, Rv);
      const int64_t o = g.up[Rv[0]];
      const int d = (int)(g.rp[Rv[0] + 1] - o);
      if (d <= 512) {
        int32_t ys[R - 1];
        int64_t at[R - 1];
#pragma unroll
        for (int i = 1; i < R; i++) ys[i - 1] = Rv[i];
        lower_bounds<R - 1>(g.col, o, o + d, ys, at);
        bool found = true;
#pragma unroll
        for (int i = 1; i < R; i++)
          found = found && at[i - 1] < o + d && g.col[at[i - 1]] == Rv[i];
        if (found) {
          v = 1ull << 63;
#pragma unroll
          for (int i = 1; i < R; i++) v |= (uint64_t)(at[i - 1] - o) << (9 * (i - 1));
        }
      }
    }
    loc[p] = v;
  }
}

__global__ void k_stamp(const uint32_t *__restrict__ F, uint32_t nF, Slot *slots, uint32_t t) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nF;
       i += (int64_t)gridDim.x * blockDim.x)
    slots[F[i]].stamp = t;
}

__global__ __launch_bounds__(256) void k_live_min(const uint32_t *__restrict__ L, uint32_t nL,
                                                  const Slot *__restrict__ slots, uint32_t *out) {
  uint32_t m = 0xFFFFFFFFu;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nL;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Slot s = slots[L[i]];
    if (s.stamp == kLive && s.cnt < m) m = s.cnt;
  }
  m = wave_min_u32(m);
  if (lane_id() == 0 && m != 0xFFFFFFFFu) atomicMin(out, m);
}

// Three-way partition of a list of live r-clique slots by count c:
// c <= k -> F (this level's frontier), k < c <= kw -> Low (level window),
// c > kw -> High; peeled entries are dropped.  Each block compacts a tile
// of 256 x 16 entries with one atomic per output per tile (a single global
// counter per wave would serialise in L2).
constexpr int kPartThreads = 256;
constexpr int kPartItems = 16;

__global__ __launch_bounds__(kPartThreads) void k_live_partition(
    const uint32_t *__restrict__ L, uint32_t nL, const Slot *__restrict__ slots, uint32_t k,
    uint32_t kw, uint32_t *F, uint32_t *nF, uint32_t *Lo, uint32_t *nLo, uint32_t *Hi,
    uint32_t *nHi) {
  __shared__ uint32_t wsum[3][kPartThreads / kWave];
  __shared__ uint32_t base[3];
  const int tid = threadIdx.x, w = tid / kWave;
  for (int64_t tile = (int64_t)blockIdx.x * kPartThreads * kPartItems; tile < nL;
       tile += (int64_t)gridDim.x * kPartThreads * kPartItems) {
    uint32_t p[kPartItems];
    uint32_t m[3] = {0, 0, 0};  // bit j: item j goes to F / Low / High
#pragma unroll
    for (int j = 0; j < kPartItems; j++) {
      const int64_t i = tile + (int64_t)j * kPartThreads + tid;
      p[j] = 0;
      if (i < nL) {
        p[j] = L[i];
        const Slot s = slots[p[j]];
        if (s.stamp == kLive) {
          const int dst = s.cnt <= k ? 0 : (s.cnt <= kw ? 1 : 2);
          m[dst] |= 1u << j;
        }
      }
    }
    uint32_t cnt[3], incl[3];
#pragma unroll
    for (int q = 0; q < 3; q++) {
      cnt[q] = (uint32_t)__popc(m[q]);
      incl[q] = wave_incl_scan(cnt[q]);
    }
    if (lane_id() == kWave - 1)
      for (int q = 0; q < 3; q++) wsum[q][w] = incl[q];
    __syncthreads();
    if (tid < 3) {
      uint32_t tot = 0;
      for (int v = 0; v < kPartThreads / kWave; v++) {
        const uint32_t c = wsum[tid][v];
        wsum[tid][v] = tot;
        tot += c;
      }
      uint32_t *ctr = tid == 0 ? nF : (tid == 1 ? nLo : nHi);
      base[tid] = tot ? atomicAdd(ctr, tot) : 0u;
    }
    __syncthreads();
    uint32_t at[3];
#pragma unroll
    for (int q = 0; q < 3; q++) at[q] = base[q] + wsum[q][w] + incl[q] - cnt[q];
#pragma unroll
    for (int j = 0; j < kPartItems; j++) {
      if (m[0] >> j & 1u) F[at[0]++] = p[j];
      if (m[1] >> j & 1u) Lo[at[1]++] = p[j];
      if (m[2] >> j & 1u) Hi[at[2]++] = p[j];
    }
    __syncthreads();
  }
}

__global__ void k_occ_flags(const Slot *__restrict__ slots, uint64_t n, uint32_t *flags) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n;
       i += (int64_t)gridDim.x * blockDim.x)
    flags[i] = slots[i].key != 0 ? 1u : 0u;
}

__global__ void k_occ_scatter(const Slot *__restrict__ slots, uint64_t n,
                              const uint32_t *__restrict__ pos, uint32_t *occ) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n;
       i += (int64_t)gridDim.x * blockDim.x)
    if (slots[i].key != 0) occ[pos[i]] = (uint32_t)i;
}

__global__ void k_gather_counts(const uint32_t *__restrict__ occ, uint64_t n_r,
                                const Slot *__restrict__ slots, uint32_t *out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n_r;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] = slots[occ[i]].cnt;
}

template <int R>
__global__ void k_emit(const uint32_t *__restrict__ occ, uint64_t n_r, TableView T,
                       const int32_t *__restrict__ new2old, const uint32_t *__restrict__ kround,
                       uint32_t nrounds, int32_t *rcl, uint32_t *kappa) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n_r;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = occ[i];
    const Slot s = T.slots[p];
    int32_t v[R];
    v[0] = T.v1[p];
    decode_key<R>(s.key, T.bits, v);
#pragma unroll
    for (int j = 0; j < R; j++) v[j] = new2old[v[j]];
    // insertion sort into ascending original ids
#pragma unroll
    for (int j = 1; j < R; j++) {
      int32_t x = v[j];
      int q = j - 1;
      while (q >= 0 && v[q] > x) {
        v[q + 1] = v[q];
        q--;
      }
      v[q + 1] = x;
    }
#pragma unroll
    for (int j = 0; j < R; j++) rcl[i * R + j] = v[j];
    kappa[i] = s.stamp < nrounds ? kround[s.stamp] : 0xFFFFFFFFu;
  }
}

// ------------------------------------------------------------ s >= r + 2
// Update for s - r >= 2, flattened over the whole round so that one heavy
// r-clique is shared by many waves instead of being walked by one.  The
// s-cliques containing a peeled R are R plus an (s-r)-clique Q of I(R), the
// common neighbourhood of R.  I(R) is the part of the row of R's driver (the
// member with the fewest neighbours) adjacent to every other member, kept
// as one flag per position of that row.  Q is listed from its lowest vertex
// x along the out-arcs of x, so each s-clique of R is met exactly once.
//   bound:  candidates of each peeled R = the driver's degree;
//   member: a thread per candidate x: x in I(R)? and its out-degree;
//   apply:  a thread per out-arc (x, y) of a member: y in I(R) closes
//           R + {x, y} (s = r + 2) or starts a deeper extension.

// Segment of x in a nondecreasing offset array: the last i < n with
// off[i] <= x (empty segments are skipped).
__device__ __forceinline__ int64_t seg_find(const uint64_t *__restrict__ off, int64_t n,
                                            uint64_t x) {
  int64_t lo = 0, hi = n - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (off[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

struct GenView {
  const uint64_t *__restrict__ ioff;  // nF + 1 candidate offsets
  const int32_t *__restrict__ fv;     // nF * R decoded r-cliques
  const int32_t *__restrict__ drv;    // nF drivers
  const uint8_t *__restrict__ flag;   // C1 membership flags
  const uint64_t *__restrict__ aoff;  // C1 + 1 arc offsets
  uint32_t nF;
  uint64_t C1;
};

template <int R>
__global__ __launch_bounds__(256) void k_gen_bound(PeelArgs a, const uint32_t *__restrict__ F,
                                                   uint32_t nF, uint64_t *ub, int32_t *fv,
                                                   int32_t *drv) {
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nF;
       f += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t p = F[f];
    const Slot sl = a.T.slots[p];
    int32_t Rv[R];
    Rv[0] = a.T.v1[p];
    decode_key<R>(sl.key, a.T.bits, Rv);
    int32_t best_v = Rv[0];
    int64_t best = a.g.rp[Rv[0] + 1] - a.g.rp[Rv[0]];
#pragma unroll
    for (int i = 0; i < R; i++) {
      fv[f * R + i] = Rv[i];
      const int64_t d = a.g.rp[Rv[i] + 1] - a.g.rp[Rv[i]];
      if (d < best) {
        best = d;
        best_v = Rv[i];
      }
    }
    drv[f] = best_v;
    ub[f] = sl.cnt != 0 ? (uint64_t)best : 0;  // cnt 0: every s-clique of R is gone
  }
}

template <int R>
__global__ __launch_bounds__(256) void k_gen_member(GraphView g, GenView gv, uint8_t *flag,
                                                    uint64_t *arcs) {
  for (uint64_t k = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; k < gv.C1;
       k += (uint64_t)gridDim.x * blockDim.x) {
    const int64_t f = seg_find(gv.ioff, gv.nF, k);
    const int32_t v = gv.drv[f];
    const int32_t x = g.col[g.rp[v] + (int64_t)(k - gv.ioff[f])];
    bool in = true;
#pragma unroll
    for (int i = 0; i < R; i++) {
      const int32_t u = gv.fv[f * R + i];
      if (u != v) in = in && adjacent(g, x, u);
    }
    flag[k] = in ? 1 : 0;
    arcs[k] = in ? (uint64_t)(g.rp[x + 1] - g.up[x]) : 0;
  }
}

// y in I(R): a position of the driver's row whose flag is set
__device__ __forceinline__ bool gen_in(const GraphView &g, const GenView &gv, int64_t lo,
                                       int64_t hi, uint64_t fbase, int32_t y) {
  const int64_t at = lower_pos(g.col, lo, hi, y);
  return at < hi && g.col[at] == y && gv.flag[fbase + (uint64_t)(at - lo)] != 0;
}

template <int R, int Q>
__device__ __forceinline__ void merge_rq(const int32_t (&Rv)[R], const int32_t (&Qv)[Q],
                                         int32_t (&Sv)[R + Q], uint32_t &rmask) {
  rmask = 0;
  int i = 0, j = 0;
#pragma unroll
  for (int o = 0; o < R + Q; o++) {
    if (j >= Q || (i < R && Rv[i] < Qv[j])) {
      Sv[o] = Rv[i++];
      rmask |= 1u << o;
    } else {
      Sv[o] = Qv[j++];
    }
  }
}

// Q[0..L-1] is a clique inside I(R); extend it by out-neighbours of Q[L-1]
// that lie in I(R) and are adjacent to Q[0..L-2].
template <int L, int R, int S>
__device__ void gen_extend(const PeelArgs &a, const GenView &gv, int64_t lo, int64_t hi,
                           uint64_t fbase, const int32_t (&Rv)[R], int32_t (&Qv)[S - R],
                           uint32_t p, LaneStats &ls) {
  const int32_t x = Qv[L - 1];
  for (int64_t e = a.g.up[x]; e < a.g.rp[x + 1]; e++) {
    const int32_t z = a.g.col[e];
    bool ok = gen_in(a.g, gv, lo, hi, fbase, z);
#pragma unroll
    for (int j = 0; j < L - 1; j++) ok = ok && adjacent(a.g, Qv[j], z);
    if (!ok) continue;
    Qv[L] = z;
    if constexpr (L + 1 == S - R) {
      int32_t Sv[S];
      uint32_t rmask;
      merge_rq<R, S - R>(Rv, Qv, Sv, rmask);
      update_func<R, S, false>(a, Sv, rmask, p, true, ls, nullptr);
    } else {
      gen_extend<L + 1, R, S>(a, gv, lo, hi, fbase, Rv, Qv, p, ls);
    }
  }
}

template <int R, int S>
__global__ __launch_bounds__(256) void k_gen_apply(PeelArgs a, GenView gv,
                                                   const uint32_t *__restrict__ F, uint64_t A) {
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  LaneStats ls;
  __shared__ uint32_t abuf[256 / kWave][2][kAppendCap];
  Appender ap[2] = {{abuf[wv][0], 0u, a.Fnext, &a.ctr->next_size},
                    {abuf[wv][1], 0u, a.Low, &a.ctr->low_size}};
  // wave-uniform trip count: every lane reaches every append
  for (uint64_t base = ((uint64_t)blockIdx.x * blockDim.x) + (uint64_t)wv * kWave; base < A;
       base += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t i = base + lane;
    bool in = i < A;
    int32_t Rv[R];
#pragma unroll
    for (int q = 0; q < R; q++) Rv[q] = q;
    int32_t Qv[S - R];
#pragma unroll
    for (int q = 0; q < S - R; q++) Qv[q] = R + q;
    uint32_t p = 0;
    int64_t lo = 0, hi = 0;
    uint64_t fbase = 0;
    if (in) {
      const int64_t kx = seg_find(gv.aoff, (int64_t)gv.C1, i);
      const int64_t f = seg_find(gv.ioff, gv.nF, (uint64_t)kx);
      const int32_t v = gv.drv[f];
      lo = a.g.rp[v];
      hi = a.g.rp[v + 1];
      fbase = gv.ioff[f];
      const int32_t x = a.g.col[lo + (int64_t)((uint64_t)kx - fbase)];
      const int32_t y = a.g.col[a.g.up[x] + (int64_t)(i - gv.aoff[kx])];
      in = gen_in(a.g, gv, lo, hi, fbase, y);
      p = F[f];
#pragma unroll
      for (int q = 0; q < R; q++) Rv[q] = gv.fv[f * R + q];
      Qv[0] = x;
      Qv[1] = y;
    }
    if constexpr (S - R == 2) {
      int32_t Sv[S];
      uint32_t rmask;
      merge_rq<R, 2>(Rv, Qv, Sv, rmask);
      update_func<R, S, true>(a, Sv, rmask, p, in, ls, ap);
    } else {
      if (in) gen_extend<2, R, S>(a, gv, lo, hi, fbase, Rv, Qv, p, ls);
    }
  }
  ap[0].flush();
  ap[1].flush();
  stat_add(a.stats, kStatDec, ls.dec);
  stat_add(a.stats, kStatDisc, ls.disc);
  if (ls.err) atomicOr(&a.ctr->err, ls.err);
}

template <int R, int S>
uint64_t gen_impl(const PeelArgs &a, const uint32_t *F, uint32_t nF, GenBufs *gb, hipStream_t st,
                  hipEvent_t ev0, hipEvent_t ev1) {
  if (gb->ioff.n < (size_t)nF + 1) gb->ioff.reset((size_t)nF + 1 + nF / 2);
  if (gb->fv.n < (size_t)nF * R) gb->fv.reset(((size_t)nF + nF / 2) * R);
  if (gb->drv.n < (size_t)nF) gb->drv.reset((size_t)nF + nF / 2);
  hipLaunchKernelGGL(k_gen_bound<R>, dim3((unsigned)grid_for(nF, 256)), dim3(256), 0, st, a, F, nF,
                     gb->ioff.get(), gb->fv.get(), gb->drv.get());
  fill_u64(gb->ioff.get() + nF, 0, 1, st);
  scan_exclusive_u64(gb->ioff.get(), gb->ioff.get(), (int64_t)nF + 1, st);
  uint64_t C1 = 0;
  hipMemcpyAsync(&C1, gb->ioff.get() + nF, 8, hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  uint64_t A = 0;
  GenView gv{gb->ioff.get(), gb->fv.get(), gb->drv.get(), nullptr, nullptr, nF, C1};
  if (C1 > 0) {
    if (gb->flag.n < C1) gb->flag.reset(C1 + C1 / 2);
    if (gb->aoff.n < C1 + 1) gb->aoff.reset(C1 + 1 + C1 / 2);
    gv.flag = gb->flag.get();
    gv.aoff = gb->aoff.get();
    hipLaunchKernelGGL(k_gen_member<R>, dim3((unsigned)grid_for(C1, 256, 1 << 16)), dim3(256), 0,
                       st, a.g, gv, gb->flag.get(), gb->aoff.get());
    fill_u64(gb->aoff.get() + C1, 0, 1, st);
    scan_exclusive_u64(gb->aoff.get(), gb->aoff.get(), (int64_t)C1 + 1, st);
    hipMemcpyAsync(&A, gb->aoff.get() + C1, 8, hipMemcpyDeviceToHost, st);
    hipStreamSynchronize(st);
  }
  if (ev0) hipEventRecord(ev0, st);
  if (A > 0)
    hipLaunchKernelGGL((k_gen_apply<R, S>), dim3((unsigned)grid_for(A, 256, 1 << 16)), dim3(256),
                       0, st, a, gv, F, A);
  if (ev1) hipEventRecord(ev1, st);
  return A;
}

template <int R, int S>
void peel_impl(const PeelArgs &a, const uint32_t *F, uint32_t nF, hipStream_t st) {
  hipLaunchKernelGGL((k_peel<R, S>), dim3((unsigned)grid_for(nF, 4, 1 << 20)), dim3(256), 0, st,
                     a, F, nF);
}

}  // namespace

void stamp_frontier(const uint32_t *F, uint32_t nF, Slot *slots, uint32_t t, hipStream_t st) {
  if (!nF) return;
  hipLaunchKernelGGL(k_stamp, dim3((unsigned)grid_for(nF, 256)), dim3(256), 0, st, F, nF, slots,
                     t);
}

#define ND_PEEL_CASE(R_, S_) \
  case (R_) * 16 + (S_): peel_impl<R_, S_>(a, F, nF, st); break;

void peel_round(const OrientedGraph &g, int r, int s, const TableView &T, const uint32_t *F,
                uint32_t nF, uint32_t t, uint32_t k, uint32_t kw, uint32_t *Fnext, uint32_t *Low,
                Counters *dctr, unsigned long long *stats, hipStream_t st) {
  if (!nF) return;
  PeelArgs a{g.view(), T, t, k, Fnext, dctr, stats, kw, Low};
  switch (r * 16 + s) {
    ND_PEEL_CASE(1, 2) ND_PEEL_CASE(1, 3) ND_PEEL_CASE(1, 4) ND_PEEL_CASE(1, 5)
    ND_PEEL_CASE(1, 6) ND_PEEL_CASE(1, 7)
    ND_PEEL_CASE(2, 3) ND_PEEL_CASE(2, 4) ND_PEEL_CASE(2, 5) ND_PEEL_CASE(2, 6)
    ND_PEEL_CASE(2, 7)
    ND_PEEL_CASE(3, 4) ND_PEEL_CASE(3, 5) ND_PEEL_CASE(3, 6) ND_PEEL_CASE(3, 7)
    ND_PEEL_CASE(4, 5) ND_PEEL_CASE(4, 6) ND_PEEL_CASE(4, 7)
    ND_PEEL_CASE(5, 6) ND_PEEL_CASE(5, 7)
    ND_PEEL_CASE(6, 7)
    default: break;
  }
}

#define ND_GEN_CASE(R_, S_) \
  case (R_) * 16 + (S_): return gen_impl<R_, S_>(a, F, nF, gb, st, ev0, ev1);

uint64_t peel_round_gen(const OrientedGraph &g, int r, int s, const TableView &T,
                        const uint32_t *F, uint32_t nF, uint32_t t, uint32_t k, uint32_t kw,
                        uint32_t *Fnext, uint32_t *Low, Counters *dctr,
                        unsigned long long *stats, GenBufs *gb, hipStream_t st, hipEvent_t ev0,
                        hipEvent_t ev1) {
  if (!nF) {
    if (ev0) hipEventRecord(ev0, st);
    if (ev1) hipEventRecord(ev1, st);
    return 0;
  }
  PeelArgs a{g.view(), T, t, k, Fnext, dctr, stats, kw, Low};
  switch (r * 16 + s) {
    ND_GEN_CASE(1, 3) ND_GEN_CASE(1, 4) ND_GEN_CASE(1, 5) ND_GEN_CASE(1, 6) ND_GEN_CASE(1, 7)
    ND_GEN_CASE(2, 4) ND_GEN_CASE(2, 5) ND_GEN_CASE(2, 6) ND_GEN_CASE(2, 7)
    ND_GEN_CASE(3, 5) ND_GEN_CASE(3, 6) ND_GEN_CASE(3, 7)
    ND_GEN_CASE(4, 6) ND_GEN_CASE(4, 7)
    ND_GEN_CASE(5, 7)
    default: break;
  }
  return 0;
}

void count_direct(const OrientedGraph &g, int r, const TableView &T, const FastIndex &fx,
                  const uint32_t *occ, uint64_t n_r, Counters *dctr, hipStream_t st) {
  if (!n_r) return;
  const GraphView gv = g.view();
  const FastView fv = fx.view();
  if (r == 2) {  // popcount of one row plus one list length: a thread per edge
    dim3 grid((unsigned)grid_for(n_r, 256, 1 << 20)), blk(256);
    hipLaunchKernelGGL(k_count_direct<2>, grid, blk, 0, st, gv, T, fv, occ, n_r, &dctr->err);
    return;
  }
  PeelArgs a{gv, T, 0u, 0u, nullptr, dctr, nullptr, 0u, nullptr};
  const uint64_t *loc = fx.loc.get();
  dim3 grid((unsigned)grid_for(n_r, 4, 1 << 20)), blk(256);
  switch (r) {
    case 3: hipLaunchKernelGGL(k_count_wave<3>, grid, blk, 0, st, a, fv, loc, occ, n_r); break;
    case 4: hipLaunchKernelGGL(k_count_wave<4>, grid, blk, 0, st, a, fv, loc, occ, n_r); break;
    case 5: hipLaunchKernelGGL(k_count_wave<5>, grid, blk, 0, st, a, fv, loc, occ, n_r); break;
    case 6: hipLaunchKernelGGL(k_count_wave<6>, grid, blk, 0, st, a, fv, loc, occ, n_r); break;
    default: break;
  }
}

template <int R>
float split_impl(const PeelArgs &a, const FastIndex &fx, const uint32_t *F, uint32_t nF,
                 SplitBufs *sb, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  const FastView fv = fx.view();
  const uint64_t *loc = fx.loc.get();
  if (sb->off.n < (size_t)nF + 1) sb->off.reset((size_t)nF + 1 + nF / 2);
  if (sb->fv.n < (size_t)nF * R) sb->fv.reset(((size_t)nF + nF / 2) * R);
  hipLaunchKernelGGL(k_expand_bound<R>, dim3((unsigned)grid_for(nF, 256)), dim3(256), 0, st, a, fv,
                     loc, F, nF, sb->off.get(), sb->fv.get());
  fill_u64(sb->off.get() + nF, 0, 1, st);
  scan_exclusive_u64(sb->off.get(), sb->off.get(), (int64_t)nF + 1, st);
  uint64_t total = 0;
  hipMemcpyAsync(&total, sb->off.get() + nF, 8, hipMemcpyDeviceToHost, st);
  hipStreamSynchronize(st);
  if (total == 0) {  // keep the event pair consistent for the caller's timing
    if (ev0) hipEventRecord(ev0, st);
    if (ev1) hipEventRecord(ev1, st);
    return 0.f;
  }
  if (sb->rec.n < total) sb->rec.reset(total + total / 2);
  hipLaunchKernelGGL(k_expand<R>, dim3((unsigned)grid_for(nF, 4, 1 << 20)), dim3(256), 0, st, a,
                     fv, loc, F, nF, sb->off.get(), sb->fv.get(), sb->rec.get());
  if (ev0) hipEventRecord(ev0, st);
  hipLaunchKernelGGL(k_apply<R>, dim3((unsigned)grid_for(total, 256, 1 << 16)), dim3(256), 0, st, a,
                     sb->rec.get(), total, F, sb->fv.get());
  if (ev1) hipEventRecord(ev1, st);
  return (float)total;
}

uint64_t peel_round_split(const OrientedGraph &g, int r, const TableView &T, const FastIndex &fx,
                          const uint32_t *F, uint32_t nF, uint32_t t, uint32_t k, uint32_t kw,
                          uint32_t *Fnext, uint32_t *Low, Counters *dctr,
                          unsigned long long *stats, SplitBufs *sb, hipStream_t st,
                          hipEvent_t ev0, hipEvent_t ev1) {
  if (!nF) {
    if (ev0) hipEventRecord(ev0, st);
    if (ev1) hipEventRecord(ev1, st);
    return 0;
  }
  PeelArgs a{g.view(), T, t, k, Fnext, dctr, stats, kw, Low};
  float tot = 0;
  switch (r) {
    case 2: tot = split_impl<2>(a, fx, F, nF, sb, st, ev0, ev1); break;
    case 3: tot = split_impl<3>(a, fx, F, nF, sb, st, ev0, ev1); break;
    case 4: tot = split_impl<4>(a, fx, F, nF, sb, st, ev0, ev1); break;
    case 5: tot = split_impl<5>(a, fx, F, nF, sb, st, ev0, ev1); break;
    case 6: tot = split_impl<6>(a, fx, F, nF, sb, st, ev0, ev1); break;
    default: break;
  }
  return (uint64_t)tot;
}

void build_slot_loc(const OrientedGraph &g, int r, const TableView &T, uint64_t n_slots,
                    FastIndex *fx, hipStream_t st) {
  fx->loc.reset(n_slots ? n_slots : 1);
  if (!n_slots) return;
  dim3 grid((unsigned)grid_for(n_slots, 256)), blk(256);
  const GraphView gv = g.view();
  switch (r) {
    case 2: hipLaunchKernelGGL(k_make_loc<2>, grid, blk, 0, st, gv, T, n_slots, fx->loc.get()); break;
    case 3: hipLaunchKernelGGL(k_make_loc<3>, grid, blk, 0, st, gv, T, n_slots, fx->loc.get()); break;
    case 4: hipLaunchKernelGGL(k_make_loc<4>, grid, blk, 0, st, gv, T, n_slots, fx->loc.get()); break;
    case 5: hipLaunchKernelGGL(k_make_loc<5>, grid, blk, 0, st, gv, T, n_slots, fx->loc.get()); break;
    case 6: hipLaunchKernelGGL(k_make_loc<6>, grid, blk, 0, st, gv, T, n_slots, fx->loc.get()); break;
    default: break;
  }
}

void clear_alive(const OrientedGraph &g, const TableView &T, const FastIndex &fx,
                 const uint32_t *F, uint32_t nF, hipStream_t st) {
  if (!nF) return;
  hipLaunchKernelGGL(k_clear_alive, dim3((unsigned)grid_for(nF, 256)), dim3(256), 0, st,
                     g.view(), T, fx.view(), F, nF);
}

void live_min(const uint32_t *L, uint32_t nL, const Slot *slots, Counters *dctr, hipStream_t st) {
  fill_u32(&dctr->live_min, 0xFFFFFFFFu, 1, st);
  if (!nL) return;
  hipLaunchKernelGGL(k_live_min, dim3((unsigned)grid_for(nL, 256 * 8, 8192)), dim3(256), 0, st, L,
                     nL, slots, &dctr->live_min);
}

void live_partition(const uint32_t *L, uint32_t nL, const Slot *slots, uint32_t k, uint32_t kw,
                    uint32_t *F, uint32_t *Low, uint32_t *High, Counters *dctr, hipStream_t st) {
  fill_u32(&dctr->next_size, 0, 1, st);
  fill_u32(&dctr->low_size, 0, 2, st);  // low_size, high_size
  if (!nL) return;
  hipLaunchKernelGGL(k_live_partition,
                     dim3((unsigned)grid_for(nL, kPartThreads * kPartItems, 8192)),
                     dim3(kPartThreads), 0, st, L, nL, slots, k, kw, F, &dctr->next_size, Low,
                     &dctr->low_size, High, &dctr->high_size);
}

void occupied_list(const Slot *slots, uint64_t n_slots, uint32_t *occ, hipStream_t st) {
  if (!n_slots) return;
  DevBuf<uint32_t> pos((size_t)n_slots);
  hipLaunchKernelGGL(k_occ_flags, dim3((unsigned)grid_for(n_slots, 256)), dim3(256), 0, st, slots,
                     n_slots, pos.get());
  scan_exclusive_u32(pos.get(), pos.get(), (int64_t)n_slots, st);
  hipLaunchKernelGGL(k_occ_scatter, dim3((unsigned)grid_for(n_slots, 256)), dim3(256), 0, st,
                     slots, n_slots, pos.get(), occ);
}

void gather_counts(const uint32_t *occ, uint64_t n_r, const Slot *slots, uint32_t *out,
                   hipStream_t st) {
  if (!n_r) return;
  hipLaunchKernelGGL(k_gather_counts, dim3((unsigned)grid_for(n_r, 256)), dim3(256), 0, st, occ,
                     n_r, slots, out);
}

void emit(int r, const uint32_t *occ, uint64_t n_r, const TableView &T, const int32_t *new2old,
          const uint32_t *kround, uint32_t nrounds, int32_t *rcl_out, uint32_t *kappa_out,
          hipStream_t st) {
  if (!n_r) return;
  dim3 grid((unsigned)grid_for(n_r, 256)), blk(256);
  switch (r) {
    case 1: hipLaunchKernelGGL(k_emit<1>, grid, blk, 0, st, occ, n_r, T, new2old, kround, nrounds, rcl_out, kappa_out); break;
    case 2: hipLaunchKernelGGL(k_emit<2>, grid, blk, 0, st, occ, n_r, T, new2old, kround, nrounds, rcl_out, kappa_out); break;
    case 3: hipLaunchKernelGGL(k_emit<3>, grid, blk, 0, st, occ, n_r, T, new2old, kround, nrounds, rcl_out, kappa_out); break;
    case 4: hipLaunchKernelGGL(k_emit<4>, grid, blk, 0, st, occ, n_r, T, new2old, kround, nrounds, rcl_out, kappa_out); break;
    case 5: hipLaunchKernelGGL(k_emit<5>, grid, blk, 0, st, occ, n_r, T, new2old, kround, nrounds, rcl_out, kappa_out); break;
    case 6: hipLaunchKernelGGL(k_emit<6>, grid, blk, 0, st, occ, n_r, T, new2old, kround, nrounds, rcl_out, kappa_out); break;
    default: break;
  }
}

}  // namespace nd
