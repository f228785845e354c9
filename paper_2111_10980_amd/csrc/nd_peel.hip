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
// the owner, subtracts 1; the other a-1 do nothing.  The total is the same and
// all counts stay 32-bit integers.  The owner is the peeled subset that comes
// first in lexicographic order of positions in the sorted s-clique (for
// s = r+1: the one that omits the largest vertex), which the s = r+1 expand
// pass can often decide from bitmaps before probing any slot.
//
// The set U of updated r-cliques is never materialised.  The only members of
// U the bucket structure needs are those that reach the current level, and
// the atomic decrement's return value identifies each of them exactly once
// (old == k+1).  They are appended to the next frontier with one atomic per
// wave (the role of the paper's per-thread list buffer).  When a round
// leaves no frontier, the level advances to the minimum live count, found by
// a reduction over a compacted list of live r-cliques.
#include <stddef.h>
#include <stdlib.h>
#include <string.h>

#include <chrono>
#include <vector>

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

struct LaneStats {  // per lane and launch: far below 2^32
  uint32_t dec = 0, disc = 0, atom = 0;
  uint32_t err = 0;
};

constexpr int kAppendCap = 512;  // LDS entries per wave for next-frontier appends
constexpr int kApexShift = 18;   // r = 3 loc word: 1 + apex-entry position in bits 18..61
constexpr uint64_t kApexMask = (1ull << 44) - 1;
using Appender = WaveAppender<kAppendCap>;

// Round kernels run only while rounds remain and the host has not been asked
// to step in (the test is uniform over the grid).
__device__ __forceinline__ bool rc_idle(const RoundCtl *rc) { return (rc->done | rc->halt) != 0; }

// The constant part of the arguments (graph, table, counters) comes by value;
// the round's level, window, round number and output lists from the control
// block.
__device__ __forceinline__ PeelArgs round_args(PeelArgs a, const RoundCtl *rc) {
  a.t = rc->t;
  a.k = rc->k;
  a.kw = rc->kw;
  a.Fnext = rc->Fnext;
  a.Low = rc->Low;
  return a;
}

// Start of a round (one thread).  If the round starts with an empty frontier
// the level advance is finished first: k <- max(k, minimum), new list sizes,
// swapped list buffers.  A window list that holds only peeled r-cliques is
// dropped instead and the round stays empty (the next one scans the high
// list).  Then the round's lists and counters.
__device__ void round_begin_body(RoundCtl *rc, Counters *dc) {
  if (rc->nF == 0) {  // finish the advance first: a rerun must not partition again
    const bool win = rc->nW != 0;
    const uint32_t mn = win ? rc->mw : rc->mh;
    // written by other blocks' atomics in the same launch (k_advance_begin)
    const uint32_t cF = __hip_atomic_load(&rc->cF, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t cW = __hip_atomic_load(&rc->cW, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t cH = __hip_atomic_load(&rc->cH, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (win && mn == kNone) {
      rc->wscan += rc->nW;
      rc->nW = 0;
    } else if (mn == kNone || cF == 0) {  // no live r-clique left, or an empty bucket
      rc->err |= kErrBucket;
      rc->halt = 3;
      return;
    } else {
      rc->k = rc->k > mn ? rc->k : mn;
      if (win) {
        rc->wscan += rc->nW;  // this advance scanned the window list
        rc->selW ^= 1u;
      } else {
        rc->kw = window_top(rc->k, rc->wlev);
        // Balance the width of the next window: the advances inside the
        // window that just closed scanned wscan window-list entries, this
        // new window scanned the nH entries of the high list.  Narrower
        // windows when the former dominates, wider when the latter does.
        // (Measured against a fixed 16 levels: rMAT (3,5) scale 15 -19%,
        // (2,4) scale 17 -9%, Chung-Lu 1M (2,4) -4%, rMAT-18 (3,4) equal,
        // Chung-Lu 1M (4,5) +2%; widening is what the deep peels gain from,
        // and capped at 16 levels they lost it.)
        const uint64_t scan_h = rc->nH;
        if (rc->wscan > 2 * scan_h && rc->wlev > 1) rc->wlev >>= 1;
        else if (2 * rc->wscan < scan_h && rc->wlev < kMaxWindowLevels) rc->wlev <<= 1;
        rc->wscan = 0;
        rc->nH = cH;
        rc->selH ^= 1u;
      }
      rc->nW = cW;
      rc->nF = cF;
      rc->advances++;
    }
    rc->mw = kNone;
    rc->mh = kNone;
    rc->cF = rc->cW = rc->cH = 0;
  }
  if (rc->t >= rc->trace_cap) {  // the host grows the round trace, then reruns
    rc->halt = 2;
    return;
  }
  const uint32_t sF = rc->selF;
  rc->F = rc->bufF[sF];
  rc->Fnext = rc->bufF[sF ^ 1u];
  rc->Low = rc->bufW[rc->selW];
  rc->total = 0;
  rc->total2 = 0;
  rc->total3 = 0;
  rc->nA = rc->nF;
  dc->next_size = 0;
  dc->low_size = rc->nW;  // window appends continue after the live entries
}

// End of a round (one thread): trace, finished += |A_t|, next frontier.  An
// empty round (one that only dropped the window list) is not counted.
__device__ void round_end_body(RoundCtl *rc, const Counters *dc) {
  if (rc->nF == 0) return;
  rc->peeled_since += rc->nF;
  if (rc->contract_every && rc->peeled_since >= rc->contract_every) rc->contract_due = 1;
  if (rc->total > rc->max_total) rc->max_total = rc->total;
  if (rc->total3 > rc->max_total3) rc->max_total3 = rc->total3;
  rc->trace_size[rc->t] = rc->nF;
  rc->trace_k[rc->t] = rc->k;
  rc->finished += rc->nF;
  rc->t++;
  rc->nF = dc->next_size;
  rc->nW = dc->low_size;
  rc->selF ^= 1u;
  if (rc->finished > rc->n_r) {
    rc->err |= kErrBucket;
    rc->halt = 3;
  } else if (rc->finished == rc->n_r) {
    rc->done = 1;
  }
}

__device__ __forceinline__ uint64_t wave_incl_scan_u64(uint64_t v) {
  const int lane = lane_id();
#pragma unroll
  for (int off = 1; off < kWave; off <<= 1) {
    const uint64_t y = __shfl_up(v, off);
    if (lane >= off) v += y;
  }
  return v;
}

// Block-wide allocation from a global counter with one atomic per block:
// every thread of the (256-thread) block asks for `want` entries and gets
// the start of its own range.  Called by all threads of the block together.
__device__ __forceinline__ uint64_t block_alloc(uint64_t want, unsigned long long *counter) {
  __shared__ uint64_t wsum[256 / kWave];
  __shared__ uint64_t base;
  const int lane = lane_id(), w = threadIdx.x / kWave;
  const uint64_t incl = wave_incl_scan_u64(want);
  if (lane == kWave - 1) wsum[w] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tot = 0;
    for (int v = 0; v < 256 / kWave; v++) {
      const uint64_t c = wsum[v];
      wsum[v] = tot;
      tot += c;
    }
    base = tot ? atomicAdd(counter, (unsigned long long)tot) : 0ull;
  }
  __syncthreads();
  const uint64_t r = base + wsum[w] + incl - want;
  __syncthreads();
  return r;
}

// Update-Func for one s-clique S (sorted) found from the peeled r-clique at
// slot p, whose vertices occupy the positions in rmask.  Called by every
// lane of the wave in lock-step (active=false lanes only join the appends).
template <int R, int S, bool kConvergent>
__device__ __forceinline__ void update_func(const PeelArgs &a, const int32_t (&Sv)[S],
                                            uint32_t rmask, uint32_t p, bool active,
                                            LaneStats &ls, Appender *ap) {
  constexpr Combos<S, R> cb{};
  constexpr int N = cb.N;
  int32_t v1[N], v2[N];
  Key key[N];
  bool want[N];
#pragma unroll
  for (int q = 0; q < N; q++) {
    int32_t Rv[R];
#pragma unroll
    for (int i = 0; i < R; i++) Rv[i] = Sv[cb.idx[q][i]];
    v1[q] = Rv[0];
    v2[q] = R > 1 ? Sv[cb.idx[q][R > 1 ? 1 : 0]] : 0;
    key[q] = rkey<R>(a.T, Rv);
    want[q] = active && cb.mask[q] != rmask;
  }
  // The other subsets are looked up two at a time, and the lookups stop at
  // the first one peeled in an earlier round: S is gone then, and the
  // remaining probes would only confirm it.  (Each s-clique is listed again
  // from every subset peeled after it was destroyed; with all probes at once
  // those repeat listings carried most of the update pass's traffic.)
  int64_t pos[N];
  Slot sl[N];
  bool alive = active;
#pragma unroll
  for (int g0 = 0; g0 < N; g0 += 2) {
    int32_t gv[2], gv2[2];
    Key gk[2];
    bool gw[2];
    int64_t gp[2];
    Slot gs[2];
#pragma unroll
    for (int j = 0; j < 2; j++) {
      const int q = g0 + j < N ? g0 + j : N - 1;
      gv[j] = v1[q];
      gv2[j] = v2[q];
      gk[j] = key[q];
      gw[j] = g0 + j < N && want[q] && alive;
    }
    table_find_n<2, (R >= 4)>(a.T, gv, gv2, gk, gw, gp, gs);
#pragma unroll
    for (int j = 0; j < 2; j++) {
      if (g0 + j >= N) continue;
      pos[g0 + j] = gp[j];
      sl[g0 + j] = gs[j];
      if (!gw[j]) continue;
      if (gp[j] < 0) {
        ls.err |= kErrLookup;
        alive = false;
      } else if (gs[j].stamp < a.t) {
        alive = false;  // S was destroyed in an earlier round
      }
    }
  }
  int self = 0;  // this r-clique's place in the subset order
#pragma unroll
  for (int q = 0; q < N; q++)
    if (cb.mask[q] == rmask) self = q;
  bool other_owner = false;
  // hot: live (not peeled) and its count read above the level.  A count read
  // at or below the level has crossed k+1 (and the window level) already:
  // its decrement changes nothing after the clamp to k and needs no atomic,
  // but it is still one of the decrements Algorithm 2 applies (n_live).
  bool hot[N];
  uint32_t n_live = 0;
#pragma unroll
  for (int q = 0; q < N; q++) {
    hot[q] = false;
    if (!want[q] || !alive) continue;  // every subset was looked up when S is alive
    if (sl[q].stamp == a.t) {
      other_owner = other_owner || q < self;  // peeled with R and first in order
    } else {
      n_live++;
      hot[q] = sl[q].cnt > a.k;
    }
  }
  if (active) ls.disc++;
  const bool mine = alive && !other_owner;
  if (mine) ls.dec += n_live;
#pragma unroll
  for (int q = 0; q < N; q++) {
    bool want_append = false, want_low = false;
    if (mine && hot[q]) {
      uint32_t old = __hip_atomic_fetch_add(&a.T.slots[pos[q]].cnt, 0xFFFFFFFFu, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
      ls.atom++;
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
__global__ __launch_bounds__(256) void k_peel(PeelArgs base, const RoundCtl *__restrict__ rc) {
  if (rc_idle(rc)) return;
  const PeelArgs a = round_args(base, rc);
  const uint32_t *__restrict__ F = rc->F;
  const uint32_t nF = rc->nF;
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
    decode_key<R>(a.T, p, sl.key, Rv);
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
  stat_add(a.stats, kStatAtom, ls.atom);
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

// r = 2 arc states, one byte per arc position of G' (both directions of an
// edge carry the same state): alive, in the current round's frontier, or
// peeled in an earlier round.
constexpr uint8_t kArcAlive = 0, kArcFront = 1, kArcDead = 2;

__device__ __forceinline__ void set_edge_state(const GraphView &g, int32_t a, int32_t b,
                                               uint8_t *st, uint8_t v) {
  const int32_t lo = a < b ? a : b, hi = a < b ? b : a;
  const int64_t e = arc_pos(g, lo, hi);
  if (e < 0) return;
  st[e] = v;
  const int64_t q = lower_pos(g.col, g.rp[hi], g.up[hi], lo);  // lo sits in hi's lower part
  if (q < g.up[hi] && g.col[q] == lo) st[q] = v;
}

// r = 2, R = {u0 < u1}: may R list the s-clique R + x (s = 3)?  Not if one of
// x's edges to R was peeled earlier (the triangle is gone), nor if one is in
// the frontier and comes before R in the triangle's subset order ({x,u0}
// does when x < u1, {x,u1} when x < u0): that edge owns it (Update-Func's
// owner rule) and R would only probe it to skip it.
__device__ __forceinline__ bool r2_lists(uint8_t s0, uint8_t s1, int32_t x, int32_t u0,
                                         int32_t u1) {
  return s0 != kArcDead && s1 != kArcDead && !(s0 == kArcFront && x < u1) &&
         !(s1 == kArcFront && x < u0);
}

// r = 3 liveness bitmaps.  A triangle's bits in its root's alive bitmap are
// cleared after the round that peels it, so the AND of two alive rows lists
// only candidates whose two triangles through v1 were not peeled earlier.
// A triangle's frontier bits are set when it joins a frontier (the level
// advance that selects it, or the update pass whose decrement brings its
// count to the level): the next round's bound and expand passes can then
// tell which s-cliques another member of the frontier owns.  When its round
// ends (kMark = false) its bits leave the alive bitmaps, the apex alive bits
// and the frontier marks.  Positions come from the slot's loc word; bits of
// different triangles may share a word, hence the atomics.
template <bool kMark>
__device__ __forceinline__ void front_bits_one(const GraphView &g,
                                               const int32_t *__restrict__ v1s,
                                               const FastView &fx,
                                               const uint64_t *__restrict__ loc, uint32_t p) {
  const uint64_t lc = loc[p];
  const uint64_t ap = (lc >> kApexShift) & kApexMask;
  if (ap) {
    const uint64_t q = ap - 1, bit = 1ull << (q & 63);
    if (kMark) {
      atomicOr((unsigned long long *)&fx.front_apex[q >> 6], bit);
    } else {
      atomicAnd((unsigned long long *)&fx.alive_apex[q >> 6], ~bit);
      atomicAnd((unsigned long long *)&fx.front_apex[q >> 6], ~bit);
    }
  }
  if (!(lc >> 63)) return;  // root without a bitmap
  const int32_t v1 = v1s[p];
  const int d = (int)(g.rp[v1 + 1] - g.up[v1]);
  const int wd = (d + 63) >> 6;
  const int64_t i = (int64_t)(lc & 511u), j = (int64_t)((lc >> 9) & 511u);
  const uint64_t bi = 1ull << (i & 63), bj = 1ull << (j & 63);
  unsigned long long *fr = (unsigned long long *)(fx.front + fx.bm_off[v1]);
  if (kMark) {
    atomicOr(&fr[i * wd + (j >> 6)], bj);
    atomicOr(&fr[j * wd + (i >> 6)], bi);
  } else {
    unsigned long long *al = (unsigned long long *)(fx.alive + fx.bm_off[v1]);
    atomicAnd(&al[i * wd + (j >> 6)], ~bj);
    atomicAnd(&al[j * wd + (i >> 6)], ~bi);
    atomicAnd(&fr[i * wd + (j >> 6)], ~bj);
    atomicAnd(&fr[j * wd + (i >> 6)], ~bi);
  }
}

// Flush hook of the r = 3 update pass: an r-clique appended to the next
// frontier gets its frontier marks as it is written out (the marking half
// of front_bits_one, with only the pointers it needs).
struct FrontMark {
  const int64_t *rp, *up;
  const int32_t *v1;
  const uint64_t *bm_off, *loc;
  uint64_t *front, *front_apex;
  __device__ __forceinline__ void operator()(uint32_t p) const {
    GraphView g{};
    g.rp = rp;
    g.up = up;
    FastView fx{};
    fx.bm_off = bm_off;
    fx.front = front;
    fx.front_apex = front_apex;
    front_bits_one<true>(g, v1, fx, loc, p);
  }
};
using FrontAppender = WaveAppender<kAppendCap, FrontMark>;

// Position of the (n+1)-th set bit of m, n < popcount(m): a halving search
// on popcounts, the same six steps in every lane.
__device__ __forceinline__ uint32_t select_bit(uint64_t m, uint32_t n) {
  uint32_t pos = 0;
  uint32_t lo = (uint32_t)m;
  uint32_t c = (uint32_t)__popc(lo);
  if (n >= c) {
    n -= c;
    lo = (uint32_t)(m >> 32);
    pos = 32;
  }
#pragma unroll
  for (int w = 16; w >= 2; w >>= 1) {
    c = (uint32_t)__popc(lo & ((1u << w) - 1u));
    if (n >= c) {
      n -= c;
      lo >>= w;
      pos += (uint32_t)w;
    }
  }
  return pos + (n >= (lo & 1u) ? 1u : 0u);
}

// Bits of word w of a bitmap row at local positions < l.
__device__ __forceinline__ uint64_t below_mask(int64_t l, int w) {
  const int64_t lo = (int64_t)w * 64;
  if (l >= lo + 64) return ~0ull;
  if (l <= lo) return 0ull;
  return (1ull << (l - lo)) - 1ull;
}

// r = 3, x > v1: candidates whose s-clique another frontier triangle owns,
// i.e. {v1, v2, x} peeled now with v3 > x, or {v1, v3, x} with v2 > x.
__device__ __forceinline__ uint64_t owned_elsewhere(const uint64_t *__restrict__ fr, int64_t l2,
                                                    int64_t l3, int wd, int w) {
  return (fr[l2 * wd + w] & below_mask(l3, w)) | (fr[l3 * wd + w] & below_mask(l2, w));
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
    decode_key<R>(T, p, sl.key, Rv);
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

// ---------------------------------------------- r = 3 ranked table lookups
// A triangle (a < b < c) whose root a keeps a bitmap sits at seg[a] + the
// number of bitmap bits above the diagonal that precede bit (i, j) in
// row-major order, i and j the local indices of b and c in N+(a).  Roots
// without a bitmap are hashed.

// r = 3 record word (rloc): the local index of x in N+(v1) (bitmap part), or
// 0xFFFF; with an index, bits 14 and 15 flag {v1, v2, x} and {v1, v3, x} as
// frontier triangles (alive is implied: the expand pass listed x from the
// alive rows).
constexpr int kRlocFront2 = 14, kRlocFront3 = 15;
constexpr uint32_t kRlocIndex = 0x3FFFu;

struct RootRow {
  int64_t o;      // up[a]
  int d;          // |N+(a)|
  int wd;         // words per bitmap row
  uint64_t bmo;   // bitmap word offset
  uint64_t segb;  // first slot of a's segment
};

__device__ __forceinline__ RootRow root_row(const PeelArgs &a, const FastView &fx, int32_t v) {
  RootRow rr;
  rr.o = a.g.up[v];
  rr.d = (int)(a.g.rp[v + 1] - rr.o);
  rr.wd = (rr.d + 63) >> 6;
  rr.bmo = rr.d <= 512 ? fx.bm_off[v] : 0;
  rr.segb = a.T.seg[v];
  return rr;
}

// bits of word w of a row strictly above local position i
__device__ __forceinline__ uint64_t bits_above(int64_t i, int w) {
  const int64_t lo = (int64_t)w * 64;
  if (i < lo) return ~0ull;
  if (i >= lo + 63) return 0ull;
  return ~((1ull << (i - lo + 1)) - 1ull);
}

// slot of (root, row i, column j), i < j, in a bitmap root's ranked segment
__device__ __forceinline__ int64_t ranked_pos(const FastView &fx, const RootRow &rr, int64_t i,
                                              int64_t j) {
  const uint64_t *row = fx.bm + rr.bmo + (uint64_t)i * rr.wd;
  uint64_t rank = fx.rowpre[rr.o + i];
  for (int w = (int)((i + 1) >> 6); w <= (int)(j >> 6); w++) {
    const int64_t lo = (int64_t)w * 64;
    const uint64_t below = j >= lo + 64 ? ~0ull : ((1ull << (j - lo)) - 1ull);
    rank += (uint64_t)__popcll(row[w] & bits_above(i, w) & below);
  }
  return (int64_t)(rr.segb + rank);
}

// slot of the triangle (x0 < x1 < x2), or -1; l1, l2 are the local indices
// of x1 and x2 in N+(x0) when known (else -1)
__device__ __forceinline__ int64_t tri_slot(const PeelArgs &a, const FastView &fx,
                                            const RootRow &rr, int32_t x0, int32_t x1, int32_t x2,
                                            int64_t l1, int64_t l2) {
  if (rr.d > 512) {
    const int32_t Tv[3] = {x0, x1, x2};
    Slot tmp;
    return table_find<false>(a.T, x0, x1, make_key<3>(Tv, a.T.bits), &tmp);
  }
  if (l1 < 0 && l2 < 0) {
    const int32_t ys[2] = {x1, x2};
    int64_t at[2];
    lower_bounds<2>(a.g.col, rr.o, rr.o + rr.d, ys, at);
    if (at[0] >= rr.o + rr.d || a.g.col[at[0]] != x1 || at[1] >= rr.o + rr.d ||
        a.g.col[at[1]] != x2)
      return -1;
    l1 = at[0] - rr.o;
    l2 = at[1] - rr.o;
  } else if (l1 < 0 || l2 < 0) {  // one of them known
    const int32_t y = l1 < 0 ? x1 : x2;
    const int64_t at = lower_pos(a.g.col, rr.o, rr.o + rr.d, y);
    if (at >= rr.o + rr.d || a.g.col[at] != y) return -1;
    (l1 < 0 ? l1 : l2) = at - rr.o;
  }
  return ranked_pos(fx, rr, l1, l2);
}

// Update-Func of the s-clique R + x for r = 3 on the ranked table: the same
// decisions as update_func, with the three other triangles located by rank
// (local indices of v2, v3 in N+(v1) come from R's loc word).  Called by every
// lane of the wave together.
// lxh: the record word (local index of x in N+(v1) and frontier flags when
// the expand pass had them, else 0xFFFF); l23: local index of v3 in N+(v2)
// (else 0xFFFFFFFF).
// The expand pass already decided the two triangles through v1 and x
// (omitting v2 or v3) whenever x came from v1's alive rows (x > v1, flags in
// lxh) or from the apex lists (x < v1: both alive and outside the frontier):
// their slots are not read, and a live one takes its decrement without the
// count check.  Only the triangle omitting v1 is read.
__device__ __forceinline__ void update_r3_ranked(const PeelArgs &a, const FastView &fx,
                                                 const int32_t (&Rv)[3], int32_t x, uint64_t lc,
                                                 uint32_t lxh, uint32_t l23, bool active,
                                                 LaneStats &ls, FrontAppender &apf,
                                                 Appender &apl) {
  constexpr Combos<4, 3> cb{};
  int32_t Sv[4];
  uint32_t rmask = 0;
  {
    int at = 0;
#pragma unroll
    for (int i = 0; i < 3; i++) at += Rv[i] < x ? 1 : 0;
#pragma unroll
    for (int o = 0, i = 0; o < 4; o++) {
      if (o == at) {
        Sv[o] = x;
      } else {
        Sv[o] = Rv[i++];
        rmask |= 1u << o;
      }
    }
  }
  const int32_t v1 = Rv[0];
  RootRow r1{};
  int64_t l2 = -1, l3 = -1, lx = -1;
  if (active) {
    r1 = root_row(a, fx, v1);
    if (r1.d <= 512 && (lc >> 63)) {
      l2 = (int64_t)(lc & 511u);
      l3 = (int64_t)((lc >> 9) & 511u);
      if (x > v1) {
        if (lxh != 0xFFFFu) {
          lx = (int64_t)(lxh & kRlocIndex);
        } else {
          lx = lower_pos(a.g.col, r1.o, r1.o + r1.d, x) - r1.o;
          if (lx >= r1.d || a.g.col[r1.o + lx] != x) lx = -1;  // tri_slot searches again
        }
      }
    }
  }
  int self = 0;
  int64_t pos[4];
  bool want[4];
#pragma unroll
  for (int q = 0; q < 4; q++) {
    if (cb.mask[q] == rmask) self = q;
    want[q] = active && cb.mask[q] != rmask;
    pos[q] = -1;
    if (!want[q]) continue;
    const int32_t t0 = Sv[cb.idx[q][0]], t1 = Sv[cb.idx[q][1]], t2 = Sv[cb.idx[q][2]];
    if (t0 == v1) {
      const int64_t h1 = t1 == Rv[1] ? l2 : (t1 == Rv[2] ? l3 : lx);
      const int64_t h2 = t2 == Rv[1] ? l2 : (t2 == Rv[2] ? l3 : lx);
      pos[q] = tri_slot(a, fx, r1, t0, t1, t2, h1, h2);
    } else {
      const RootRow rr = root_row(a, fx, t0);
      // (v2, v3, x) rooted at v2: v3's local index in N+(v2) is known
      const int64_t h1 = (t0 == Rv[1] && t1 == Rv[2] && l23 != 0xFFFFFFFFu) ? (int64_t)l23 : -1;
      const int64_t h2 = (t0 == Rv[1] && t2 == Rv[2] && l23 != 0xFFFFFFFFu) ? (int64_t)l23 : -1;
      pos[q] = tri_slot(a, fx, rr, t0, t1, t2, h1, h2);
    }
  }
  // known[q]: 0 read the slot, 1 live, 2 in the frontier after R
  int known[4];
  const bool apex = x < v1;
  const bool flagged = !apex && lxh != 0xFFFFu;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    known[q] = 0;
    const uint32_t omit = rmask & ~(uint32_t)cb.mask[q];  // R's vertex missing from q
    const bool omits_v2 = omit != 0 && Sv[__builtin_ctz(omit)] == Rv[1];
    const bool omits_v3 = omit != 0 && Sv[__builtin_ctz(omit)] == Rv[2];
    if (apex && (omits_v2 || omits_v3)) known[q] = 1;
    if (flagged && omits_v3) known[q] = (lxh >> kRlocFront2) & 1u ? 2 : 1;  // {v1, v2, x}
    if (flagged && omits_v2) known[q] = (lxh >> kRlocFront3) & 1u ? 2 : 1;  // {v1, v3, x}
  }
  Slot sl[4];
  bool alive = active, other_owner = false, hot[4];  // as in update_func
  uint32_t n_live = 0;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    hot[q] = false;
    if (!want[q]) continue;
    if (pos[q] < 0) {
      ls.err |= kErrLookup;
      alive = false;
      continue;
    }
    if (known[q] == 1) {
      n_live++;
      hot[q] = true;
      continue;
    }
    if (known[q] == 2) continue;
    sl[q] = a.T.slots[pos[q]];
    const int32_t Tv[3] = {Sv[cb.idx[q][0]], Sv[cb.idx[q][1]], Sv[cb.idx[q][2]]};
    if (sl[q].key != make_key<3>(Tv, a.T.bits).lo) {  // the rank must land on the triangle
      ls.err |= kErrLookup;
      alive = false;
    } else if (sl[q].stamp < a.t) {
      alive = false;  // S was destroyed in an earlier round
    } else if (sl[q].stamp == a.t) {
      other_owner = other_owner || q < self;  // peeled with R and first in order
    } else {
      n_live++;
      hot[q] = sl[q].cnt > a.k;
    }
  }
  if (active) ls.disc++;
  const bool mine = alive && !other_owner;
  if (mine) ls.dec += n_live;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    bool want_append = false, want_low = false;
    if (mine && hot[q]) {
      const uint32_t old = __hip_atomic_fetch_add(&a.T.slots[pos[q]].cnt, 0xFFFFFFFFu,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      ls.atom++;
      want_append = old == a.k + 1;
      want_low = a.kw > a.k && old == a.kw + 1;
    }
    apf.push(want_append, (uint32_t)pos[q]);
    apl.push(want_low, (uint32_t)pos[q]);
  }
}

constexpr int kListCap = 1024;  // LDS entries per wave for a staged apex list

// position of x in the sorted LDS array a[0..n), or -1
__device__ __forceinline__ int lds_find(const int32_t *a, int n, int32_t x) {
  int lo = 0, hi = n;
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    const int32_t v = a[mid];
    if (v == x) return mid;
    if (v < x) lo = mid + 1;
    else hi = mid;
  }
  return -1;
}

__device__ __forceinline__ bool apex_alive(const uint64_t *__restrict__ bits, uint64_t q) {
  return (bits[q >> 6] >> (q & 63)) & 1ull;
}

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

// What the expand pass needs of a peeled r-clique, written by the bound pass
// so that expand starts from one load instead of re-deriving it.
struct ExpandDesc {
  uint64_t o;      // up[v1]: N+(v1) = col[o, o + d)
  uint64_t bmo;    // word offset of v1's bitmap (d <= 512)
  uint64_t lb;     // first entry of the driving apex list
  uint64_t ob;     // r = 3: first entry of the other apex list
  uint32_t d;      // |N+(v1)|
  uint32_t len2;   // driving list length
  uint32_t olen;   // r = 3: other list length
  uint32_t drv;    // 1..r-1: the member whose arc (v1, v_drv) drives
  uint32_t l[5];   // local indices of v2..vr in N+(v1)
  uint32_t pad;
};

// Also stamps A_t with t (the apply pass of the same round reads the stamps)
// and allocates each r-clique's record range with one atomic per block.
template <int R>
__global__ __launch_bounds__(256) void k_expand_bound(PeelArgs base, RoundCtl *rc, FastView fx,
                                                      const uint64_t *__restrict__ loc,
                                                      uint64_t *off, uint32_t *len, int32_t *fv,
                                                      ExpandDesc *desc, uint32_t *f23) {
  if (rc_idle(rc)) return;
  const PeelArgs a = round_args(base, rc);
  const uint32_t *__restrict__ F = rc->F;
  const uint32_t nF = rc->nF;
  for (int64_t f0 = (int64_t)blockIdx.x * 256; f0 < nF; f0 += (int64_t)gridDim.x * 256) {
    const int64_t f = f0 + threadIdx.x;
    uint64_t bound = 0;
    if (f < nF) {
    const uint32_t p = F[f];
    const Slot sl = a.T.slots[p];
    a.T.slots[p].stamp = a.t;
    int32_t Rv[R];
    Rv[0] = a.T.v1[p];
    decode_key<R>(a.T, p, sl.key, Rv);
#pragma unroll
    for (int i = 0; i < R; i++) fv[f * R + i] = Rv[i];
    if constexpr (R == 2)  // frontier edges are marked for this round's expand pass
      if (fx.arcst) set_edge_state(a.g, Rv[0], Rv[1], fx.arcst, kArcFront);
    if (sl.cnt != 0) {  // otherwise every s-clique of R is already gone
      const int64_t o = a.g.up[Rv[0]];
      const int d = (int)(a.g.rp[Rv[0] + 1] - o);
      int64_t e[R];
      if (front_positions<R>(a, loc[p], Rv, o, d, e)) {
        uint64_t total1 = 0;
        if (d <= 512) {
          const int wd = (d + 63) >> 6;
          const uint64_t *rows =
              (R == 3 || (R == 2 && fx.alive) ? fx.alive : fx.bm) + fx.bm_off[Rv[0]];
          for (int w = 0; w < wd; w++) {
            uint64_t x = ~0ull;
#pragma unroll
            for (int i = 1; i < R; i++) x &= rows[(e[i] - o) * wd + w];
            if constexpr (R == 3)
              x &= ~owned_elsewhere(fx.front + fx.bm_off[Rv[0]], e[1] - o, e[2] - o, wd, w);
            total1 += (uint64_t)__popcll(x);
          }
        } else {
          total1 = (uint64_t)d;
        }
        int drv = 1;
        uint64_t len2 = (R == 2 && fx.llen) ? fx.llen[e[1]] : fx.lptr[e[1] + 1] - fx.lptr[e[1]];
#pragma unroll
        for (int i = 2; i < R; i++) {
          const uint64_t len = fx.lptr[e[i] + 1] - fx.lptr[e[i]];
          if (len < len2) {
            len2 = len;
            drv = i;
          }
        }
        bound = total1 + len2;
        ExpandDesc ds;
        ds.o = (uint64_t)o;
        ds.bmo = d <= 512 ? fx.bm_off[Rv[0]] : 0;
        ds.lb = fx.lptr[e[drv]];
        ds.d = (uint32_t)d;
        ds.len2 = (uint32_t)len2;
        ds.drv = (uint32_t)drv;
        ds.ob = 0;
        ds.olen = 0;
        if constexpr (R == 3) {
          const int other = drv == 1 ? 2 : 1;
          ds.ob = fx.lptr[e[other]];
          ds.olen = (uint32_t)(fx.lptr[e[other] + 1] - ds.ob);
        }
#pragma unroll
        for (int i = 0; i < 5; i++) ds.l[i] = i + 1 < R ? (uint32_t)(e[i + 1] - o) : 0u;
        ds.pad = 0;
        desc[f] = ds;
        if constexpr (R == 3) {  // v3's place in N+(v2), for the triangles (v2, v3, x)
          const int64_t o2 = a.g.up[Rv[1]];
          const int64_t d2 = a.g.rp[Rv[1] + 1] - o2;
          uint32_t l = 0xFFFFFFFFu;
          if (d2 <= 512) {
            const int64_t at = lower_pos(a.g.col, o2, o2 + d2, Rv[2]);
            if (at < o2 + d2 && a.g.col[at] == Rv[2]) l = (uint32_t)(at - o2);
          }
          f23[f] = l;
        }
      } else {
        atomicOr(&a.ctr->err, kErrLookup);
      }
    }
    }
    const uint64_t at = block_alloc(bound, (unsigned long long *)&rc->total);
    if (f < nF) {
      off[f] = at;
      len[f] = (uint32_t)bound;
    }
  }
}

template <int R>
// 8 waves per SIMD: the pass is a chain of dependent loads per wave, and the
// occupancy hides them (measured ~2% of a rMAT-18 (3,4) decomposition over
// the default 6)
__global__ __launch_bounds__(256, 8) void k_expand(PeelArgs base, RoundCtl *rc, FastView fx,
                                                const ExpandDesc *__restrict__ desc,
                                                const uint64_t *__restrict__ off,
                                                const uint32_t *__restrict__ len,
                                                const int32_t *__restrict__ fv, int2 *rec,
                                                uint16_t *rloc) {
  if (rc_idle(rc)) return;
  if (rc->total > rc->cap) {  // records do not fit: the host grows the buffer, reruns the round
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      rc->need = rc->total;
      rc->halt = 1;
    }
    return;
  }
  const PeelArgs a = round_args(base, rc);
  const uint32_t *__restrict__ F = rc->F;
  const uint32_t nF = rc->nF;
  const int wpb = blockDim.x / kWave;
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  __shared__ int32_t lbuf[256 / kWave][R == 3 ? kListCap + 1 : 1];  // padded: see k_count_group
  for (int64_t f = (int64_t)blockIdx.x * wpb + wv; f < nF; f += (int64_t)gridDim.x * wpb) {
    const uint64_t b = off[f];
    const uint64_t total = len[f];
    if (total == 0) continue;
    const ExpandDesc ds = desc[f];
    const int64_t o = (int64_t)ds.o;
    const int d = (int)ds.d;
    int64_t e[R];
#pragma unroll
    for (int i = 1; i < R; i++) e[i] = o + (int64_t)ds.l[i - 1];
    const bool has_bm = d <= 512;
    uint32_t total1, iw[8];
    uint64_t cw = 0;
    uint64_t fw2 = 0, fw3 = 0;  // r = 3: frontier marks of rows v2, v3 (this lane's word)
    if (has_bm) {
      const int wd = (d + 63) >> 6;
      const uint64_t *rows = (R == 3 || (R == 2 && fx.alive) ? fx.alive : fx.bm) + ds.bmo;
      if (lane < wd) {
        cw = ~0ull;
#pragma unroll
        for (int i = 1; i < R; i++) cw &= rows[(e[i] - o) * wd + lane];
        if constexpr (R == 3) {
          const int64_t l2 = e[1] - o, l3 = e[2] - o;
          fw2 = fx.front[ds.bmo + l2 * wd + lane];
          fw3 = fx.front[ds.bmo + l3 * wd + lane];
          // a frontier triangle {v1, v2, x} or {v1, v3, x} before R owns R + x
          cw &= ~((fw2 & below_mask(l3, lane)) | (fw3 & below_mask(l2, lane)));
        }
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
    const int drv = (int)ds.drv;
    const uint64_t len2 = ds.len2;
    const uint64_t lb = ds.lb;
    int staged_len = -1;
    uint64_t ob = 0, oe = 0;
    if constexpr (R == 3) {
      ob = ds.ob;
      oe = ds.ob + ds.olen;
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
      uint64_t fr2 = 0, fr3 = 0;
      if constexpr (R == 3) {
        fr2 = __shfl(fw2, w);
        fr3 = __shfl(fw3, w);
      }
      uint32_t lxw = 0xFFFFu;  // local index of x in N+(v1), bitmap part only
      if (in && k < total1) {
        if (has_bm) {
          const uint32_t bit = select_bit(wordw, kk - before);
          lxw = (uint32_t)w * 64u + bit;
          x = a.g.col[o + lxw];
          // r = 3: {v1, v2, x} and {v1, v3, x} are alive (the alive rows); a
          // frontier one comes after R and owns nothing: its flag tells the
          // update pass, which then needs neither triangle's slot
          if constexpr (R == 3)
            lxw |= (uint32_t)((fr2 >> bit) & 1u) << kRlocFront2 |
                   (uint32_t)((fr3 >> bit) & 1u) << kRlocFront3;
        } else {
          x = a.g.col[o + (int64_t)k];
          if constexpr (R != 2) {
#pragma unroll
            for (int i = 1; i < R; i++) in = in && adjacent(a.g, x, fv[f * R + i]);
          }
        }
        if constexpr (R == 2) {  // x > v1: edge {v1,x} at its place in N+(v1)
          const int32_t v1 = fv[f * 2], v2 = fv[f * 2 + 1];
          const int64_t e1 = o + (int64_t)(has_bm ? lxw : (uint32_t)k);
          const int64_t e2 = arc_pos(a.g, v2, x);
          in = in && e2 >= 0;
          if (in && fx.arcst) in = r2_lists(fx.arcst[e1], fx.arcst[e2], x, v1, v2);
        }
      } else if (in) {
        const uint64_t q1 = lb + (k - total1);
        x = (R == 2 && fx.lvr) ? fx.lvr[q1] : fx.lval[q1];
        if constexpr (R == 2) {  // x < v1: both edges sit in N+(x)
          if (fx.arcst) {
            const int32_t v1 = fv[f * 2], v2 = fv[f * 2 + 1];
            const int64_t e1 = arc_pos(a.g, x, v1), e2 = arc_pos(a.g, x, v2);
            in = e1 >= 0 && e2 >= 0 && r2_lists(fx.arcst[e1], fx.arcst[e2], x, v1, v2);
          }
        }
        if constexpr (R == 3) {
          // x < v1: S = {x, v1, v2, v3}; the triangles {x, v1, v2} and {x, v1, v3}
          // are the apex entries at q1 and at x's place in the other list
          int64_t q2 = -1;
          if (staged_len >= 0) {
            const int at = lds_find(lbuf[wv], staged_len, x);
            q2 = at >= 0 ? (int64_t)ob + at : -1;
          } else {
            const int64_t at = lower_pos(fx.lval, (int64_t)ob, (int64_t)oe, x);
            q2 = at < (int64_t)oe && fx.lval[at] == x ? at : -1;
          }
          // both triangles still alive, and neither peeled now (it would own S)
          in = q2 >= 0 && apex_alive(fx.alive_apex, q1) && apex_alive(fx.alive_apex, (uint64_t)q2) &&
               !apex_alive(fx.front_apex, q1) && !apex_alive(fx.front_apex, (uint64_t)q2);
        } else {
#pragma unroll
          for (int i = 1; i < R; i++)
            if (i != drv)
              in = in && sorted_contains(fx.lval, fx.lptr[e[i]], fx.lptr[e[i] + 1], x);
        }
      }
      if (k < total) {
        rec[b + k] = make_int2((int)f, in ? x : -1);
        if constexpr (R == 3) rloc[b + k] = (uint16_t)lxw;
      }
    }
    __builtin_amdgcn_wave_barrier();
  }
}

template <int R>
__device__ __forceinline__ void apply_body(const PeelArgs &base, const RoundCtl *__restrict__ rc,
                                               const int2 *__restrict__ rec,
                                               const int32_t *__restrict__ fv, FastView fx,
                                               const uint64_t *__restrict__ loc,
                                               const uint16_t *__restrict__ rloc,
                                               const uint32_t *__restrict__ f23,
                                               uint32_t (*abuf_mem)[2][kAppendCap]) {
  const PeelArgs a = round_args(base, rc);
  const uint32_t *__restrict__ F = rc->F;
  const uint64_t total = rc->total;
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  LaneStats ls;
  uint32_t(*abuf)[2][kAppendCap] = abuf_mem;
  // wave-uniform trip count: every lane reaches every append
  auto each_record = [&](auto &&update) {
    for (uint64_t b0 = ((uint64_t)blockIdx.x * blockDim.x) + (uint64_t)wv * kWave; b0 < total;
         b0 += (uint64_t)gridDim.x * blockDim.x) {
      const uint64_t i = b0 + lane;
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
      update(Rv, in, rc, p, i);
    }
  };
  if constexpr (R == 3) {  // r = 3 plans keep the ranked table and the frontier marks
    FrontAppender apf{abuf[wv][0], 0u, a.Fnext, &a.ctr->next_size,
                      FrontMark{a.g.rp, a.g.up, a.T.v1, fx.bm_off, loc, fx.front,
                                fx.front_apex}};
    Appender apl{abuf[wv][1], 0u, a.Low, &a.ctr->low_size};
    each_record([&](const int32_t(&Rv)[R], bool in, int2 rc, uint32_t p, uint64_t i) {
      update_r3_ranked(a, fx, Rv, in ? rc.y : R, in ? loc[p] : 0ull, in ? rloc[i] : 0xFFFFu,
                       in ? f23[rc.x] : 0xFFFFFFFFu, in, ls, apf, apl);
    });
    apf.flush();
    apl.flush();
  } else {
    Appender ap[2] = {{abuf[wv][0], 0u, a.Fnext, &a.ctr->next_size},
                      {abuf[wv][1], 0u, a.Low, &a.ctr->low_size}};
    each_record([&](const int32_t(&Rv)[R], bool in, int2 rc, uint32_t p, uint64_t) {
      peel_candidate<R>(a, Rv, in ? rc.y : R, in, p, ls, ap);
    });
    ap[0].flush();
    ap[1].flush();
  }
  stat_add(a.stats, kStatDec, ls.dec);
  stat_add(a.stats, kStatDisc, ls.disc);
  stat_add(a.stats, kStatAtom, ls.atom);
  if (ls.err) atomicOr(&a.ctr->err, ls.err);
}

// r = 4: at least 4 waves per SIMD.  (Before the paired early-exit lookups
// the compiler took 133 registers and 3 waves without the bound, ~60 ms
// slower per Chung-Lu 1M (4,5) decomposition; the pass now fits 92 registers
// and 5 waves.)  r = 5, 6 keep the default (the bound spilled their larger
// subset arrays).
template <int R>
__global__ __launch_bounds__(256, R == 4 ? 4 : 1) void k_apply(PeelArgs base, const RoundCtl *__restrict__ rc,
                                               const int2 *__restrict__ rec,
                                               const int32_t *__restrict__ fv, FastView fx,
                                               const uint64_t *__restrict__ loc,
                                               const uint16_t *__restrict__ rloc,
                                               const uint32_t *__restrict__ f23) {
  if (rc_idle(rc)) return;
  __shared__ uint32_t abuf[256 / kWave][2][kAppendCap];
  apply_body<R>(base, rc, rec, fv, fx, loc, rloc, f23, abuf);
}

// r = 3: at least 6 waves per SIMD.  The ranked lookups need more registers
// than that allows by default, and the occupancy hides their dependent loads
// (measured: 5 waves 391 ms, 6 waves 376 ms, 8 waves with spills 434 ms per
// rMAT-18 (3,4) decomposition).  Other r keep the default (their larger
// subset arrays would spill).
// It also retires the frontier: its triangles leave the liveness bitmaps and
// frontier marks (no pass of the round reads them after expand).  The
// round's bookkeeping stays in k_round_end: a block-arrival counter over
// this kernel's thousands of blocks cost more than the launch it saves.
__global__ __launch_bounds__(256, 6) void k_apply3(PeelArgs base, const RoundCtl *rc,
                                                   const int2 *__restrict__ rec,
                                                   const int32_t *__restrict__ fv, FastView fx,
                                                   const uint64_t *__restrict__ loc,
                                                   const uint16_t *__restrict__ rloc,
                                                   const uint32_t *__restrict__ f23) {
  if (rc_idle(rc)) return;
  __shared__ uint32_t abuf[256 / kWave][2][kAppendCap];
  apply_body<3>(base, rc, rec, fv, fx, loc, rloc, f23, abuf);
  const uint32_t *__restrict__ F = rc->F;
  const uint32_t nF = rc->nF;
  for (int64_t it = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; it < nF;
       it += (int64_t)gridDim.x * blockDim.x)
    front_bits_one<false>(base.g, base.T.v1, fx, loc, F[it]);
}

// Direct count, 8 lanes per r-clique (r >= 3), eight r-cliques per wave: the
// part x > v1 is a popcount of the AND of v1's bitmap rows (at most 8 words,
// d <= 512); the part x < v1 is the intersection of the apex lists, the
// shortest one split across the group's lanes and, for r = 3, the other one
// staged in the group's LDS share.  Most apex lists are short, so a whole
// wave per r-clique left most lanes idle (measured on rMAT-18 (3,4): 50 ms
// with a wave, 32 ms with 16 lanes, 30 ms with 8).
// (The expand pass keeps a whole wave per r-clique: its record loop ran
// slower with 32 or 16 lanes.)
constexpr int kCountGroup = 8;
constexpr int kGroupList = kListCap * kCountGroup / kWave;

template <int R>
__global__ __launch_bounds__(256) void k_count_group(PeelArgs a, FastView fx,
                                                     const uint64_t *__restrict__ loc,
                                                     const uint32_t *__restrict__ occ,
                                                     uint64_t n_r) {
  constexpr int G = kCountGroup;
  const int gpb = blockDim.x / G;
  const int gi = threadIdx.x / G;
  const int gl = threadIdx.x % G;
  // one word of padding per group's share: the groups' binary searches start
  // at similar midpoints, and unpadded shares 128 words apart put them in the
  // same LDS bank (2.1 conflict cycles per LDS instruction measured)
  __shared__ int32_t lbuf[256 / G][R == 3 ? kGroupList + 1 : 1];
  for (int64_t it = (int64_t)blockIdx.x * gpb + gi; it < (int64_t)n_r;
       it += (int64_t)gridDim.x * gpb) {  // group-uniform
    const uint32_t p = occ[it];
    const Slot sl = a.T.slots[p];
    int32_t Rv[R];
    Rv[0] = a.T.v1[p];
    decode_key<R>(a.T, p, sl.key, Rv);
    const int64_t o = a.g.up[Rv[0]];
    const int d = (int)(a.g.rp[Rv[0] + 1] - o);
    int64_t e[R];
    if (!front_positions<R>(a, loc[p], Rv, o, d, e)) {  // group-uniform
      if (gl == 0) atomicOr(&a.ctr->err, kErrLookup);
      continue;
    }
    uint32_t c = 0;
    if (d <= 512) {
      const int wd = (d + 63) >> 6;
      const uint64_t *rows = fx.bm + fx.bm_off[Rv[0]];
      if (gl < wd) {
        uint64_t x = ~0ull;
#pragma unroll
        for (int i = 1; i < R; i++) x &= rows[(e[i] - o) * wd + gl];
        c = (uint32_t)__popcll(x);
      }
    } else {
      for (int64_t j = o + gl; j < o + d; j += G) {
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
      const int other = 3 - drv;
      ob = fx.lptr[e[other]];
      oe = fx.lptr[e[other] + 1];
      if (len2 > 0 && oe - ob <= (uint64_t)kGroupList) {
        staged_len = (int)(oe - ob);
        for (int i = gl; i < staged_len; i += G) lbuf[gi][i] = fx.lval[ob + i];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
      }
    }
    for (uint64_t j = gl; j < len2; j += G) {
      const int32_t x = fx.lval[lb + j];
      bool in = true;
      if constexpr (R == 3) {
        in = staged_len >= 0 ? lds_contains(lbuf[gi], staged_len, x)
                             : sorted_contains(fx.lval, ob, oe, x);
      } else {
#pragma unroll
        for (int i = 1; i < R; i++)
          if (i != drv) in = in && sorted_contains(fx.lval, fx.lptr[e[i]], fx.lptr[e[i] + 1], x);
      }
      c += in ? 1u : 0u;
    }
#pragma unroll
    for (int off = G / 2; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if (gl == 0) a.T.slots[p].cnt = c;
    __builtin_amdgcn_wave_barrier();
  }
}

// Local indices of v2..vr in N+(v1) for every occupied slot of a bitmap
// root (9 bits each, bit 63 marks them valid).  For r = 3 bits 18..61 also
// hold 1 + the position of the triangle's apex entry (v1 in the list of the
// arc (v2, v3)), 0 if it has none.

template <int R>
__global__ void k_make_loc(GraphView g, TableView T, FastView fx, uint64_t n_slots,
                           uint64_t *loc) {
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < (int64_t)n_slots;
       p += (int64_t)gridDim.x * blockDim.x) {
    const Slot sl = T.slots[p];
    uint64_t v = 0;
    if (sl.key != 0) {
      int32_t Rv[R];
      Rv[0] = T.v1[p];
      decode_key<R>(T, p, sl.key, Rv);
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
      if constexpr (R == 3) {
        const int64_t arc = lower_pos(g.col, g.up[Rv[1]], g.rp[Rv[1] + 1], Rv[2]);
        const int64_t lb = (int64_t)fx.lptr[arc], le = (int64_t)fx.lptr[arc + 1];
        const int64_t q = lower_pos(fx.lval, lb, le, Rv[0]);
        if (q < le && fx.lval[q] == Rv[0]) v |= (((uint64_t)q + 1) & kApexMask) << kApexShift;
      }
    }
    loc[p] = v;
  }
}

// ---------------------------------------------------------- round control
// The first round the host queues after reading the state is
//   k_adv_min, k_adv_partition
//       level advance (B.next_bucket of Algorithm 2), queued when the round
//       starts with an empty frontier, on grids sized to the list;
//   k_round_begin            one thread: finishes an advance (or drops a
//                            window list of peeled entries), then the
//                            round's lists and counters;
//   the update passes of the path (the first one stamps A_t with t);
//   k_round_end              one thread: trace, finished += |A_t|, next
//                            frontier; over the grid, when another round
//                            is queued behind it and the next frontier is
//                            empty, the minimum of that round's advance.
// A round queued behind others starts with k_advance_begin instead: the
// partition by that minimum, if its frontier is empty, and k_round_begin's
// work in one launch on a small grid.
// Every kernel returns at once once the peel has finished or halted, so the
// host may queue rounds past the last one and read the state only now and
// then.

__global__ void k_stamp(const RoundCtl *__restrict__ rc, Slot *slots) {
  if (rc_idle(rc)) return;
  const uint32_t *__restrict__ F = rc->F;
  const uint32_t nF = rc->nF, t = rc->t;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nF;
       i += (int64_t)gridDim.x * blockDim.x)
    slots[F[i]].stamp = t;
}

// Minimum count over the live entries of the window list (nW entries), or
// of the high list when the window list is empty.  Recomputing it gives the
// same value as long as no count changes (atomicMin).
__device__ __forceinline__ void adv_min_body(RoundCtl *rc, const Slot *__restrict__ slots,
                                             uint32_t nW) {
  const bool win = nW != 0;
  const uint32_t *__restrict__ L = win ? rc->bufW[rc->selW] : rc->bufH[rc->selH];
  const uint32_t nL = win ? nW : rc->nH;
  uint32_t m = kNone;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nL;
       i += (int64_t)gridDim.x * blockDim.x) {
    const Slot s = slots[L[i]];
    if (s.stamp == kLive && s.cnt < m) m = s.cnt;
  }
  m = wave_min_u32(m);
  if (lane_id() == 0 && m != kNone) atomicMin(win ? &rc->mw : &rc->mh, m);
}

__global__ __launch_bounds__(256) void k_adv_min(RoundCtl *rc, const Slot *__restrict__ slots) {
  if (rc_idle(rc) || rc->nF != 0) return;
  adv_min_body(rc, slots, rc->nW);
}

// Three-way partition of the list the advance works on, by count c:
// c <= k -> the frontier, k < c <= kw -> the window list, c > kw -> the
// high list; peeled entries are dropped.  Inside the window (kw = max) the
// window list is compacted into its other buffer; when a new window is
// opened the high list is split.  Each block compacts a tile of 256 x 16
// entries with one atomic per output per tile (a single global counter per
// wave would serialise in L2).  With mark (r = 3 on the s = r+1 path) the
// new frontier's triangles get their frontier marks.
constexpr int kPartThreads = 256;
constexpr int kPartItems = 16;

__device__ __forceinline__ void partition_body(RoundCtl *rc, const Slot *__restrict__ slots,
                                               bool win, uint32_t mn, bool mark,
                                               const GraphView &g,
                                               const int32_t *__restrict__ v1s,
                                               const FastView &fx,
                                               const uint64_t *__restrict__ loc) {
  const uint32_t k = rc->k > mn ? rc->k : mn;
  const uint32_t kw = win ? 0xFFFFFFFEu : window_top(k, rc->wlev);
  const uint32_t *__restrict__ L = win ? rc->bufW[rc->selW] : rc->bufH[rc->selH];
  const uint32_t nL = win ? rc->nW : rc->nH;
  uint32_t *F = rc->bufF[rc->selF];
  uint32_t *Lo = win ? rc->bufW[rc->selW ^ 1u] : rc->bufW[rc->selW];
  uint32_t *Hi = rc->bufH[rc->selH ^ 1u];
  uint32_t *ctr3[3] = {&rc->cF, &rc->cW, &rc->cH};
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
      base[tid] = tot ? atomicAdd(ctr3[tid], tot) : 0u;
    }
    __syncthreads();
    uint32_t at[3];
#pragma unroll
    for (int q = 0; q < 3; q++) at[q] = base[q] + wsum[q][w] + incl[q] - cnt[q];
#pragma unroll
    for (int j = 0; j < kPartItems; j++) {
      if (m[0] >> j & 1u) {
        F[at[0]++] = p[j];
        if (mark) front_bits_one<true>(g, v1s, fx, loc, p[j]);
      }
      if (m[1] >> j & 1u) Lo[at[1]++] = p[j];
      if (m[2] >> j & 1u) Hi[at[2]++] = p[j];
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kPartThreads) void k_adv_partition(
    RoundCtl *rc, const Slot *__restrict__ slots, bool mark, GraphView g,
    const int32_t *__restrict__ v1s, FastView fx, const uint64_t *__restrict__ loc) {
  if (rc_idle(rc) || rc->nF != 0) return;
  const bool win = rc->nW != 0;
  const uint32_t mn = win ? rc->mw : rc->mh;
  if (mn == kNone) return;  // round_begin_body drops the window or reports the error
  partition_body(rc, slots, win, mn, mark, g, v1s, fx, loc);
}

__global__ void k_round_begin(RoundCtl *rc, Counters *dc) {
  if (rc_idle(rc)) return;
  round_begin_body(rc, dc);
}

// Level advance and start of a round in one launch, for rounds queued behind
// others (every block's fence and count is cheap only on their small grids:
// on grids of thousands of blocks it cost more than the launch it saves).
// Without an advance
// (frontier not empty) block 0 starts the round at once: round_begin_body
// then leaves nF, done and halt as the other blocks read them (halt 2 only
// makes them return, as they do anyway).  With an advance every block
// partitions its tiles and counts itself done; the last one, after a fence,
// finishes the advance and starts the round.  Every block reads the state it
// branches on before it counts itself, so no block sees the last one's
// writes.  No block waits for another.
__global__ __launch_bounds__(kPartThreads) void k_advance_begin(
    RoundCtl *rc, Counters *dc, const Slot *__restrict__ slots, bool mark, GraphView g,
    const int32_t *__restrict__ v1s, FastView fx, const uint64_t *__restrict__ loc) {
  if (rc_idle(rc)) return;
  if (rc->nF != 0) {
    if (blockIdx.x == 0 && threadIdx.x == 0) round_begin_body(rc, dc);
    return;
  }
  const bool win = rc->nW != 0;
  const uint32_t mn = win ? rc->mw : rc->mh;
  // mn == kNone: round_begin_body drops the window or reports the error
  if (mn != kNone) partition_body(rc, slots, win, mn, mark, g, v1s, fx, loc);
  __shared__ uint32_t last;
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    last = atomicAdd(&rc->ndone, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (last && threadIdx.x == 0) {
    __threadfence();
    rc->ndone = 0;
    round_begin_body(rc, dc);
  }
}

// Over the grid of a round's end that another queued round follows (the
// first round the host queues after reading the state runs k_adv_min on a
// grid sized to the list instead): when the next frontier is empty, the
// minimum its level advance partitions by.  Every block decides from the
// round's counters, which the bookkeeping of round_end_body leaves alone:
// the next frontier holds next_size entries (zero after an empty round) and
// the window list low_size.
__device__ __forceinline__ void end_min(RoundCtl *rc, const Counters *dc,
                                        const Slot *__restrict__ slots) {
  if (dc->next_size != 0) return;
  adv_min_body(rc, slots, dc->low_size);
}

__global__ __launch_bounds__(256) void k_round_end(RoundCtl *rc, const Counters *dc,
                                                   const Slot *__restrict__ slots,
                                                   uint32_t min_next) {
  if (rc_idle(rc)) return;
  if (blockIdx.x == 0 && threadIdx.x == 0) round_end_body(rc, dc);
  if (min_next) end_min(rc, dc, slots);
}

// r = 2, end of a round: the bookkeeping and the next advance's minimum as
// in k_round_end and, over the grid, the frontier's edges becoming dead for the candidate tests
// of later rounds (both arc directions), counted as lost neighbours of both
// endpoints when graph contraction is on (lost non-null).  The retirement
// reads the round's |A_t| from nA, which the bookkeeping leaves alone.
__global__ __launch_bounds__(256) void k_round_end_r2(RoundCtl *rc, const Counters *dc,
                                                      const Slot *__restrict__ slots,
                                                      uint32_t min_next, GraphView g,
                                                      const int32_t *__restrict__ fv,
                                                      uint8_t *arcst, uint32_t *lost) {
  if (rc_idle(rc)) return;
  const uint32_t nA = rc->nA;
  if (blockIdx.x == 0 && threadIdx.x == 0) round_end_body(rc, dc);
  if (min_next) end_min(rc, dc, slots);
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < nA;
       f += (int64_t)gridDim.x * blockDim.x) {
    const int32_t a = fv[f * 2], b = fv[f * 2 + 1];
    set_edge_state(g, a, b, arcst, kArcDead);
    if (lost) {
      atomicAdd(&lost[a], 1u);
      atomicAdd(&lost[b], 1u);
    }
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
    decode_key<R>(T, p, s.key, v);
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
//   bound:  thread per peeled R: stamp it, pick the driver, allocate one
//           flag per position of the driver's row;
//   spread: wave per peeled R: its index over its candidate range;
//   member: thread per candidate: flag the positions in I(R), list the
//           members that have out-arcs;
//   apply:  the out-arcs (x, y) of 64 members spread over a wave: y in I(R)
//           closes R + {x, y} (s = r + 2) or starts a deeper extension.

template <int R>
__global__ __launch_bounds__(256) void k_gen_bound(PeelArgs base, RoundCtl *rc, uint64_t *ioff,
                                                   uint32_t *ilen, int32_t *fv, int32_t *drv,
                                                   uint8_t *arcst) {
  if (rc_idle(rc)) return;
  const PeelArgs a = round_args(base, rc);
  const uint32_t *__restrict__ F = rc->F;
  const uint32_t nF = rc->nF;
  for (int64_t f0 = (int64_t)blockIdx.x * 256; f0 < nF; f0 += (int64_t)gridDim.x * 256) {
    const int64_t f = f0 + threadIdx.x;
    uint64_t bound = 0;
    if (f < nF) {
      const uint32_t p = F[f];
      const Slot sl = a.T.slots[p];
      a.T.slots[p].stamp = a.t;
      int32_t Rv[R];
      Rv[0] = a.T.v1[p];
      decode_key<R>(a.T, p, sl.key, Rv);
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
      bound = sl.cnt != 0 ? (uint64_t)best : 0;  // cnt 0: every s-clique of R is gone
      if constexpr (R == 2) set_edge_state(a.g, Rv[0], Rv[1], arcst, kArcFront);
    }
    const uint64_t at = block_alloc(bound, (unsigned long long *)&rc->total);
    if (f < nF) {
      ioff[f] = at;
      ilen[f] = (uint32_t)bound;
    }
  }
}

// One wave per peeled r-clique writes its index over its candidate range, so
// the member pass can be flattened over all candidates of the round.  (Done
// by the bound pass's own blocks instead, the writes of a round with a few
// hundred r-cliques fell to four waves: the Chung-Lu 1M (2,4) peel took 15%
// longer.)
__global__ __launch_bounds__(256) void k_gen_spread(RoundCtl *rc, const uint64_t *__restrict__ ioff,
                                                    const uint32_t *__restrict__ ilen,
                                                    uint32_t *owner) {
  if (rc_idle(rc)) return;
  if (rc->total > rc->cap) {  // candidates do not fit: the host grows the buffers, reruns
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      rc->need = rc->total;
      rc->halt = 1;
    }
    return;
  }
  const uint32_t nF = rc->nF;
  const int wpb = blockDim.x / kWave;
  for (int64_t f = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; f < nF;
       f += (int64_t)gridDim.x * wpb) {
    const uint32_t len = ilen[f];
    const uint64_t fb = ioff[f];
    for (uint32_t c = lane_id(); c < len; c += kWave) owner[fb + c] = (uint32_t)f;
  }
}

// A thread per candidate x of the round: flag x when it lies in I(R) and
// list the members that have out-arcs as (frontier index, x).
// Candidates whose s-cliques with R are all gone or all owned by another
// frontier r-clique are left out: r = 1 by vertex stamps, r = 2 by edge
// states, r >= 3 by looking up the r-subsets of R + x through x.
// r = 2: arcst[e] says whether the edge of arc position e was peeled in an
// earlier round (dead) or is in this round's frontier.  A candidate x joins
// I(R), R = {u < v}, only if both its edges to R are alive (no s-clique
// destroyed earlier is listed again) and neither is a frontier edge that
// comes before R in the subset order of every s-clique containing R and x:
// {x,u} does when x < v, {x,v} when x < u.  Such an s-clique is owned by
// that edge (Update-Func's owner rule), so R would only probe it to skip it.
template <int R>
__global__ __launch_bounds__(256) void k_gen_member(GraphView g, RoundCtl *rc,
                                                    const uint64_t *__restrict__ ioff,
                                                    const uint32_t *__restrict__ owner,
                                                    const int32_t *__restrict__ fv,
                                                    const int32_t *__restrict__ drv, uint8_t *flag,
                                                    int2 *mrec, uint64_t *mbeg, uint32_t *aown,
                                                    const uint8_t *__restrict__ arcst,
                                                    TableView T) {
  if (rc_idle(rc)) return;
  const uint64_t C = rc->total;
  const uint64_t cap3 = rc->cap3;
  const int lane = lane_id();
  // wave-uniform trip count for the ballot below
  for (uint64_t k0 = ((uint64_t)blockIdx.x * blockDim.x) + (threadIdx.x / kWave) * kWave; k0 < C;
       k0 += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t k = k0 + lane;
    bool in = k < C;
    int32_t x = 0;
    uint32_t f = 0;
    if (in) {
      f = owner[k];
      const int32_t v = drv[f];
      const int64_t ev = g.rp[v] + (int64_t)(k - ioff[f]);
      x = g.col[ev];
      if constexpr (R == 1) {
        // r = 1: the r-subsets are the vertices, stamped in their one-slot
        // segments.  x peeled earlier: every s-clique through it is gone; x
        // in this round's frontier below v: it owns them (Update-Func's
        // owner rule).  Either way R = {v} would only probe them to skip them.
        const uint32_t sx = T.slots[T.seg[x]].stamp;
        const uint32_t t = rc->t;
        in = !(sx != kLive && (sx < t || (sx == t && x < v)));
      } else if constexpr (R == 2) {
        const int32_t u0 = fv[(int64_t)f * 2], u1 = fv[(int64_t)f * 2 + 1];  // u0 < u1
        const int32_t w = u0 == v ? u1 : u0;
        const int64_t ew = arc_pos(g, x, w);
        if (ew < 0) {
          in = false;
        } else {
          const uint8_t sv = arcst[ev], sw = arcst[ew];
          const uint8_t s0 = v == u0 ? sv : sw, s1 = v == u0 ? sw : sv;  // {x,u0}, {x,u1}
          in = sv != kArcDead && sw != kArcDead && !(s0 == kArcFront && x < u1) &&
               !(s1 == kArcFront && x < u0);
        }
      } else {
#pragma unroll
        for (int i = 0; i < R; i++) {
          const int32_t u = fv[(int64_t)f * R + i];
          if (in && u != v) in = adjacent(g, x, u);
        }
        // r >= 3: the other r-subsets of R + x are R minus one vertex plus x.
        // One peeled earlier: every s-clique through R + x is gone.  One in
        // this round's frontier that precedes R lexicographically: it owns
        // each of them (Update-Func's owner rule: subsets of a sorted s-clique
        // compare by position as they compare by vertex).  Either way R
        // would only list them to skip them.
        if (in) {
          int32_t Rv[R], v1s[R], v2s[R];
          Key keys[R];
          bool want[R], before[R];
#pragma unroll
          for (int i = 0; i < R; i++) Rv[i] = fv[(int64_t)f * R + i];
#pragma unroll
          for (int a = 0; a < R; a++) {
            int32_t Tv[R];  // R without Rv[a], with x, ascending
            int o = 0;
            bool placed = false;
#pragma unroll
            for (int i = 0; i < R; i++) {
              if (i == a) continue;
              if (!placed && x < Rv[i]) {
                Tv[o++] = x;
                placed = true;
              }
              Tv[o++] = Rv[i];
            }
            if (!placed) Tv[R - 1] = x;
            int d = 0;  // first place where Tv and R differ (they differ somewhere)
#pragma unroll
            for (int i = R - 1; i >= 0; i--)
              if (Tv[i] != Rv[i]) d = i;
            before[a] = Tv[d] < Rv[d];
            v1s[a] = Tv[0];
            v2s[a] = Tv[1];
            keys[a] = rkey<R>(T, Tv);
            want[a] = true;
          }
          int64_t pos[R];
          Slot sl[R];
          table_find_n<R, (R >= 4)>(T, v1s, v2s, keys, want, pos, sl);
          const uint32_t t = rc->t;
#pragma unroll
          for (int a = 0; a < R; a++) {
            const uint32_t st = sl[a].stamp;
            if (pos[a] >= 0 && st != kLive && (st < t || (st == t && before[a]))) in = false;
          }
        }
      }
      flag[k] = in ? 1 : 0;
    }
    const uint64_t deg = in ? (uint64_t)(g.rp[x + 1] - g.up[x]) : 0;
    const bool emit = deg != 0;
    const uint64_t m = __ballot(emit);
    if (m) {
      // member index and out-arc range, one atomic each per wave
      const uint64_t incl = wave_incl_scan_u64(deg);
      const uint64_t tot = __shfl(incl, kWave - 1);
      unsigned long long at = 0, arc = 0;
      if (lane == 0) {
        at = atomicAdd((unsigned long long *)&rc->total2, (unsigned long long)__popcll(m));
        arc = atomicAdd((unsigned long long *)&rc->total3, (unsigned long long)tot);
      }
      at = __shfl(at, 0);
      arc = __shfl(arc, 0);
      if (emit) {
        const uint64_t i = at + (uint64_t)__popcll(m & lanes_below());
        const uint64_t a0 = arc + incl - deg;
        mrec[i] = make_int2((int)f, x);
        mbeg[i] = a0;
        if (a0 + deg <= cap3)  // otherwise the apply pass halts the round
          for (uint64_t q = 0; q < deg; q++) aown[a0 + q] = (uint32_t)i;
      }
    }
  }
}

// y in I(R): a position of the driver's row whose flag is set
__device__ __forceinline__ bool gen_in(const GraphView &g, const uint8_t *__restrict__ flag,
                                       int64_t lo, int64_t hi, uint64_t fbase, int32_t y) {
  const int64_t at = lower_pos(g.col, lo, hi, y);
  return at < hi && g.col[at] == y && flag[fbase + (uint64_t)(at - lo)] != 0;
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
__device__ void gen_extend(const PeelArgs &a, const uint8_t *__restrict__ flag, int64_t lo,
                           int64_t hi, uint64_t fbase, const int32_t (&Rv)[R],
                           int32_t (&Qv)[S - R], uint32_t p, LaneStats &ls,
                           const uint8_t *__restrict__ arcst) {
  const int32_t x = Qv[L - 1];
  for (int64_t e = a.g.up[x]; e < a.g.rp[x + 1]; e++) {
    const int32_t z = a.g.col[e];
    bool ok = gen_in(a.g, flag, lo, hi, fbase, z);
    if constexpr (R == 2) {
      // every edge of S other than R alive; an edge {q, z} of Q (q < z)
      // that is in the frontier comes before R = {u0, ...} when q < u0
      ok = ok && arcst[e] != kArcDead && !(arcst[e] == kArcFront && x < Rv[0]);
#pragma unroll
      for (int j = 0; j < L - 1; j++) {
        if (!ok) break;
        const int64_t q = arc_pos(a.g, Qv[j], z);
        ok = q >= 0 && arcst[q] != kArcDead && !(arcst[q] == kArcFront && Qv[j] < Rv[0]);
      }
    } else {
#pragma unroll
      for (int j = 0; j < L - 1; j++) ok = ok && adjacent(a.g, Qv[j], z);
    }
    if (!ok) continue;
    Qv[L] = z;
    if constexpr (L + 1 == S - R) {
      int32_t Sv[S];
      uint32_t rmask;
      merge_rq<R, S - R>(Rv, Qv, Sv, rmask);
      update_func<R, S, false>(a, Sv, rmask, p, true, ls, nullptr);
    } else {
      gen_extend<L + 1, R, S>(a, flag, lo, hi, fbase, Rv, Qv, p, ls, arcst);
    }
  }
}

// A thread per out-arc (x, y) of a member x of I(R): y in I(R) closes
// R + {x, y} (s = r+2) or starts a deeper extension.
template <int R, int S>
__global__ __launch_bounds__(256) void k_gen_apply(PeelArgs base, RoundCtl *rc,
                                                   const uint64_t *__restrict__ ioff,
                                                   const int32_t *__restrict__ fv,
                                                   const int32_t *__restrict__ drv,
                                                   const uint8_t *__restrict__ flag,
                                                   const int2 *__restrict__ mrec,
                                                   const uint64_t *__restrict__ mbeg,
                                                   const uint32_t *__restrict__ aown,
                                                   const uint8_t *__restrict__ arcst) {
  if (rc_idle(rc)) return;
  if (rc->total3 > rc->cap3) {  // arcs did not fit: the host grows the buffer, reruns the round
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      rc->need = rc->total3;
      rc->halt = 4;
    }
    return;
  }
  const PeelArgs a = round_args(base, rc);
  const uint32_t *__restrict__ F = rc->F;
  const uint64_t A = rc->total3;
  const int wv = threadIdx.x / kWave;
  const int lane = lane_id();
  LaneStats ls;
  __shared__ uint32_t abuf[256 / kWave][2][kAppendCap];
  Appender ap[2] = {{abuf[wv][0], 0u, a.Fnext, &a.ctr->next_size},
                    {abuf[wv][1], 0u, a.Low, &a.ctr->low_size}};
  // wave-uniform trip count: every lane reaches every append
  for (uint64_t b0 = ((uint64_t)blockIdx.x * blockDim.x) + (uint64_t)wv * kWave; b0 < A;
       b0 += (uint64_t)gridDim.x * blockDim.x) {
    const uint64_t j = b0 + lane;
    bool in = j < A;
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
      const uint32_t i = aown[j];
      const int2 mr = mrec[i];
      const int32_t f = mr.x, x = mr.y;
      const int32_t v = drv[f];
      lo = a.g.rp[v];
      hi = a.g.rp[v + 1];
      fbase = ioff[f];
      const int64_t exy = a.g.up[x] + (int64_t)(j - mbeg[i]);
      const int32_t y = a.g.col[exy];
      in = gen_in(a.g, flag, lo, hi, fbase, y);
      if constexpr (R == 2)  // {x, y} alive, and not a frontier edge before R
        in = in && arcst[exy] != kArcDead &&
             !(arcst[exy] == kArcFront && x < fv[(int64_t)f * 2]);
      p = F[f];
#pragma unroll
      for (int q = 0; q < R; q++) Rv[q] = fv[(int64_t)f * R + q];
      Qv[0] = x;
      Qv[1] = y;
    }
    if constexpr (S - R == 2) {
      int32_t Sv[S];
      uint32_t rmask;
      merge_rq<R, 2>(Rv, Qv, Sv, rmask);
      update_func<R, S, true>(a, Sv, rmask, p, in, ls, ap);
    } else {
      if (in) gen_extend<2, R, S>(a, flag, lo, hi, fbase, Rv, Qv, p, ls, arcst);
    }
  }
  ap[0].flush();
  ap[1].flush();
  stat_add(a.stats, kStatDec, ls.dec);
  stat_add(a.stats, kStatDisc, ls.disc);
  stat_add(a.stats, kStatAtom, ls.atom);
  if (ls.err) atomicOr(&a.ctr->err, ls.err);
}

// Graph contraction for (2,3) (Section 4.6): once the peeled edges since the
// last contraction reach the threshold (twice the vertex count), every
// vertex v that lost at least a quarter of its neighbours since its last
// contraction has its adjacency filtered of its peeled edges.  Here v's
// adjacency as the peel lists it is v's bitmap over N+(v), whose rows and
// columns of dead out-edges {v, a_i} are cleared, and the apex lists of v's
// out-arcs, from which the lower neighbours x with a dead edge {x, v} are
// compacted away.  A wave per vertex; runs between rounds, when no edge is
// in a frontier.  Listing stays exact without it (the per-candidate edge
// states decide); it only removes work.
__global__ __launch_bounds__(256) void k_contract2(GraphView g, FastView fx) {
  __shared__ uint64_t dead_col[256 / kWave][kMaxBitmapWords];
  const int wv = threadIdx.x / kWave, lane = lane_id();
  for (int64_t v = (int64_t)blockIdx.x * (256 / kWave) + wv; v < g.n;
       v += (int64_t)gridDim.x * (256 / kWave)) {
    const uint32_t lost = fx.lost[v];
    if (lost == 0 || 4ull * lost < fx.deg_at[v]) continue;  // wave-uniform
    const int64_t o = g.up[v];
    const int d = (int)(g.rp[v + 1] - o);
    if (d > 0 && d <= 64 * kMaxBitmapWords) {
      const int wd = (d + 63) >> 6;
      uint64_t *rows = fx.alive + fx.bm_off[v];
      if (lane < kMaxBitmapWords) dead_col[wv][lane] = 0;
      __builtin_amdgcn_wave_barrier();
      for (int i = lane; i < d; i += kWave)
        if (fx.arcst[o + i] == kArcDead)
          atomicOr((unsigned long long *)&dead_col[wv][i >> 6], 1ull << (i & 63));
      __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
      __builtin_amdgcn_wave_barrier();
      // each lane owns whole rows: plain stores
      for (int i = lane; i < d; i += kWave) {
        const bool row_dead = (dead_col[wv][i >> 6] >> (i & 63)) & 1ull;
        for (int w = 0; w < wd; w++) {
          const uint64_t x = rows[(int64_t)i * wd + w];
          const uint64_t y = row_dead ? 0ull : x & ~dead_col[wv][w];
          if (y != x) rows[(int64_t)i * wd + w] = y;
        }
      }
    }
    for (int i = lane; i < d; i += kWave) {  // apex lists of v's out-arcs
      const int64_t e = o + i;
      if (fx.arcst[e] == kArcDead) {  // its own edge is gone: never listed again
        fx.llen[e] = 0;
        continue;
      }
      const uint64_t b0 = fx.lptr[e];
      const uint32_t n0 = fx.llen[e];
      uint32_t keep = 0;
      for (uint32_t q = 0; q < n0; q++) {
        const int32_t x = fx.lvr[b0 + q];
        const int64_t e1 = arc_pos(g, x, (int32_t)v);
        if (e1 >= 0 && fx.arcst[e1] != kArcDead) fx.lvr[b0 + keep++] = x;
      }
      fx.llen[e] = keep;
    }
    if (lane == 0) {
      fx.deg_at[v] -= lost;
      fx.lost[v] = 0;
    }
  }
}

__global__ void k_contract_done(RoundCtl *rc) {
  rc->peeled_since = 0;
  rc->contract_due = 0;
  rc->contractions++;
}

dim3 blocks_for(uint64_t n, uint64_t per, uint64_t lo, uint64_t hi) {
  uint64_t b = (n + per - 1) / per;
  b = b < lo ? lo : b;
  b = b > hi ? hi : b;
  return dim3((unsigned)b);
}

// Buffers and launch parameters of one peel loop.  Every device buffer is a
// DevBuf taken from the run's workspace; peel_ws_bytes adds up the same list.
struct Engine {
  int r = 0, s = 0, path = 0;
  GraphView gv{};
  TableView T{};
  FastView fxv{};
  const uint64_t *loc = nullptr;
  Counters *dc = nullptr;
  unsigned long long *stats = nullptr;
  hipStream_t st = nullptr;
  RoundCtl *rc = nullptr;  // owned by the plan
  DevBuf<uint32_t> lists;  // F, F', W, W', H, H' (n_r each)
  DevBuf<uint64_t> off;    // per frontier entry: first record / flag
  DevBuf<uint32_t> len;    // per frontier entry: records / flags
  DevBuf<int32_t> fv;      // per frontier entry: its r vertices
  DevBuf<int32_t> drv;     // per frontier entry: driver (s >= r+2)
  DevBuf<ExpandDesc> desc; // per frontier entry: expand descriptor (s = r+1)
  DevBuf<uint32_t> f23;    // r = 3: per frontier entry, v3's local index in N+(v2)
  DevBuf<uint16_t> rloc;   // r = 3: per record, x's local index in N+(v1) (or 0xFFFF)
  DevBuf<int2> rec;        // candidate records (s = r+1) or member records (s >= r+2)
  DevBuf<uint8_t> flag;    // s >= r+2: membership flags
  DevBuf<uint32_t> owner;  // s >= r+2: frontier index of each candidate
  DevBuf<uint64_t> mbeg;   // s >= r+2: first out-arc of each member
  DevBuf<uint32_t> aown;   // s >= r+2: member of each out-arc
  DevBuf<uint8_t> dead;    // s >= r+2, r = 2: per arc position, alive / frontier / dead
  bool track_lost = false; // (2,3) with graph contraction: count lost neighbours
  uint64_t cap3 = 0;
  DevBuf<uint32_t> tsize, tk;
  uint64_t cap = 0;
  uint32_t tcap = 0;
};

template <int R, int S>
void launch_walker(Engine &E, const PeelArgs &base, dim3 gf, dim3 gw, hipEvent_t e0,
                   hipEvent_t e1) {
  hipLaunchKernelGGL(k_stamp, gf, dim3(256), 0, E.st, E.rc, E.T.slots);
  if (e0) hipEventRecord(e0, E.st);
  hipLaunchKernelGGL((k_peel<R, S>), gw, dim3(256), 0, E.st, base, E.rc);
  if (e1) hipEventRecord(e1, E.st);
}

template <int R>
void launch_fast(Engine &E, const PeelArgs &base, dim3 gf, dim3 gw, dim3 ga, hipEvent_t e0,
                 hipEvent_t e1) {
  hipLaunchKernelGGL(k_expand_bound<R>, gf, dim3(256), 0, E.st, base, E.rc, E.fxv, E.loc,
                     E.off.get(), E.len.get(), E.fv.get(), E.desc.get(), E.f23.get());
  hipLaunchKernelGGL(k_expand<R>, gw, dim3(256), 0, E.st, base, E.rc, E.fxv, E.desc.get(),
                     E.off.get(), E.len.get(), E.fv.get(), E.rec.get(), E.rloc.get());
  if (e0) hipEventRecord(e0, E.st);
  if constexpr (R == 3)
    hipLaunchKernelGGL(k_apply3, ga, dim3(256), 0, E.st, base, E.rc, E.rec.get(),
                       E.fv.get(), E.fxv, E.loc, E.rloc.get(), E.f23.get());
  else
    hipLaunchKernelGGL(k_apply<R>, ga, dim3(256), 0, E.st, base, E.rc, E.rec.get(),
                       E.fv.get(), E.fxv, E.loc, E.rloc.get(), E.f23.get());
  if (e1) hipEventRecord(e1, E.st);
}

template <int R, int S>
void launch_gen(Engine &E, const PeelArgs &base, dim3 gf, dim3 gw, dim3 gc, dim3 ga,
                hipEvent_t e0, hipEvent_t e1) {
  hipLaunchKernelGGL(k_gen_bound<R>, gf, dim3(256), 0, E.st, base, E.rc, E.off.get(),
                     E.len.get(), E.fv.get(), E.drv.get(), E.dead.get());
  hipLaunchKernelGGL(k_gen_spread, gw, dim3(256), 0, E.st, E.rc, E.off.get(), E.len.get(),
                     E.owner.get());
  hipLaunchKernelGGL(k_gen_member<R>, gc, dim3(256), 0, E.st, E.gv, E.rc, E.off.get(),
                     E.owner.get(), E.fv.get(), E.drv.get(), E.flag.get(), E.rec.get(),
                     E.mbeg.get(), E.aown.get(), E.dead.get(), E.T);
  if (e0) hipEventRecord(e0, E.st);
  hipLaunchKernelGGL((k_gen_apply<R, S>), ga, dim3(256), 0, E.st, base, E.rc, E.off.get(),
                     E.fv.get(), E.drv.get(), E.flag.get(), E.rec.get(), E.mbeg.get(),
                     E.aown.get(), E.dead.get());
  if (e1) hipEventRecord(e1, E.st);
}

#define ND_WALK(R_, S_) \
  case (R_) * 16 + (S_): launch_walker<R_, S_>(E, base, gf, gw, e0, e1); break;
#define ND_GEN(R_, S_) \
  case (R_) * 16 + (S_): launch_gen<R_, S_>(E, base, gf, gw, gc, ga, e0, e1); break;

// Grids of one round's kernels.
struct RoundGrids {
  bool exact;           // first round of a batch: separate advance kernels
  bool advance;         // the round may start with a level advance
  dim3 amin, apart;     // level advance: minimum, partition
  dim3 aend;            // round end: the next advance's minimum
  dim3 gf, gw, ga, gc;  // per frontier entry, per frontier wave, record passes
};

uint32_t pow2_at_least(uint64_t x) {
  uint32_t p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Grids for one round.  m is the last state read back: exact when nothing is
// in flight (the first round of a batch), otherwise only a guide for the grid
// sizes (every kernel loops over the true sizes it reads on the device).
// With `quantized` every size is rounded up to a power of two, so that the
// captured graphs of queued rounds are reused across batches.
RoundGrids round_grids(const Engine &E, const RoundCtl &m, bool exact, bool quantized) {
  RoundGrids g{};
  auto q = [&](dim3 d) { return quantized ? dim3(pow2_at_least(d.x)) : d; };
  g.exact = exact;
  g.advance = !exact || m.nF == 0;
  // queued behind other rounds the advance kernels act only now and then:
  // small grids
  const uint64_t cap_b = exact ? 8192 : 256;
  const uint64_t nl = m.nW != 0 ? m.nW : m.nH;
  g.amin = q(blocks_for(nl, 256 * 8, 1, cap_b));
  g.apart = q(blocks_for(nl, kPartThreads * kPartItems, 1, cap_b));
  // the next frontier is rarely empty: the small grid of queued rounds
  g.aend = q(blocks_for(nl, 256 * 8, 1, 256));
  // Grids: sized to the frontier when it is known (nothing in flight and no
  // level advance), otherwise wide enough to fill the chip, so that a large
  // round queued behind small ones never runs on a small grid.  Measured and
  // dropped: sizing queued rounds from the recent ones (on rMAT-18 (3,4) a
  // batch of 32 rounds swings between a few dozen and 10^6 records, and the
  // big rounds on small grids tripled the update pass), and record-pass
  // floors of 256 or 512 blocks or caps of 2048 (up to 1.9x slower peels on
  // rMAT-18 (3,4) and Chung-Lu 1M (4,5), no gain on (2,4)).
  const bool known = exact && m.nF != 0;
  g.gf = known ? blocks_for(m.nF, 256, 1, 4096) : dim3(1024);
  g.gw = known ? blocks_for(m.nF, 256 / kWave, 1, 1u << 16) : dim3(4096);
  if (E.path == 2) {
    g.gc = q(blocks_for(2 * m.total, 256, 1024, 8192));
    g.ga = q(blocks_for(2 * m.total3, 256, 1024, 8192));
  } else {
    g.ga = q(blocks_for(2 * m.total, 256, 1024, 8192));
    g.gc = g.ga;
  }
  return g;
}

// Queue one round with the given grids on E.st; next_queued: another round
// follows it in the same batch.
void launch_round(Engine &E, const RoundGrids &G, bool next_queued, hipEvent_t e0,
                  hipEvent_t e1, hipEvent_t e_adv) {
  const hipStream_t st = E.st;
  RoundCtl *rc = E.rc;
  // r = 3 on the s = r+1 path: frontier marks at selection
  const bool r3 = E.path == 1 && E.r == 3;
  if (G.exact) {
    if (G.advance) {
      hipLaunchKernelGGL(k_adv_min, G.amin, dim3(256), 0, st, rc, E.T.slots);
      hipLaunchKernelGGL(k_adv_partition, G.apart, dim3(kPartThreads), 0, st, rc, E.T.slots, r3,
                         E.gv, E.T.v1, E.fxv, E.loc);
    }
    if (e_adv) hipEventRecord(e_adv, st);
    hipLaunchKernelGGL(k_round_begin, dim3(1), dim3(1), 0, st, rc, E.dc);
  } else {
    hipLaunchKernelGGL(k_advance_begin, G.apart, dim3(kPartThreads), 0, st, rc, E.dc,
                       E.T.slots, r3, E.gv, E.T.v1, E.fxv, E.loc);
    if (e_adv) hipEventRecord(e_adv, st);
  }
  const dim3 gf = G.gf, gw = G.gw;
  const PeelArgs base{E.gv, E.T, 0u, 0u, nullptr, E.dc, E.stats, 0u, nullptr};
  if (E.path == 1) {
    const dim3 ga = G.ga;
    switch (E.r) {
      case 2: launch_fast<2>(E, base, gf, gw, ga, e0, e1); break;
      case 3: launch_fast<3>(E, base, gf, gw, ga, e0, e1); break;
      case 4: launch_fast<4>(E, base, gf, gw, ga, e0, e1); break;
      case 5: launch_fast<5>(E, base, gf, gw, ga, e0, e1); break;
      case 6: launch_fast<6>(E, base, gf, gw, ga, e0, e1); break;
      default: break;
    }
  } else if (E.path == 2) {
    const dim3 gc = G.gc, ga = G.ga;
    switch (E.r * 16 + E.s) {
      ND_GEN(1, 3) ND_GEN(1, 4) ND_GEN(1, 5) ND_GEN(1, 6) ND_GEN(1, 7)
      ND_GEN(2, 4) ND_GEN(2, 5) ND_GEN(2, 6) ND_GEN(2, 7)
      ND_GEN(3, 5) ND_GEN(3, 6) ND_GEN(3, 7)
      ND_GEN(4, 6) ND_GEN(4, 7)
      ND_GEN(5, 7)
      ND_GEN(1, 8) ND_GEN(2, 8) ND_GEN(3, 8) ND_GEN(4, 8) ND_GEN(5, 8) ND_GEN(6, 8)
      default: break;
    }
  } else {
    switch (E.r * 16 + E.s) {
      ND_WALK(1, 2) ND_WALK(1, 3) ND_WALK(1, 4) ND_WALK(1, 5) ND_WALK(1, 6) ND_WALK(1, 7)
      ND_WALK(2, 3) ND_WALK(2, 4) ND_WALK(2, 5) ND_WALK(2, 6) ND_WALK(2, 7)
      ND_WALK(3, 4) ND_WALK(3, 5) ND_WALK(3, 6) ND_WALK(3, 7)
      ND_WALK(4, 5) ND_WALK(4, 6) ND_WALK(4, 7)
      ND_WALK(5, 6) ND_WALK(5, 7)
      ND_WALK(6, 7)
      ND_WALK(1, 8) ND_WALK(2, 8) ND_WALK(3, 8) ND_WALK(4, 8) ND_WALK(5, 8) ND_WALK(6, 8)
      ND_WALK(7, 8)
      default: break;
    }
  }
  // r = 2 keeps per-arc edge states: the round's end also retires its edges
  uint8_t *arcst = E.r != 2 ? nullptr : (E.path == 2 ? E.dead.get() : E.fxv.arcst);
  const uint32_t ge = next_queued && G.aend.x > gf.x ? G.aend.x : gf.x;
  if (arcst)
    hipLaunchKernelGGL(k_round_end_r2, dim3(ge), dim3(256), 0, st, rc,
                       E.dc, E.T.slots, (uint32_t)next_queued, E.gv, E.fv.get(), arcst,
                       E.track_lost ? E.fxv.lost : nullptr);
  else
    hipLaunchKernelGGL(k_round_end, next_queued ? G.aend : dim3(1), dim3(256), 0, st, rc, E.dc,
                       E.T.slots, (uint32_t)next_queued);
}

// Instantiated graphs of `rest` queued rounds (one run's cache: the graphs
// hold the run's workspace pointers), keyed by the round count and the
// quantized grids.  Rounds queued past the first of a batch are captured
// once per key on a private stream and then replayed with one launch.
struct GraphCache {
  struct Entry {
    uint64_t key;
    hipGraphExec_t exec;
  };
  std::vector<Entry> v;
  ~GraphCache() {
    for (auto &e : v) hipGraphExecDestroy(e.exec);
  }
};

uint64_t graph_key(int rest, const RoundGrids &G, bool timing) {
  auto lg = [](uint32_t x) {
    uint64_t l = 0;
    while ((1u << l) < x) l++;
    return l;
  };
  return (uint64_t)rest | lg(G.amin.x) << 8 | lg(G.apart.x) << 14 | lg(G.ga.x) << 20 |
         lg(G.gc.x) << 26 | (uint64_t)timing << 32;
}

// Queue rounds 1..rest of a batch (the first one is queued by the caller) as
// one graph launch; returns false if capture or instantiation failed.
bool launch_rounds_graph(Engine &E, GraphCache &gc, hipStream_t cap, int rest,
                         const RoundGrids &G, hipEvent_t *ev) {
  const uint64_t key = graph_key(rest, G, ev != nullptr);
  hipGraphExec_t exec = nullptr;
  for (auto &e : gc.v)
    if (e.key == key) exec = e.exec;
  if (!exec) {
    const hipStream_t st = E.st;
    if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) return false;
    E.st = cap;
    for (int d = 1; d <= rest; d++)
      launch_round(E, G, d < rest, ev ? ev[2 * d] : nullptr, ev ? ev[2 * d + 1] : nullptr,
                   nullptr);
    E.st = st;
    hipGraph_t g = nullptr;
    if (hipStreamEndCapture(cap, &g) != hipSuccess || !g) return false;
    const hipError_t ie = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ie != hipSuccess) return false;
    gc.v.push_back({key, exec});
  }
  return hipGraphLaunch(exec, E.st) == hipSuccess;
}

void alloc_records(Engine &E, uint64_t cap) {
  E.rec.reset(cap);
  E.rloc.reset(E.path == 1 && E.r == 3 ? cap : 1);
  if (E.path == 2) {
    E.flag.reset(cap);
    E.owner.reset(cap);
    E.mbeg.reset(cap);
    E.cap3 = kArcsPerRecord * cap;
    E.aown.reset(E.cap3);
  }
  E.cap = cap;
}


}  // namespace

uint64_t peel_ws_bytes(int r, int path, uint64_t n_r, uint64_t nnz, uint64_t rec_cap,
                       uint32_t trace_cap) {
  if (n_r == 0) return ws_buf<uint32_t>(1);  // the empty round trace
  uint64_t b = ws_buf<uint32_t>(6 * n_r) + ws_buf<uint64_t>(n_r) + ws_buf<uint32_t>(n_r) +
               ws_buf<int32_t>(n_r * (uint64_t)r);
  if (path == 2) b += ws_buf<int32_t>(n_r);
  if (path == 2 && r == 2) b += ws_buf<uint8_t>(nnz ? nnz : 1);
  if (path == 1) b += ws_buf<ExpandDesc>(n_r) + ws_buf<uint32_t>(r == 3 ? n_r : 1);
  if (path != 0) {
    b += ws_buf<int2>(rec_cap) + ws_buf<uint16_t>(path == 1 && r == 3 ? rec_cap : 1);
    if (path == 2)
      b += ws_buf<uint8_t>(rec_cap) + ws_buf<uint32_t>(rec_cap) + ws_buf<uint64_t>(rec_cap) +
           ws_buf<uint32_t>(kArcsPerRecord * rec_cap);
  }
  return b + 2 * ws_buf<uint32_t>(trace_cap);
}

uint32_t peel_all(const OrientedGraph &g, int r, int s, int path, const TableView &T,
                  const FastIndex *fx, const uint32_t *occ, uint64_t n_r, Counters *dc,
                  unsigned long long *stats, const PeelState &ps, uint64_t rec_cap,
                  uint32_t trace_cap, hipStream_t st, hipEvent_t ev_first,
                  DevBuf<uint32_t> *kround, PeelResult *res, PeelSuspend *sus) {
  res->sizes.clear();
  res->levels.clear();
  res->advances = 0;
  res->apply_ms = 0;
  res->apply_launches = 0;
  res->need_rec = 0;
  res->need_trace = 0;
  res->max_rec = 0;
  res->max_arcs = 0;
  if (n_r == 0) {
    if (ev_first) hipEventRecord(ev_first, st);
    kround->reset(1);
    return 0;
  }
  const bool timing = ps.ev != nullptr;
  Engine E;
  E.r = r;
  E.s = s;
  E.path = path;
  E.gv = g.view();
  E.T = T;
  if (fx) {
    E.fxv = fx->view();
    E.loc = fx->loc.get();
  }
  E.dc = dc;
  E.stats = stats;
  E.st = st;
  E.rc = ps.rc;
  E.track_lost = ps.contract_every != 0 && fx && fx->lost.get();
  // resume: the state a round that outgrew the previous workspace left
  const bool resume = sus && sus->on;
  // the live part of the bucket lists: frontier F[selF], window W[selW] and
  // high list H[selH] (the other buffer of each pair is scratch between
  // rounds); a round that stopped appended nothing yet
  auto live = [&](const RoundCtl &c, int i, uint64_t &off, uint64_t &len) {
    const uint32_t sel = i == 0 ? c.selF : i == 1 ? c.selW : c.selH;
    off = (uint64_t)(2 * i + (sel & 1u)) * n_r;
    len = i == 0 ? c.nF : i == 1 ? c.nW : c.nH;
  };
  if (resume) {
    uint64_t tot = 0;
    for (int i = 0; i < 3; i++) {
      uint64_t o, l;
      live(sus->rc, i, o, l);
      if (l > n_r) return kErrRuntime;
      tot += l;
    }
    if (sus->lists.size() != tot || sus->rc.t > trace_cap || sus->tsize.size() != sus->rc.t ||
        sus->tk.size() != sus->rc.t)
      return kErrRuntime;
  }
  const uint64_t na = g.nnz > 0 ? (uint64_t)g.nnz : 1;  // arc positions
  E.lists.reset(6 * n_r);
  uint32_t *L = E.lists.get();
  if (resume) {
    uint64_t at = 0;
    for (int i = 0; i < 3; i++) {
      uint64_t o, l;
      live(sus->rc, i, o, l);
      if (l && hipMemcpyAsync(L + o, sus->lists.data() + at, 4 * l, hipMemcpyHostToDevice, st) !=
                   hipSuccess)
        return kErrRuntime;
      at += l;
    }
  } else if (hipMemcpyAsync(L + 4 * n_r, occ, 4 * n_r, hipMemcpyDeviceToDevice, st) !=
             hipSuccess) {  // H = every r-clique
    return kErrRuntime;
  }
  E.off.reset(n_r);
  E.len.reset(n_r);
  E.fv.reset(n_r * (uint64_t)r);
  if (path == 2) E.drv.reset(n_r);
  if (path == 2 && r == 2) {
    E.dead.reset(na);
    if (!resume) {
      fill_u32((uint32_t *)E.dead.get(), 0, (int64_t)(ws_block(na) / 4), st);
    } else if (sus->dead.size() != na ||
               hipMemcpyAsync(E.dead.get(), sus->dead.data(), na, hipMemcpyHostToDevice, st) !=
                   hipSuccess) {
      return kErrRuntime;
    }
  }
  if (path == 1) {
    E.desc.reset(n_r);
    E.f23.reset(r == 3 ? n_r : 1);
  }
  // capacities fixed by the workspace layout: a round that needs more stops
  // the peel and reports what it needs
  E.tcap = trace_cap;
  if (path != 0) alloc_records(E, rec_cap);
  E.tsize.reset(E.tcap);
  E.tk.reset(E.tcap);
  if (resume && sus->rc.t &&
      (hipMemcpyAsync(E.tsize.get(), sus->tsize.data(), 4ull * sus->rc.t, hipMemcpyHostToDevice,
                      st) != hipSuccess ||
       hipMemcpyAsync(E.tk.get(), sus->tk.data(), 4ull * sus->rc.t, hipMemcpyHostToDevice, st) !=
           hipSuccess))
    return kErrRuntime;

  RoundCtl h;
  if (resume) {  // the stopped round starts again; its lists now sit in this workspace
    h = sus->rc;
    h.halt = 0;
    h.need = 0;
    h.F = nullptr;
    h.Fnext = nullptr;
    h.Low = nullptr;
  } else {
    memset(&h, 0, sizeof(h));
    h.n_r = n_r;
    h.nH = (uint32_t)n_r;
    h.contract_every = ps.contract_every;
    h.mw = kNone;
    h.mh = kNone;
    h.wlev = kWindowLevels;
  }
  for (int i = 0; i < 2; i++) {
    h.bufF[i] = L + (uint64_t)i * n_r;
    h.bufW[i] = L + (uint64_t)(2 + i) * n_r;
    h.bufH[i] = L + (uint64_t)(4 + i) * n_r;
  }
  h.trace_size = E.tsize.get();
  h.trace_k = E.tk.get();
  h.trace_cap = E.tcap;
  h.cap = E.cap;
  h.cap3 = E.cap3;
  if (sus) sus->on = false;
  RoundCtl *mirror = ps.mirror;
  *mirror = h;  // staged through pinned memory: the copy is asynchronous
  if (hipMemcpyAsync(E.rc, mirror, sizeof(h), hipMemcpyHostToDevice, st) != hipSuccess ||
      hipStreamSynchronize(st) != hipSuccess)
    return kErrRuntime;
  hipEvent_t *ev = ps.ev;
  uint32_t status = 0;
  RoundCtl m = h;
  int depth = 1;
  const int dmax = ps.queue_depth >= 1 && ps.queue_depth <= kPeelMaxDepth ? ps.queue_depth
                                                                          : kPeelMaxDepth;
  bool first = true;
  GraphCache gcache;
  for (;;) {
    const auto t0 = std::chrono::steady_clock::now();
    launch_round(E, round_grids(E, m, true, false), depth > 1, timing ? ev[0] : nullptr,
                 timing ? ev[1] : nullptr, first ? ev_first : nullptr);
    if (depth > 1 && ps.graph_stream) {
      if (!launch_rounds_graph(E, gcache, ps.graph_stream, depth - 1,
                               round_grids(E, m, false, true), timing ? ev : nullptr)) {
        hipGetLastError();
        status = kErrRuntime;
        break;
      }
    } else {
      const RoundGrids G = round_grids(E, m, false, false);
      for (int d = 1; d < depth; d++)
        launch_round(E, G, d + 1 < depth, timing ? ev[2 * d] : nullptr,
                     timing ? ev[2 * d + 1] : nullptr, nullptr);
    }
    first = false;
    if (hipMemcpyAsync(mirror, E.rc, sizeof(RoundCtl), hipMemcpyDeviceToHost, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess) {
      status = kErrRuntime;
      break;
    }
    const RoundCtl prev = m;
    m = *mirror;
    if (timing) {
      for (int d = 0; d < depth; d++) {
        float ms = 0;
        if (hipEventElapsedTime(&ms, ev[2 * d], ev[2 * d + 1]) == hipSuccess) res->apply_ms += ms;
      }
    }
    if (m.err) {
      status = m.err;
      break;
    }
    if (m.halt == 1 || m.halt == 4 || m.halt == 2) {
      // a round outgrew the workspace: nothing of it has been applied; report
      // the capacity it needs (records, arcs in units of kArcsPerRecord
      // records, or round-trace entries)
      if (m.halt == 1) res->need_rec = m.need;
      if (m.halt == 4) res->need_rec = (m.need + kArcsPerRecord - 1) / kArcsPerRecord;
      if (m.halt == 2) res->need_trace = 2ull * E.tcap;
      res->max_rec = m.max_total;
      res->max_arcs = m.max_total3;
      status = kErrCapacity;
      // records or out-arcs: keep the state between rounds for a larger
      // workspace (the trace capacity is part of the layout: a run that
      // outgrew it starts again)
      if (sus && m.halt != 2) {
        sus->rc = m;
        uint64_t tot = 0;
        for (int i = 0; i < 3; i++) {
          uint64_t o, l;
          live(m, i, o, l);
          tot += l;
        }
        sus->lists.resize(tot);
        sus->tsize.resize(m.t);
        sus->tk.resize(m.t);
        sus->dead.resize(path == 2 && r == 2 ? na : 0);
        bool ok = true;
        uint64_t at = 0;
        for (int i = 0; i < 3; i++) {
          uint64_t o, l;
          live(m, i, o, l);
          if (l)
            ok = ok && hipMemcpyAsync(sus->lists.data() + at, L + o, 4 * l,
                                      hipMemcpyDeviceToHost, st) == hipSuccess;
          at += l;
        }
        if (m.t)
          ok = ok &&
               hipMemcpyAsync(sus->tsize.data(), E.tsize.get(), 4ull * m.t,
                              hipMemcpyDeviceToHost, st) == hipSuccess &&
               hipMemcpyAsync(sus->tk.data(), E.tk.get(), 4ull * m.t, hipMemcpyDeviceToHost,
                              st) == hipSuccess;
        if (!sus->dead.empty())
          ok = ok && hipMemcpyAsync(sus->dead.data(), E.dead.get(), na, hipMemcpyDeviceToHost,
                                    st) == hipSuccess;
        sus->on = ok && hipStreamSynchronize(st) == hipSuccess;
      }
      break;
    }
    if (m.halt) {
      status = kErrBucket;
      break;
    }
    if (m.done) break;
    if (m.contract_due) {  // graph contraction before the next batch of rounds
      hipLaunchKernelGGL(k_contract2, dim3((unsigned)grid_for(g.n, 256 / kWave, 16384)), dim3(256),
                         0, st, E.gv, E.fxv);
      hipLaunchKernelGGL(k_contract_done, dim3(1), dim3(1), 0, st, E.rc);
      m.contract_due = 0;
      m.peeled_since = 0;
    }
    // deepen the queue while rounds are short, back off while they are long
    const double dt =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    if (m.t == prev.t) depth = 1;
    else if (dt < 2.0 && depth < dmax) depth = depth * 2 < dmax ? depth * 2 : dmax;
    else if (dt > 20.0 && depth > 1) depth /= 2;
  }
  if (status) return status;
  res->advances = m.advances;
  res->contractions = m.contractions;
  res->max_rec = m.max_total;
  res->max_arcs = m.max_total3;
  res->apply_launches = m.t;
  std::vector<uint32_t> sz(m.t);
  res->levels.resize(m.t);
  if (m.t) {
    if (hipMemcpyAsync(sz.data(), E.tsize.get(), 4ull * m.t, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipMemcpyAsync(res->levels.data(), E.tk.get(), 4ull * m.t, hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      return kErrRuntime;
  }
  res->sizes.assign(sz.begin(), sz.end());
  *kround = std::move(E.tk);
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
  dim3 gg((unsigned)grid_for(n_r, 256 / kCountGroup, 1 << 20)), blk(256);
  switch (r) {
    case 3: hipLaunchKernelGGL(k_count_group<3>, gg, blk, 0, st, a, fv, loc, occ, n_r); break;
    case 4: hipLaunchKernelGGL(k_count_group<4>, gg, blk, 0, st, a, fv, loc, occ, n_r); break;
    case 5: hipLaunchKernelGGL(k_count_group<5>, gg, blk, 0, st, a, fv, loc, occ, n_r); break;
    case 6: hipLaunchKernelGGL(k_count_group<6>, gg, blk, 0, st, a, fv, loc, occ, n_r); break;
    default: break;
  }
}

void build_slot_loc(const OrientedGraph &g, int r, const TableView &T, uint64_t n_slots,
                    FastIndex *fx, hipStream_t st) {
  fx->loc.reset(n_slots ? n_slots : 1);
  if (!n_slots) return;
  dim3 grid((unsigned)grid_for(n_slots, 256)), blk(256);
  const GraphView gv = g.view();
  const FastView fv = fx->view();
  switch (r) {
    case 2: hipLaunchKernelGGL(k_make_loc<2>, grid, blk, 0, st, gv, T, fv, n_slots, fx->loc.get()); break;
    case 3: hipLaunchKernelGGL(k_make_loc<3>, grid, blk, 0, st, gv, T, fv, n_slots, fx->loc.get()); break;
    case 4: hipLaunchKernelGGL(k_make_loc<4>, grid, blk, 0, st, gv, T, fv, n_slots, fx->loc.get()); break;
    case 5: hipLaunchKernelGGL(k_make_loc<5>, grid, blk, 0, st, gv, T, fv, n_slots, fx->loc.get()); break;
    case 6: hipLaunchKernelGGL(k_make_loc<6>, grid, blk, 0, st, gv, T, fv, n_slots, fx->loc.get()); break;
    default: break;
  }
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
    case 7: hipLaunchKernelGGL(k_emit<7>, grid, blk, 0, st, occ, n_r, T, new2old, kround, nrounds, rcl_out, kappa_out); break;
    default: break;
  }
}

}  // namespace nd
