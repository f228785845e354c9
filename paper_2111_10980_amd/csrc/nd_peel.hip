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
};

struct LaneStats {
  uint64_t dec = 0, disc = 0;
  uint32_t err = 0;
};

// Update-Func for one s-clique S (sorted) found from the peeled r-clique at
// slot p, whose vertices occupy the positions in rmask.  Called by every
// lane of the wave in lock-step (active=false lanes only join the appends).
template <int R, int S, bool kConvergent>
__device__ __forceinline__ void update_func(const PeelArgs &a, const int32_t (&Sv)[S],
                                            uint32_t rmask, uint32_t p, bool active,
                                            LaneStats &ls) {
  constexpr Combos<S, R> cb{};
  uint32_t pos[cb.N];
  bool live[cb.N];
  bool alive = active;
  uint32_t owner = p;
#pragma unroll
  for (int q = 0; q < cb.N; q++) {
    pos[q] = p;
    live[q] = false;
    if (alive && cb.mask[q] != rmask) {
      int32_t Rv[R];
#pragma unroll
      for (int i = 0; i < R; i++) Rv[i] = Sv[cb.idx[q][i]];
      Slot sl;
      int64_t x = table_find(a.T, Rv[0], make_key<R>(Rv, a.T.bits), &sl);
      if (x < 0) {
        ls.err |= kErrLookup;
        alive = false;
      } else if (sl.stamp < a.t) {
        alive = false;  // S was destroyed in an earlier round
      } else {
        pos[q] = (uint32_t)x;
        if (sl.stamp == a.t) owner = (uint32_t)x < owner ? (uint32_t)x : owner;
        else live[q] = true;
      }
    }
  }
  if (active) ls.disc++;
  const bool mine = alive && owner == p;
#pragma unroll
  for (int q = 0; q < cb.N; q++) {
    bool want = false;
    if (mine && live[q]) {
      uint32_t old = __hip_atomic_fetch_add(&a.T.slots[pos[q]].cnt, 0xFFFFFFFFu, __ATOMIC_RELAXED,
                                            __HIP_MEMORY_SCOPE_AGENT);
      ls.dec++;
      want = old == a.k + 1;
    }
    if constexpr (kConvergent) {
      wave_append(want, pos[q], a.Fnext, &a.ctr->next_size);
    } else if (want) {
      a.Fnext[atomicAdd(&a.ctr->next_size, 1u)] = pos[q];
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
      update_func<R, S, false>(a, Sv, rmask, p, true, ls);
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
        update_func<R, S, true>(a, Sv, rmask, p, in, ls);
      } else {
        if (in) {
          int32_t Q[S - R];
          Q[0] = x;
          extend_q<1, R, S>(a, Rv, Q, p, ls);
        }
      }
    }
  }
  uint64_t d = wave_sum_u64(ls.dec), c = wave_sum_u64(ls.disc);
  if (lane == 0) {
    if (d) atomicAdd((unsigned long long *)&a.ctr->decrements, (unsigned long long)d);
    if (c) atomicAdd((unsigned long long *)&a.ctr->discoveries, (unsigned long long)c);
  }
  if (ls.err) atomicOr(&a.ctr->err, ls.err);
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

__global__ __launch_bounds__(256) void k_live_partition(const uint32_t *__restrict__ L, uint32_t nL,
                                                        const Slot *__restrict__ slots, uint32_t k,
                                                        uint32_t *F, uint32_t *nF, uint32_t *Lo,
                                                        uint32_t *nLo) {
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nL;
       base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = base + threadIdx.x;
    bool f = false, keep = false;
    uint32_t p = 0;
    if (i < nL) {
      p = L[i];
      const Slot s = slots[p];
      if (s.stamp == kLive) {
        f = s.cnt <= k;
        keep = !f;
      }
    }
    wave_append(f, p, F, nF);
    wave_append(keep, p, Lo, nLo);
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
                uint32_t nF, uint32_t t, uint32_t k, uint32_t *Fnext, Counters *dctr,
                hipStream_t st) {
  if (!nF) return;
  PeelArgs a{g.view(), T, t, k, Fnext, dctr};
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

void live_min(const uint32_t *L, uint32_t nL, const Slot *slots, Counters *dctr, hipStream_t st) {
  fill_u32(&dctr->live_min, 0xFFFFFFFFu, 1, st);
  if (!nL) return;
  hipLaunchKernelGGL(k_live_min, dim3((unsigned)grid_for(nL, 256 * 8, 8192)), dim3(256), 0, st, L,
                     nL, slots, &dctr->live_min);
}

void live_partition(const uint32_t *L, uint32_t nL, const Slot *slots, uint32_t k, uint32_t *F,
                    uint32_t *Lout, Counters *dctr, hipStream_t st) {
  fill_u32(&dctr->next_size, 0, 1, st);
  fill_u32(&dctr->live_size, 0, 1, st);
  if (!nL) return;
  hipLaunchKernelGGL(k_live_partition, dim3((unsigned)grid_for(nL, 256 * 4, 16384)), dim3(256), 0,
                     st, L, nL, slots, k, F, &dctr->next_size, Lout, &dctr->live_size);
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
