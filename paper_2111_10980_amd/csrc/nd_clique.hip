// Clique listing on the oriented graph (paper Algorithm 1, rec-list-cliques)
// and the two clients of it on the hot path:
//   - r-clique table build (Algorithm 2 "Initialize T"; Sections 4.1-4.3:
//     two-level table, last-level tables placed contiguously after a prefix
//     sum, slot position = r-clique index): count per first vertex, then
//     insert;
//   - s-clique counting (Algorithm 2 Count-Func): every s-clique is listed
//     once, from its lowest-ranked vertex, and each of its C(s,r) r-subsets
//     gets one 32-bit atomic increment.
//
// MI355X mapping.  One wave (64 lanes) owns one root vertex v.  Its
// out-neighbours N+(v) (d <= 512) are staged in LDS together with the
// adjacency bitmap of the subgraph they induce: row i has bit j set when
// N+(v)[j] is an out-neighbour of N+(v)[i] (built by merging sorted lists),
// so every deeper intersection of Algorithm 1 is a W-word AND in LDS.  Work
// is spread over the wave by flattening the first two levels: the pairs
// (i, j) with bit j of row i set (the triangles rooted at v) are numbered by
// a wave prefix sum of the row popcounts, and lane p takes pair p.  Roots are
// binned by d into W = 1, 2, 4, 8 words so the LDS footprint follows the
// root.  Roots with d > 512 go to a wave-per-root kernel whose lanes extend
// cliques with binary-search edge tests instead of bitmaps.  For s-clique
// counting with s >= 4 the pairs of a root are split over `split` waves (each
// stages the root itself): the few roots of the wide bins hold most of the
// deep listing work, and one wave each left most of the chip idle.
#include "nd_host.h"

namespace nd {

namespace {

int64_t grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  return b < cap ? b : cap;
}

template <int W>
__device__ __forceinline__ int select_bit(const uint64_t *row, uint32_t rank) {
#pragma unroll
  for (int w = 0; w < W; w++) {
    uint64_t x = row[w];
    uint32_t c = (uint32_t)__popcll(x);
    if (rank < c) {
      for (uint32_t q = 0; q < rank; q++) x &= x - 1;
      return w * 64 + __ffsll((unsigned long long)x) - 1;
    }
    rank -= c;
  }
  return -1;
}

// Extend the clique S[0..L-1] with every vertex whose bit is set in cand.
template <int L, int C, int W, class Op>
__device__ void bitmap_dfs(const uint64_t *rows, const int32_t *nb, int32_t (&S)[C],
                           const uint64_t (&cand)[W], Op &op, typename Op::Lane &ls) {
#pragma unroll
  for (int w = 0; w < W; w++) {
    uint64_t m = cand[w];
    while (m) {
      int b = __ffsll((unsigned long long)m) - 1;
      m &= m - 1;
      int x = w * 64 + b;
      S[L] = nb[x];
      if constexpr (L == C - 1) {
        op(ls, S);
      } else {
        uint64_t nc[W];
        bool any = false;
#pragma unroll
        for (int q = 0; q < W; q++) {
          nc[q] = cand[q] & rows[x * W + q];
          any |= nc[q] != 0;
        }
        if (any) bitmap_dfs<L + 1, C, W, Op>(rows, nb, S, nc, op, ls);
      }
    }
  }
}

template <int C, int W, class Op>
__global__ __launch_bounds__(kWave) void k_list_bitmap(GraphView g, const uint32_t *__restrict__ roots,
                                                       uint32_t nroots, Op op, uint32_t split) {
  constexpr int D = 64 * W;
  __shared__ int32_t nb[D];
  __shared__ uint64_t rows[C >= 3 ? D * W : 1];
  __shared__ uint32_t pre[C >= 3 ? D + 1 : 1];
  const int lane = threadIdx.x;
  typename Op::Lane ls;
  op.lane_init(ls);
  // item = (root, part): the part-th of the root's `split` waves
  const uint64_t items = (uint64_t)nroots * split;
  for (uint64_t it = blockIdx.x; it < items; it += gridDim.x) {
    const uint32_t ri = (uint32_t)(it / split), part = (uint32_t)(it % split);
    const int32_t v = (int32_t)roots[ri];
    const int64_t o = g.up[v];
    const int d = (int)(g.rp[v + 1] - o);
    for (int i = lane; i < d; i += kWave) nb[i] = g.col[o + i];
    __syncthreads();
    op.root_begin(ls, v);
    if constexpr (C == 2) {
      for (int i = (int)(part * kWave) + lane; i < d; i += (int)(split * kWave)) {
        int32_t S[2] = {v, nb[i]};
        op(ls, S);
      }
    } else {
      for (int i = lane; i < d; i += kWave) {
        uint64_t *row = rows + i * W;
#pragma unroll
        for (int w = 0; w < W; w++) row[w] = 0;
        const int32_t x = nb[i];
        int64_t a = g.up[x];
        const int64_t ae = g.rp[x + 1];
        int q = i + 1;
        uint32_t c = 0;
        while (a < ae && q < d) {
          int32_t y = g.col[a], z = nb[q];
          if (y == z) {
            row[q >> 6] |= 1ull << (q & 63);
            c++;
            a++;
            q++;
          } else if (y < z) {
            a++;
          } else {
            q++;
          }
        }
        pre[i] = c;
      }
      __syncthreads();
      uint32_t carry = 0;
      for (int base = 0; base < d; base += kWave) {
        int i = base + lane;
        uint32_t c = i < d ? pre[i] : 0u;
        uint32_t inc = wave_incl_scan(c);
        if (i < d) pre[i] = carry + inc - c;
        carry += __shfl(inc, kWave - 1);
      }
      if (lane == 0) pre[d] = carry;
      __syncthreads();
      const uint32_t P = pre[d];
      for (uint32_t p = part * kWave + lane; p < P; p += split * kWave) {
        int lo = 0, hi = d - 1;
        while (lo < hi) {
          int mid = (lo + hi + 1) >> 1;
          if (pre[mid] <= p) lo = mid;
          else hi = mid - 1;
        }
        const int i = lo;
        const uint64_t *ri_ = rows + i * W;
        const int j = select_bit<W>(ri_, p - pre[i]);
        int32_t S[C];
        S[0] = v;
        S[1] = nb[i];
        S[2] = nb[j];
        if constexpr (C == 3) {
          op(ls, S);
        } else {
          uint64_t cand[W];
          bool any = false;
#pragma unroll
          for (int w = 0; w < W; w++) {
            cand[w] = ri_[w] & rows[j * W + w];
            any |= cand[w] != 0;
          }
          if (any) bitmap_dfs<3, C, W, Op>(rows, nb, S, cand, op, ls);
        }
      }
    }
    op.root_end(ls, v);
    __syncthreads();
  }
  op.lane_finish(ls);
}

// Extension by edge tests: candidates for S[L] are the out-neighbours of
// S[L-1] adjacent to every earlier member.
template <int L, int C, class Op>
__device__ void adj_dfs(const GraphView &g, int32_t (&S)[C], Op &op, typename Op::Lane &ls) {
  const int32_t x = S[L - 1];
  for (int64_t a = g.up[x]; a < g.rp[x + 1]; a++) {
    const int32_t y = g.col[a];
    bool ok = true;
#pragma unroll
    for (int j = 0; j < L - 1; j++) ok = ok && adjacent(g, S[j], y);
    if (!ok) continue;
    S[L] = y;
    if constexpr (L == C - 1) op(ls, S);
    else adj_dfs<L + 1, C, Op>(g, S, op, ls);
  }
}

template <int C, class Op>
__global__ __launch_bounds__(kWave) void k_list_heavy(GraphView g, const uint32_t *__restrict__ roots,
                                                      uint32_t nroots, Op op) {
  typename Op::Lane ls;
  op.lane_init(ls);
  for (uint32_t ri = blockIdx.x; ri < nroots; ri += gridDim.x) {
    const int32_t v = (int32_t)roots[ri];
    const int64_t o = g.up[v];
    const int d = (int)(g.rp[v + 1] - o);
    op.root_begin(ls, v);
    for (int i = threadIdx.x; i < d; i += kWave) {
      int32_t S[C];
      S[0] = v;
      S[1] = g.col[o + i];
      if constexpr (C == 2) op(ls, S);
      else adj_dfs<2, C, Op>(g, S, op, ls);
    }
    op.root_end(ls, v);
  }
  op.lane_finish(ls);
}

// ------------------------------------------------------------------- ops

// Count-Func: +1 on the count of every r-subset of the s-clique.
template <int R, int S>
struct CountOp {
  static constexpr bool kSplit = true;  // no per-root state: a root may span waves
  TableView T;
  Counters *ctr;
  unsigned long long *stats;
  struct Lane {
    uint64_t ns;
    uint32_t err;
  };
  __device__ void lane_init(Lane &l) const { l.ns = 0; l.err = 0; }
  __device__ void root_begin(Lane &, int32_t) const {}
  __device__ void root_end(Lane &, int32_t) const {}
  // all C(s,r) probes are issued together (independent lookups), then the
  // increments
  __device__ void operator()(Lane &l, const int32_t (&Sv)[S]) const {
    constexpr Combos<S, R> cb{};
    constexpr int N = cb.N;
    l.ns++;
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
      key[q] = rkey<R>(T, Rv);
      want[q] = true;
    }
    int64_t pos[N];
    Slot sl[N];
    table_find_n<N, (R >= 4)>(T, v1, v2, key, want, pos, sl);
#pragma unroll
    for (int q = 0; q < N; q++) {
      if (pos[q] < 0) {
        l.err |= kErrLookup;
        continue;
      }
      __hip_atomic_fetch_add(&T.slots[pos[q]].cnt, 1u, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
  }
  __device__ void lane_finish(Lane &l) const {
    stat_add(stats, kStatNs, l.ns);
    if (l.err) atomicOr(&ctr->err, l.err);
  }
};

// Number of r-cliques whose lowest-ranked vertex is the root.
template <int R>
struct CountROp {
  static constexpr bool kSplit = false;  // root_end writes the root's total
  uint32_t *cnt;
  struct Lane {
    uint32_t c;
  };
  __device__ void lane_init(Lane &l) const { l.c = 0; }
  __device__ void root_begin(Lane &l, int32_t) const { l.c = 0; }
  __device__ void root_end(Lane &l, int32_t v) const {
    uint64_t t = wave_sum_u64(l.c);
    if (lane_id() == 0) cnt[v] = (uint32_t)t;
  }
  __device__ void operator()(Lane &l, const int32_t (&)[R]) const { l.c++; }
  __device__ void lane_finish(Lane &) const {}
};

// Number of r-cliques on each out-arc (v1, v2) of the oriented graph, by arc
// position (three-level tables).
template <int R>
struct CountArcOp {
  static constexpr bool kSplit = false;
  GraphView g;
  uint32_t *cnt;
  struct Lane {};
  __device__ void lane_init(Lane &) const {}
  __device__ void root_begin(Lane &, int32_t) const {}
  __device__ void root_end(Lane &, int32_t) const {}
  __device__ void operator()(Lane &, const int32_t (&Sv)[R]) const {
    const int64_t e = arc_pos(g, Sv[0], Sv[1]);
    if (e >= 0) atomicAdd(&cnt[e], 1u);
  }
  __device__ void lane_finish(Lane &) const {}
};

template <int R>
struct InsertOp {
  static constexpr bool kSplit = false;
  TableView T;
  Counters *ctr;
  struct Lane {
    uint32_t err;
  };
  __device__ void lane_init(Lane &l) const { l.err = 0; }
  __device__ void root_begin(Lane &, int32_t) const {}
  __device__ void root_end(Lane &, int32_t) const {}
  __device__ void operator()(Lane &l, const int32_t (&Sv)[R]) const {
    if (table_insert<(R >= 4)>(T, Sv[0], R > 1 ? Sv[R > 1 ? 1 : 0] : 0, rkey<R>(T, Sv)) < 0)
      l.err |= kErrTable;
  }
  __device__ void lane_finish(Lane &l) const {
    if (l.err) atomicOr(&ctr->err, l.err);
  }
};

// Apex lists: each triangle (x < y < z) contributes its lowest vertex x to
// the list of the arc (y, z); the arc is named by the position of z in row y
// of the relabeled CSR.  Keys are (arc << xbits) | x, written at per-root
// cursors so no two lanes contend on one counter.
struct ApexOp {
  static constexpr bool kSplit = false;
  GraphView g;
  unsigned long long *cursor;
  uint64_t *keys;
  int xbits;
  struct Lane {
    uint32_t dummy;
  };
  __device__ void lane_init(Lane &) const {}
  __device__ void root_begin(Lane &, int32_t) const {}
  __device__ void root_end(Lane &, int32_t) const {}
  __device__ void operator()(Lane &, const int32_t (&Sv)[3]) const {
    const int32_t y = Sv[1], z = Sv[2];
    int64_t lo = g.up[y], hi = g.rp[y + 1];
    while (lo < hi) {
      int64_t mid = (lo + hi) >> 1;
      if (g.col[mid] < z) lo = mid + 1;
      else hi = mid;
    }
    // the wave lists one root at a time (Sv[0] is wave-uniform): one atomic
    // per call reserves the active lanes' places, in lane order
    const uint64_t m = __ballot(1);
    const int first = __ffsll((unsigned long long)m) - 1;
    unsigned long long base = 0;
    if (lane_id() == first) base = atomicAdd(&cursor[Sv[0]], (unsigned long long)__popcll(m));
    base = __shfl(base, first);
    const unsigned long long at = base + (unsigned long long)__popcll(m & lanes_below());
    keys[at] = ((uint64_t)lo << xbits) | (uint64_t)(uint32_t)Sv[0];
  }
  __device__ void lane_finish(Lane &) const {}
};

// ---------------------------------------------------------- root binning

// class 0..3: bitmap kernels with W = 1, 2, 4, 8; class 4: heavy roots
__global__ void k_bin_roots(GraphView g, int minout, uint32_t *lists, int32_t n,
                            uint32_t *sizes) {
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n;
       base += (int64_t)gridDim.x * blockDim.x) {
    int64_t v = base + threadIdx.x;
    int cls = -1;
    if (v < n) {
      int64_t d = g.rp[v + 1] - g.up[v];
      if (d >= minout) cls = d <= 64 ? 0 : d <= 128 ? 1 : d <= 256 ? 2 : d <= 512 ? 3 : 4;
    }
#pragma unroll
    for (int c = 0; c < 5; c++)
      wave_append(cls == c, (uint32_t)v, lists + (int64_t)c * n, sizes + c);
  }
}

struct Bins {
  DevBuf<uint32_t> lists;
  uint32_t size[5] = {0, 0, 0, 0, 0};
  int32_t n = 0;
  const uint32_t *list(int c) const { return lists.get() + (int64_t)c * n; }
};

void bin_roots(const OrientedGraph &g, int minout, Counters *dctr, Bins *b, hipStream_t st) {
  b->n = g.n;
  b->lists.reset((size_t)5 * (g.n > 0 ? g.n : 1));
  fill_u32(dctr->class_size, 0, 8, st);
  if (g.n > 0)
    hipLaunchKernelGGL(k_bin_roots, dim3((unsigned)grid_for(g.n, 256)), dim3(256), 0, st,
                       g.view(), minout, b->lists.get(), g.n, dctr->class_size);
  read_back(b->size, dctr->class_size, sizeof(uint32_t) * 5, st);
}

template <int C, class Op>
void launch_listing(const OrientedGraph &g, const Bins &b, const Op &op, hipStream_t st) {
  const GraphView gv = g.view();
  auto grid = [](uint64_t n) { return dim3((unsigned)(n < 262144u ? n : 262144u)); };
  // waves per root of bins 0..3 (d <= 64, 128, 256, 512).  Measured on rMAT
  // (3,5) and (2,4): 5-cliques gain from the wider split (scale 13 count
  // 180 -> 110 ms), 4-cliques lose from it (scale 17: 285 -> 329 ms).
  const bool deep = Op::kSplit && C >= 4;
  const uint32_t sp4[4] = {2u, 8u, 16u, 32u}, sp5[4] = {4u, 32u, 64u, 64u};
  uint32_t sp[4];
  for (int i = 0; i < 4; i++) sp[i] = !deep ? 1u : C >= 5 ? sp5[i] : sp4[i];
  if (b.size[0])
    hipLaunchKernelGGL((k_list_bitmap<C, 1, Op>), grid((uint64_t)b.size[0] * sp[0]), dim3(kWave),
                       0, st, gv, b.list(0), b.size[0], op, sp[0]);
  if (b.size[1])
    hipLaunchKernelGGL((k_list_bitmap<C, 2, Op>), grid((uint64_t)b.size[1] * sp[1]), dim3(kWave),
                       0, st, gv, b.list(1), b.size[1], op, sp[1]);
  if (b.size[2])
    hipLaunchKernelGGL((k_list_bitmap<C, 4, Op>), grid((uint64_t)b.size[2] * sp[2]), dim3(kWave),
                       0, st, gv, b.list(2), b.size[2], op, sp[2]);
  if (b.size[3])
    hipLaunchKernelGGL((k_list_bitmap<C, 8, Op>), grid((uint64_t)b.size[3] * sp[3]), dim3(kWave),
                       0, st, gv, b.list(3), b.size[3], op, sp[3]);
  if (b.size[4])
    hipLaunchKernelGGL((k_list_heavy<C, Op>), grid(b.size[4]), dim3(kWave), 0, st, gv,
                       b.list(4), b.size[4], op);
}

__global__ void k_outdeg(GraphView g, uint32_t *cnt) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
       v += (int64_t)gridDim.x * blockDim.x)
    cnt[v] = (uint32_t)(g.rp[v + 1] - g.up[v]);
}

__global__ void k_insert_singletons(TableView T, int32_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    T.slots[T.seg[v]].key = kOcc;
    T.v1[T.seg[v]] = (int32_t)v;
  }
}

template <int R>
void count_r_impl(const OrientedGraph &g, uint32_t *cnt, Counters *dctr, hipStream_t st) {
  Bins b;
  bin_roots(g, R - 1, dctr, &b, st);
  fill_u32(cnt, 0, g.n, st);
  launch_listing<R>(g, b, CountROp<R>{cnt}, st);
}

template <int R>
void count_arc_impl(const OrientedGraph &g, uint32_t *cnt, Counters *dctr, hipStream_t st) {
  Bins b;
  bin_roots(g, R - 1, dctr, &b, st);
  fill_u32(cnt, 0, g.nnz + 1, st);
  launch_listing<R>(g, b, CountArcOp<R>{g.view(), cnt}, st);
}

template <int R>
void insert_r_impl(const OrientedGraph &g, const TableView &T, Counters *dctr, hipStream_t st) {
  Bins b;
  bin_roots(g, R - 1, dctr, &b, st);
  launch_listing<R>(g, b, InsertOp<R>{T, dctr}, st);
}

template <int R, int S>
void count_s_impl(const OrientedGraph &g, const TableView &T, Counters *dctr,
                  unsigned long long *stats, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  Bins b;
  bin_roots(g, S - 1, dctr, &b, st);
  if (ev0) hipEventRecord(ev0, st);
  launch_listing<S>(g, b, CountOp<R, S>{T, dctr, stats}, st);
  if (ev1) hipEventRecord(ev1, st);
}

}  // namespace

void count_rcliques(const OrientedGraph &g, int r, uint32_t *cnt, hipStream_t st) {
  if (g.n == 0) return;
  DevBuf<Counters> tmp(1);
  switch (r) {
    case 1: fill_u32(cnt, 1, g.n, st); break;
    case 2:
      hipLaunchKernelGGL(k_outdeg, dim3((unsigned)grid_for(g.n, 256)), dim3(256), 0, st,
                         g.view(), cnt);
      break;
    case 3: count_r_impl<3>(g, cnt, tmp.get(), st); break;
    case 4: count_r_impl<4>(g, cnt, tmp.get(), st); break;
    case 5: count_r_impl<5>(g, cnt, tmp.get(), st); break;
    case 6: count_r_impl<6>(g, cnt, tmp.get(), st); break;
    case 7: count_r_impl<7>(g, cnt, tmp.get(), st); break;
    default: break;
  }
}

void count_rcliques_arcs(const OrientedGraph &g, int r, uint32_t *cnt, hipStream_t st) {
  if (g.n == 0) return;
  DevBuf<Counters> tmp(1);
  switch (r) {
    case 4: count_arc_impl<4>(g, cnt, tmp.get(), st); break;
    case 5: count_arc_impl<5>(g, cnt, tmp.get(), st); break;
    case 6: count_arc_impl<6>(g, cnt, tmp.get(), st); break;
    case 7: count_arc_impl<7>(g, cnt, tmp.get(), st); break;
    default: break;
  }
}

void insert_rcliques(const OrientedGraph &g, int r, const TableView &T, Counters *dctr,
                     hipStream_t st) {
  if (g.n == 0) return;
  switch (r) {
    case 1:
      hipLaunchKernelGGL(k_insert_singletons, dim3((unsigned)grid_for(g.n, 256)), dim3(256), 0,
                         st, T, g.n);
      break;
    case 2: insert_r_impl<2>(g, T, dctr, st); break;
    case 3: insert_r_impl<3>(g, T, dctr, st); break;
    case 4: insert_r_impl<4>(g, T, dctr, st); break;
    case 5: insert_r_impl<5>(g, T, dctr, st); break;
    case 6: insert_r_impl<6>(g, T, dctr, st); break;
    case 7: insert_r_impl<7>(g, T, dctr, st); break;
    default: break;
  }
}

void insert_rcliques_heavy3(const OrientedGraph &g, const TableView &T, Counters *dctr,
                            hipStream_t st) {
  if (g.n == 0) return;
  Bins b;
  bin_roots(g, 2, dctr, &b, st);
  if (b.size[4])
    hipLaunchKernelGGL((k_list_heavy<3, InsertOp<3>>),
                       dim3(b.size[4] < 262144u ? b.size[4] : 262144u), dim3(kWave), 0, st,
                       g.view(), b.list(4), b.size[4], InsertOp<3>{T, dctr});
}

void list_apex_keys(const OrientedGraph &g, uint64_t *cursor, uint64_t *keys, int xbits,
                    Counters *dctr, hipStream_t st) {
  if (g.n == 0) return;
  Bins b;
  bin_roots(g, 2, dctr, &b, st);
  launch_listing<3>(g, b, ApexOp{g.view(), (unsigned long long *)cursor, keys, xbits}, st);
}

__global__ __launch_bounds__(256) void k_stats_collect(const unsigned long long *__restrict__ stats,
                                                       Counters *dctr) {
  // one block: thread i sums column i's lines for the four statistics
  uint64_t acc[4] = {0, 0, 0, 0};
  for (int line = threadIdx.x; line < kStatLines; line += blockDim.x)
    for (int w = 0; w < 4; w++) acc[w] += stats[line * kStatStride + w];
  for (int w = 0; w < 4; w++) {
    const uint64_t t = wave_sum_u64(acc[w]);
    if (lane_id() == 0 && t) {
      unsigned long long *dst = (unsigned long long *)(w == kStatDec    ? &dctr->decrements
                                                       : w == kStatDisc ? &dctr->discoveries
                                                       : w == kStatAtom ? &dctr->atomics
                                                                        : &dctr->n_s);
      atomicAdd(dst, (unsigned long long)t);
    }
  }
}

void stats_collect(unsigned long long *stats, Counters *dctr, hipStream_t st) {
  hipLaunchKernelGGL(k_stats_collect, dim3(1), dim3(256), 0, st, stats, dctr);
}

uint64_t count_scliques_ws_bytes(const OrientedGraph &g) {
  return g.n == 0 ? 0 : ws_buf<uint32_t>((uint64_t)5 * (uint64_t)g.n);
}

#define ND_COUNT_CASE(R_, S_) \
  case (R_) * 16 + (S_): count_s_impl<R_, S_>(g, T, dctr, stats, st, ev0, ev1); break;

void count_scliques(const OrientedGraph &g, int r, int s, const TableView &T, Counters *dctr,
                    unsigned long long *stats, hipStream_t st, hipEvent_t ev0, hipEvent_t ev1) {
  if (g.n == 0) {
    if (ev0) hipEventRecord(ev0, st);
    if (ev1) hipEventRecord(ev1, st);
    return;
  }
  switch (r * 16 + s) {
    ND_COUNT_CASE(1, 2) ND_COUNT_CASE(1, 3) ND_COUNT_CASE(1, 4) ND_COUNT_CASE(1, 5)
    ND_COUNT_CASE(1, 6) ND_COUNT_CASE(1, 7)
    ND_COUNT_CASE(2, 3) ND_COUNT_CASE(2, 4) ND_COUNT_CASE(2, 5) ND_COUNT_CASE(2, 6)
    ND_COUNT_CASE(2, 7)
    ND_COUNT_CASE(3, 4) ND_COUNT_CASE(3, 5) ND_COUNT_CASE(3, 6) ND_COUNT_CASE(3, 7)
    ND_COUNT_CASE(4, 5) ND_COUNT_CASE(4, 6) ND_COUNT_CASE(4, 7)
    ND_COUNT_CASE(5, 6) ND_COUNT_CASE(5, 7)
    ND_COUNT_CASE(6, 7)
    ND_COUNT_CASE(1, 8) ND_COUNT_CASE(2, 8) ND_COUNT_CASE(3, 8) ND_COUNT_CASE(4, 8)
    ND_COUNT_CASE(5, 8) ND_COUNT_CASE(6, 8) ND_COUNT_CASE(7, 8)
    default: break;
  }
}

}  // namespace nd
