// Index for the s = r+1 path: for r-clique R = {v1 < v2 < ... < vr} the
// s-cliques containing R are R + x for every common neighbour x of R
// (Algorithm 2, Update: I = intersection of N(v) over v in R).  The
// orientation splits I in two disjoint parts, each served by an index built
// once per plan:
//   x > v1: x is an out-neighbour of v1.  Every root v with d = |N+(v)| <= 512
//           keeps the symmetric adjacency bitmap of the subgraph induced on
//           N+(v) (row i, bit j set iff N+(v)[i] ~ N+(v)[j]); the part is the
//           AND of the rows of v2..vr in v1's bitmap.
//   x < v1: x is adjacent to v1 and to each vi, i.e. (x, v1, vi) is a
//           triangle with lowest vertex x.  The apex list of the arc (y, z)
//           holds every such x for (y, z), sorted; the part is the
//           intersection of the lists of the arcs (v1, vi).
// Both indexes are O(m + #triangles) words; nothing per s-clique is stored.
#include "nd_host.h"

namespace nd {

namespace {

int64_t grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  return b < cap ? b : cap;
}

__device__ __forceinline__ uint64_t bitmap_words(int64_t d) {
  return (d >= 1 && d <= 512) ? (uint64_t)d * (uint64_t)((d + 63) / 64) : 0ull;
}

__global__ void k_bitmap_sizes(GraphView g, uint64_t *words) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
       v += (int64_t)gridDim.x * blockDim.x)
    words[v] = bitmap_words(g.rp[v + 1] - g.up[v]);
}

// One block per root of the class: rows built by merging sorted lists in
// LDS, the lower triangle mirrored with LDS atomics, then stored.
template <int W, int NT>
__global__ __launch_bounds__(NT) void k_build_bitmap(GraphView g, const uint32_t *__restrict__ roots,
                                                     uint32_t nroots,
                                                     const uint64_t *__restrict__ bm_off,
                                                     uint64_t *bm) {
  constexpr int D = 64 * W;
  __shared__ int32_t nb[D];
  __shared__ unsigned long long rows[D * W];
  for (uint32_t ri = blockIdx.x; ri < nroots; ri += gridDim.x) {
    const int32_t v = (int32_t)roots[ri];
    const int64_t o = g.up[v];
    const int d = (int)(g.rp[v + 1] - o);
    const int wd = (d + 63) / 64;  // words per row actually stored
    for (int i = threadIdx.x; i < d; i += NT) nb[i] = g.col[o + i];
    for (int i = threadIdx.x; i < d * W; i += NT) rows[i] = 0ull;
    __syncthreads();
    for (int i = threadIdx.x; i < d; i += NT) {
      const int32_t x = nb[i];
      int64_t a = g.up[x];
      const int64_t ae = g.rp[x + 1];
      int q = i + 1;
      while (a < ae && q < d) {
        int32_t y = g.col[a], z = nb[q];
        if (y == z) {
          atomicOr(&rows[i * W + (q >> 6)], 1ull << (q & 63));
          atomicOr(&rows[q * W + (i >> 6)], 1ull << (i & 63));
          a++;
          q++;
        } else if (y < z) {
          a++;
        } else {
          q++;
        }
      }
    }
    __syncthreads();
    uint64_t *dst = bm + bm_off[v];
    for (int e = threadIdx.x; e < d * wd; e += NT) {
      const int i = e / wd, w = e - i * wd;
      dst[e] = rows[i * W + w];
    }
    __syncthreads();
  }
}

__global__ void k_bitmap_classes(GraphView g, uint32_t *lists, int32_t n, uint32_t *sizes) {
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n;
       base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t v = base + threadIdx.x;
    int cls = -1;
    if (v < n) {
      const int64_t d = g.rp[v + 1] - g.up[v];
      if (d >= 1) cls = d <= 64 ? 0 : d <= 128 ? 1 : d <= 256 ? 2 : d <= 512 ? 3 : -1;
    }
#pragma unroll
    for (int c = 0; c < 4; c++)
      wave_append(cls == c, (uint32_t)v, lists + (int64_t)c * n, sizes + c);
  }
}

// Apex-list lengths.  The keys are sorted, so the lanes of a wave mostly
// share an arc: each run of equal arcs is added by its last lane with one
// atomic.
__global__ void k_arc_hist(const uint64_t *__restrict__ keys, uint64_t nk, int xbits,
                           unsigned long long *cnt) {
  const int lane = lane_id();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x + (threadIdx.x & ~(kWave - 1));
       b < (int64_t)nk; b += stride) {  // wave-uniform
    const int64_t i = b + lane;
    const bool in = i < (int64_t)nk;
    const uint64_t a = in ? keys[i] >> xbits : ~0ull;
    const uint64_t an = __shfl_down(a, 1);
    const bool last = in && (lane == kWave - 1 || an != a);
    const uint64_t m = __ballot(last);
    if (last) {
      const uint64_t below = m & lanes_below();
      const int prev = below ? 63 - __clzll((long long)below) : -1;
      atomicAdd(&cnt[a], (unsigned long long)(lane - prev));
    }
  }
}

__global__ void k_apex_values(const uint64_t *__restrict__ keys, uint64_t nk, uint64_t xmask,
                              int32_t *lval) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)nk;
       i += (int64_t)gridDim.x * blockDim.x)
    lval[i] = (int32_t)(keys[i] & xmask);
}

int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) b++;
  return b;
}

}  // namespace

// ---- ranked triangle table (r = 3)

namespace {

// bits of word w of a row that lie strictly above local position i
__device__ __forceinline__ uint64_t above_mask(int i, int w) {
  const int lo = w * 64;
  if (i < lo) return ~0ull;
  if (i >= lo + 63) return 0ull;
  return ~((1ull << (i - lo + 1)) - 1ull);
}

// One wave per bitmap root: triangles per row above the diagonal, prefix
// summed over the root's rows into rowpre (indexed by out-arc position).
__global__ __launch_bounds__(256) void k_rank_rows(GraphView g, const uint64_t *__restrict__ bm_off,
                                                   const uint64_t *__restrict__ bm,
                                                   uint32_t *rowpre) {
  const int wpb = blockDim.x / kWave;
  const int lane = lane_id();
  for (int64_t v = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; v < g.n;
       v += (int64_t)gridDim.x * wpb) {
    const int64_t o = g.up[v];
    const int d = (int)(g.rp[v + 1] - o);
    if (d < 1 || d > 512) continue;
    const int wd = (d + 63) >> 6;
    const uint64_t *rows = bm + bm_off[v];
    uint32_t carry = 0;
    for (int b0 = 0; b0 < d; b0 += kWave) {
      const int i = b0 + lane;
      uint32_t c = 0;
      if (i < d)
        for (int w = 0; w < wd; w++) c += (uint32_t)__popcll(rows[i * wd + w] & above_mask(i, w));
      const uint32_t incl = wave_incl_scan(c);
      if (i < d) rowpre[o + i] = carry + incl - c;
      carry += __shfl(incl, kWave - 1);
    }
  }
}

// bitmap roots: exactly their triangle count; others: hashed capacity
__global__ void k_caps_ranked(GraphView g, float lf, const uint32_t *__restrict__ cnt,
                              uint64_t *cap) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < g.n;
       v += (int64_t)gridDim.x * blockDim.x) {
    const int64_t d = g.rp[v + 1] - g.up[v];
    const uint64_t c = cnt[v];
    uint64_t k = 0;
    if (c != 0) {
      if (d <= 512) {
        k = c;
      } else {
        k = (uint64_t)((double)c / (double)lf + 0.999999);
        if (k < c + 1) k = c + 1;  // an empty slot ends every probe chain
      }
    }
    cap[v] = k;
  }
}

// One wave per bitmap root, a lane per row: the triangles of the row in
// column order at consecutive slots.
__global__ __launch_bounds__(256) void k_insert_ranked(GraphView g, const uint64_t *__restrict__ bm_off,
                                                       const uint64_t *__restrict__ bm,
                                                       const uint32_t *__restrict__ rowpre,
                                                       TableView T) {
  const int wpb = blockDim.x / kWave;
  const int lane = lane_id();
  for (int64_t v = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; v < g.n;
       v += (int64_t)gridDim.x * wpb) {
    const int64_t o = g.up[v];
    const int d = (int)(g.rp[v + 1] - o);
    if (d < 1 || d > 512) continue;
    const int wd = (d + 63) >> 6;
    const uint64_t *rows = bm + bm_off[v];
    const uint64_t base = T.seg[v];
    for (int i = lane; i < d; i += kWave) {
      uint64_t pos = base + rowpre[o + i];
      const int32_t a = g.col[o + i];
      for (int w = 0; w < wd; w++) {
        uint64_t m = rows[i * wd + w] & above_mask(i, w);
        while (m) {
          const int j = w * 64 + __ffsll((unsigned long long)m) - 1;
          m &= m - 1;
          const int32_t Rv[3] = {(int32_t)v, a, g.col[o + j]};
          T.slots[pos].key = make_key<3>(Rv, T.bits).lo;  // one word for r = 3
          T.v1[pos] = (int32_t)v;
          pos++;
        }
      }
    }
  }
}

}  // namespace

void ranked_caps(const OrientedGraph &g, FastIndex *fx, const uint32_t *tri_per_root, float lf,
                 uint64_t *cap, hipStream_t st) {
  fx->rowpre.reset((size_t)g.nnz + 1);
  if (g.n == 0) return;
  const GraphView gv = g.view();
  hipLaunchKernelGGL(k_rank_rows, dim3((unsigned)grid_for(g.n, 4)), dim3(256), 0, st, gv,
                     fx->bm_off.get(), fx->bm.get(), fx->rowpre.get());
  hipLaunchKernelGGL(k_caps_ranked, dim3((unsigned)grid_for(g.n, 256)), dim3(256), 0, st, gv, lf,
                     tri_per_root, cap);
}

void ranked_insert(const OrientedGraph &g, const FastIndex &fx, const TableView &T,
                   hipStream_t st) {
  if (g.n == 0) return;
  hipLaunchKernelGGL(k_insert_ranked, dim3((unsigned)grid_for(g.n, 4)), dim3(256), 0, st,
                     g.view(), fx.bm_off.get(), fx.bm.get(), fx.rowpre.get(), T);
}

void build_fast_index(const OrientedGraph &g, FastIndex *fx, Counters *dctr, hipStream_t st,
                      uint32_t *tri_per_root) {
  const int32_t n = g.n;
  const GraphView gv = g.view();
  fx->bm_off.reset((size_t)n + 1);
  fx->lptr.reset((size_t)g.nnz + 1);
  fill_u64(fx->lptr.get(), 0, g.nnz + 1, st);
  if (n == 0) {
    fill_u64(fx->bm_off.get(), 0, 1, st);
    fx->bm.reset(1);
    fx->lval.reset(1);
    return;
  }
  // ---- bitmaps
  fill_u64(fx->bm_off.get() + n, 0, 1, st);
  hipLaunchKernelGGL(k_bitmap_sizes, dim3((unsigned)grid_for(n, 256)), dim3(256), 0, st, gv,
                     fx->bm_off.get());
  scan_exclusive_u64(fx->bm_off.get(), fx->bm_off.get(), (int64_t)n + 1, st);
  uint64_t words = 0;
  read_back(&words, fx->bm_off.get() + n, 8, st);
  fx->bm_words = words;
  fx->bm.reset(words ? words : 1);
  {
    DevBuf<uint32_t> lists((size_t)4 * n);
    fill_u32(dctr->class_size, 0, 4, st);
    hipLaunchKernelGGL(k_bitmap_classes, dim3((unsigned)grid_for(n, 256)), dim3(256), 0, st, gv,
                       lists.get(), n, dctr->class_size);
    uint32_t sz[4];
    read_back(sz, dctr->class_size, sizeof(sz), st);
    auto grid = [](uint32_t k) { return dim3(k < 262144u ? k : 262144u); };
    if (sz[0])
      hipLaunchKernelGGL((k_build_bitmap<1, 64>), grid(sz[0]), dim3(64), 0, st, gv, lists.get(),
                         sz[0], fx->bm_off.get(), fx->bm.get());
    if (sz[1])
      hipLaunchKernelGGL((k_build_bitmap<2, 128>), grid(sz[1]), dim3(128), 0, st, gv,
                         lists.get() + n, sz[1], fx->bm_off.get(), fx->bm.get());
    if (sz[2])
      hipLaunchKernelGGL((k_build_bitmap<4, 256>), grid(sz[2]), dim3(256), 0, st, gv,
                         lists.get() + 2 * (int64_t)n, sz[2], fx->bm_off.get(), fx->bm.get());
    if (sz[3])
      hipLaunchKernelGGL((k_build_bitmap<8, 512>), grid(sz[3]), dim3(512), 0, st, gv,
                         lists.get() + 3 * (int64_t)n, sz[3], fx->bm_off.get(), fx->bm.get());
  }
  // ---- apex lists
  DevBuf<uint32_t> own_tri;
  uint32_t *tri = tri_per_root;
  if (!tri) {
    own_tri.reset((size_t)n);
    tri = own_tri.get();
  }
  count_rcliques(g, 3, tri, st);
  DevBuf<uint64_t> cur((size_t)n + 1);
  widen_u32_to_u64(tri, cur.get(), n, st);
  fill_u64(cur.get() + n, 0, 1, st);
  scan_exclusive_u64(cur.get(), cur.get(), (int64_t)n + 1, st);
  read_back(&fx->n_tri, cur.get() + n, 8, st);
  const uint64_t T = fx->n_tri;
  fx->lval.reset(T ? T : 1);
  if (T) {
    const int xb = bits_for((uint64_t)(n - 1)) < 1 ? 1 : bits_for((uint64_t)(n - 1));
    const int eb = bits_for((uint64_t)g.nnz);
    DevBuf<uint64_t> keys(T);
    list_apex_keys(g, cur.get(), keys.get(), xb, dctr, st);
    // the keys arrive grouped by x in ascending order, so a stable sort on
    // the arc bits alone leaves each list sorted by x
    radix_sort(keys.get(), nullptr, (int64_t)T, xb + eb, st, xb);
    DevBuf<uint64_t> cnt((size_t)g.nnz + 1);
    fill_u64(cnt.get(), 0, g.nnz + 1, st);
    hipLaunchKernelGGL(k_arc_hist, dim3((unsigned)grid_for(T, 256)), dim3(256), 0, st, keys.get(),
                       T, xb, (unsigned long long *)cnt.get());
    scan_exclusive_u64(cnt.get(), fx->lptr.get(), g.nnz + 1, st);
    hipLaunchKernelGGL(k_apex_values, dim3((unsigned)grid_for(T, 256)), dim3(256), 0, st,
                       keys.get(), T, (1ull << xb) - 1ull, fx->lval.get());
  }
}

}  // namespace nd
