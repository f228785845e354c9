// Ingest + validation (the input must be a simple undirected graph in CSR,
// paper Section 2 "Graph Notation" and "Graph Storage") and the
// orientation + relabeling step (Section 2 "O(alpha)-Orientation",
// Algorithm 2 Orient, Section 4.4 "Graph Relabeling").
//
// Orientations (a total order; arcs point from lower to higher rank):
//   0  degree order: rank by (degree, id).  Every out-neighbour of v has
//      degree >= deg(v), so out-degree <= sqrt(2m).
//   1  core order: vertices ranked by the round in which bulk k-core peeling
//      removes them (ties by id); out-degree <= the degeneracy.
// Vertex ids are then replaced by ranks, so "sorted by id" = "discovery
// order" and the out-neighbours of v are the suffix of its row above v.
#include <vector>

#include "nd_host.h"

namespace nd {

namespace {

int64_t grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  return b < cap ? b : cap;
}

__device__ __forceinline__ int32_t source_of(const int64_t *__restrict__ rp, int32_t n, int64_t a) {
  // largest v with rp[v] <= a
  int32_t lo = 0, hi = n;
  while (lo < hi) {
    int32_t mid = lo + ((hi - lo + 1) >> 1);
    if (rp[mid] <= a) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_validate_rows(int32_t n, int64_t nnz, const int64_t *__restrict__ rp,
                                uint32_t *err) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    int64_t a = rp[v], b = rp[v + 1];
    bool bad = b < a || a < 0 || b > nnz;
    if (v == 0 && a != 0) bad = true;
    if (v == n - 1 && b != nnz) bad = true;
    if (bad) atomicOr(err, kErrGraph);
  }
}

__global__ void k_validate_arcs(int32_t n, int64_t nnz, const int64_t *__restrict__ rp,
                                const int32_t *__restrict__ col, uint32_t *err) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nnz;
       a += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = source_of(rp, n, a);
    int32_t u = col[a];
    bool bad = u < 0 || u >= n || u == v;
    if (!bad && a > rp[v] && col[a - 1] >= u) bad = true;
    if (!bad && !sorted_contains(col, rp[u], rp[u + 1], v)) bad = true;
    if (bad) atomicOr(err, kErrGraph);
  }
}

__global__ void k_degree_keys(int32_t n, const int64_t *__restrict__ rp, uint64_t *keys,
                              uint32_t *vals) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    keys[v] = (uint64_t)(rp[v + 1] - rp[v]);
    vals[v] = (uint32_t)v;
  }
}

__global__ void k_invert(int32_t n, const uint32_t *__restrict__ new2old, int32_t *old2new,
                         int32_t *new2old_i32, const int64_t *__restrict__ rp, uint64_t *newdeg) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    uint32_t v = new2old[x];
    old2new[v] = (int32_t)x;
    new2old_i32[x] = (int32_t)v;
    newdeg[x] = (uint64_t)(rp[v + 1] - rp[v]);
  }
}

__global__ void k_arc_keys(int32_t n, int64_t nnz, const int64_t *__restrict__ rp,
                           const int32_t *__restrict__ col, const int32_t *__restrict__ old2new,
                           int bits, uint64_t *keys) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nnz;
       a += (int64_t)gridDim.x * blockDim.x) {
    int32_t v = source_of(rp, n, a);
    keys[a] = ((uint64_t)(uint32_t)old2new[v] << bits) | (uint64_t)(uint32_t)old2new[col[a]];
  }
}

__global__ void k_arc_cols(int64_t nnz, const uint64_t *__restrict__ keys, uint64_t mask,
                           int32_t *col) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < nnz;
       a += (int64_t)gridDim.x * blockDim.x)
    col[a] = (int32_t)(keys[a] & mask);
}

__global__ void k_out_start(int32_t n, const int64_t *__restrict__ rp,
                            const int32_t *__restrict__ col, int64_t *up, uint32_t *outdeg) {
  for (int64_t x = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < n;
       x += (int64_t)gridDim.x * blockDim.x) {
    int64_t lo = rp[x], hi = rp[x + 1];
    int64_t end = hi;
    while (lo < hi) {  // first position holding a neighbour > x
      int64_t mid = (lo + hi) >> 1;
      if (col[mid] > (int32_t)x) hi = mid;
      else lo = mid + 1;
    }
    up[x] = lo;
    outdeg[x] = (uint32_t)(end - lo);
  }
}

// ---- core order: bulk k-core peeling on vertices (the (1,2) case of the
// peel, on the input graph), recording each vertex's removal round.
__global__ void k_core_init(int32_t n, const int64_t *__restrict__ rp, uint32_t *deg,
                            uint32_t *round) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    deg[v] = (uint32_t)(rp[v + 1] - rp[v]);
    round[v] = kLive;
  }
}

__global__ void k_core_min(int32_t n, const uint32_t *__restrict__ deg,
                           const uint32_t *__restrict__ round, uint32_t *out) {
  uint32_t m = 0xFFFFFFFFu;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x)
    if (round[v] == kLive && deg[v] < m) m = deg[v];
  m = wave_min_u32(m);
  if (lane_id() == 0 && m != 0xFFFFFFFFu) atomicMin(out, m);
}

__global__ void k_core_frontier(int32_t n, const uint32_t *__restrict__ deg,
                                const uint32_t *__restrict__ round, uint32_t k, uint32_t *F,
                                uint32_t *nF) {
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n;
       base += (int64_t)gridDim.x * blockDim.x) {
    int64_t v = base + threadIdx.x;
    bool want = v < n && round[v] == kLive && deg[v] <= k;
    wave_append(want, (uint32_t)v, F, nF);
  }
}

__global__ void k_core_stamp(const uint32_t *__restrict__ F, uint32_t nF, uint32_t t,
                             uint32_t *round) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nF;
       i += (int64_t)gridDim.x * blockDim.x)
    round[F[i]] = t;
}

// one wave per removed vertex: decrement live neighbours, append crossings
__global__ __launch_bounds__(256) void k_core_peel(const int64_t *__restrict__ rp,
                                                   const int32_t *__restrict__ col,
                                                   const uint32_t *__restrict__ F, uint32_t nF,
                                                   uint32_t k, uint32_t *deg,
                                                   const uint32_t *__restrict__ round,
                                                   uint32_t *Fn, uint32_t *nFn) {
  int wpb = blockDim.x / kWave;
  for (int64_t i = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; i < nF;
       i += (int64_t)gridDim.x * wpb) {
    uint32_t v = F[i];
    for (int64_t a = rp[v]; a < rp[v + 1]; a += kWave) {
      int64_t e = a + lane_id();
      bool want = false;
      uint32_t u = 0;
      if (e < rp[v + 1]) {
        u = (uint32_t)col[e];
        if (round[u] == kLive) {
          uint32_t old = atomicSub(&deg[u], 1u);
          want = old == k + 1;
        }
      }
      wave_append(want, u, Fn, nFn);
    }
  }
}

void core_rounds(int32_t n, const int64_t *rp, const int32_t *col, uint32_t *round_out,
                 hipStream_t st) {
  DevBuf<uint32_t> deg((size_t)n), F((size_t)n), Fn((size_t)n), ctr(4);
  int64_t gb = grid_for(n, 256);
  hipLaunchKernelGGL(k_core_init, dim3((unsigned)gb), dim3(256), 0, st, n, rp, deg.get(),
                     round_out);
  uint32_t k = 0, t = 0, nF = 0;
  int64_t done = 0;
  uint32_t h[2];
  while (done < n) {
    if (nF == 0) {
      fill_u32(ctr.get(), 0xFFFFFFFFu, 1, st);
      fill_u32(ctr.get() + 1, 0, 1, st);
      hipLaunchKernelGGL(k_core_min, dim3((unsigned)gb), dim3(256), 0, st, n, deg.get(),
                         round_out, ctr.get());
      read_back(h, ctr.get(), 4, st);
      if (h[0] > k) k = h[0];
      hipLaunchKernelGGL(k_core_frontier, dim3((unsigned)gb), dim3(256), 0, st, n, deg.get(),
                         round_out, k, F.get(), ctr.get() + 1);
      read_back(&nF, ctr.get() + 1, 4, st);
      if (nF == 0) break;
    }
    hipLaunchKernelGGL(k_core_stamp, dim3((unsigned)grid_for(nF, 256)), dim3(256), 0, st, F.get(),
                       nF, t, round_out);
    fill_u32(ctr.get() + 2, 0, 1, st);
    hipLaunchKernelGGL(k_core_peel, dim3((unsigned)grid_for(nF, 4, 16384)), dim3(256), 0, st, rp,
                       col, F.get(), nF, k, deg.get(), round_out, Fn.get(), ctr.get() + 2);
    done += nF;
    read_back(&nF, ctr.get() + 2, 4, st);
    std::swap(F.p, Fn.p);
    t++;
  }
}

__global__ void k_round_keys(int32_t n, const uint32_t *__restrict__ round, uint64_t *keys,
                             uint32_t *vals) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    keys[v] = round[v];
    vals[v] = (uint32_t)v;
  }
}

int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) b++;
  return b;
}

}  // namespace

uint32_t validate_csr(int32_t n, int64_t nnz, const int64_t *rp, const int32_t *col,
                      Counters *dctr, hipStream_t st) {
  if (n == 0) return 0;
  uint32_t *err = &dctr->err;
  fill_u32(err, 0, 1, st);
  hipLaunchKernelGGL(k_validate_rows, dim3((unsigned)grid_for(n, 256)), dim3(256), 0, st, n, nnz,
                     rp, err);
  uint32_t h = 0;
  read_back(&h, err, 4, st);
  if (h) return h;
  if (nnz > 0)
    hipLaunchKernelGGL(k_validate_arcs, dim3((unsigned)grid_for(nnz, 256)), dim3(256), 0, st, n,
                       nnz, rp, col, err);
  read_back(&h, err, 4, st);
  return h;
}

void orient_relabel(int32_t n, int64_t nnz, const int64_t *rp, const int32_t *col, int mode,
                    OrientedGraph *og, hipStream_t st) {
  og->n = n;
  og->nnz = nnz;
  og->rp.reset((size_t)n + 1);
  og->up.reset(n > 0 ? (size_t)n : 1);
  og->col.reset(nnz > 0 ? (size_t)nnz : 1);
  og->new2old.reset(n > 0 ? (size_t)n : 1);
  if (n == 0) {
    fill_u64((uint64_t *)og->rp.get(), 0, 1, st);
    og->max_out = 0;
    return;
  }
  int64_t gb = grid_for(n, 256);
  // 1. rank order
  DevBuf<uint64_t> keys((size_t)n);
  DevBuf<uint32_t> order((size_t)n);
  int key_bits;
  if (mode == 1) {
    DevBuf<uint32_t> round((size_t)n);
    core_rounds(n, rp, col, round.get(), st);
    hipLaunchKernelGGL(k_round_keys, dim3((unsigned)gb), dim3(256), 0, st, n, round.get(),
                       keys.get(), order.get());
    key_bits = 32;
  } else {
    hipLaunchKernelGGL(k_degree_keys, dim3((unsigned)gb), dim3(256), 0, st, n, rp, keys.get(),
                       order.get());
    key_bits = bits_for((uint64_t)nnz);
  }
  radix_sort(keys.get(), order.get(), n, key_bits, st);
  // 2. inverse map and relabeled degrees
  DevBuf<int32_t> old2new((size_t)n);
  DevBuf<uint64_t> newdeg((size_t)n + 1);
  fill_u64(newdeg.get() + n, 0, 1, st);
  hipLaunchKernelGGL(k_invert, dim3((unsigned)gb), dim3(256), 0, st, n, order.get(),
                     old2new.get(), og->new2old.get(), rp, newdeg.get());
  scan_exclusive_u64(newdeg.get(), (uint64_t *)og->rp.get(), (int64_t)n + 1, st);
  // 3. relabeled arcs, sorted by (new source, new target)
  if (nnz > 0) {
    int vb = bits_for((uint64_t)(n - 1));
    if (vb < 1) vb = 1;
    DevBuf<uint64_t> akeys((size_t)nnz);
    hipLaunchKernelGGL(k_arc_keys, dim3((unsigned)grid_for(nnz, 256)), dim3(256), 0, st, n, nnz,
                       rp, col, old2new.get(), vb, akeys.get());
    radix_sort(akeys.get(), nullptr, nnz, 2 * vb, st);
    hipLaunchKernelGGL(k_arc_cols, dim3((unsigned)grid_for(nnz, 256)), dim3(256), 0, st, nnz,
                       akeys.get(), (1ull << vb) - 1ull, og->col.get());
  }
  // 4. start of the out-neighbours in each row
  DevBuf<uint32_t> outdeg((size_t)n);
  hipLaunchKernelGGL(k_out_start, dim3((unsigned)gb), dim3(256), 0, st, n, og->rp.get(),
                     og->col.get(), og->up.get(), outdeg.get());
  og->max_out = max_u32_host(outdeg.get(), n, st);
}

}  // namespace nd
