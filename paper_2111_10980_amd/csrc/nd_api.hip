// Host runtime and C ABI (include/nd.h).
//
// Memory.  A plan's own device state (relabeled graph, r-clique table, index,
// round control block, liveness bitmaps) comes from the device's
// stream-ordered memory pool (hipMallocAsync / hipFreeAsync on the plan's
// stream) with the release threshold raised, so buffers freed by one plan
// are reused by the next one without returning to the driver;
// nd_release_cached() trims the pool.  Everything a run needs beyond that
// (bucket lists, per-frontier scratch, round records, round trace, sort
// buffers) is carved from the caller's workspace: nd_run allocates nothing.
// run_ws_bytes() adds up exactly the buffers a run carves, so
// nd_plan_sizes reports the workspace size a run needs.
//
// The peel loop (Algorithm 2, "while finished < |T|") is driven by the
// device (nd_peel.hip); the host queues rounds and reads the round state
// every few rounds.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/nd.h"
#include "nd_host.h"

namespace nd {

namespace {

thread_local hipStream_t g_stream = nullptr;
thread_local std::string g_last_error;
thread_local Workspace *g_ws = nullptr;

struct Failure {
  nd_status st;
};

[[noreturn]] void fail(nd_status st, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  throw Failure{st};
}

void hip_check(hipError_t e, const char *what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) fail(ND_ENOMEM, "%s: %s", what, hipGetErrorString(e));
    fail(ND_EHIP, "%s: %s", what, hipGetErrorString(e));
  }
}

std::once_flag g_pool_once;

void configure_pool() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return;
  hipMemPool_t pool;
  if (hipDeviceGetDefaultMemPool(&pool, dev) == hipSuccess) {
    uint64_t thr = UINT64_MAX;
    hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr);
  }
}

struct StreamScope {
  hipStream_t prev;
  explicit StreamScope(hipStream_t s) : prev(g_stream) {
    std::call_once(g_pool_once, configure_pool);
    g_stream = s;
  }
  ~StreamScope() { g_stream = prev; }
};

// levels covered by the window list of the bucket structure

int64_t grid_for(int64_t n, int threads, int64_t cap = 65536) {
  int64_t b = (n + threads - 1) / threads;
  if (b < 1) b = 1;
  return b < cap ? b : cap;
}

__global__ void k_caps(int64_t n, int r, float lf, const uint32_t *__restrict__ cnt,
                       uint64_t *cap) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    uint64_t c = cnt[v];
    uint64_t k;
    if (r == 1) k = 1;
    else if (c == 0) k = 0;
    else {
      k = (uint64_t)((double)c / (double)lf + 0.999999);
      if (k < c + 1) k = c + 1;  // at least one empty slot ends every probe chain
    }
    cap[v] = k;
  }
}

// out[0] += sum of the slot counts, out[1] = max(out[1], largest count)
__global__ __launch_bounds__(256) void k_sum_slot_counts(const Slot *__restrict__ s, uint64_t n,
                                                         unsigned long long *out) {
  uint64_t acc = 0;
  uint32_t mx = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint32_t c = s[i].cnt;
    acc += c;
    mx = c > mx ? c : mx;
  }
  acc = wave_sum_u64(acc);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint32_t o = __shfl_xor(mx, off);
    mx = o > mx ? o : mx;
  }
  if (lane_id() == 0) {
    if (acc) atomicAdd(&out[0], (unsigned long long)acc);
    if (mx) atomicMax(&out[1], (unsigned long long)mx);
  }
}

// (2,3) run state: every apex list at its full length, every edge alive; no
// vertex has lost a neighbour, each at its full degree.
__global__ void k_r2_init_arcs(const uint64_t *__restrict__ lptr, uint64_t nnz, uint32_t *llen,
                               uint8_t *arcst) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)nnz;
       e += (int64_t)gridDim.x * blockDim.x) {
    llen[e] = (uint32_t)(lptr[e + 1] - lptr[e]);
    arcst[e] = 0;
  }
}

__global__ void k_r2_init_vertices(const int64_t *__restrict__ rp, int32_t n, uint32_t *lost,
                                   uint32_t *deg_at) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n;
       v += (int64_t)gridDim.x * blockDim.x) {
    lost[v] = 0;
    deg_at[v] = (uint32_t)(rp[v + 1] - rp[v]);
  }
}

// A re-run starts from the table as built: counts 0, every r-clique live.
__global__ void k_reset_slots(Slot *s, uint64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n;
       i += (int64_t)gridDim.x * blockDim.x) {
    s[i].cnt = 0;
    s[i].stamp = kLive;
  }
}

// Canonical row order: key of row idx[i] from its vertices [from, to) (ids
// ascending in the row), first vertex most significant, b bits per vertex.
__global__ void k_row_keys(const int32_t *__restrict__ rows, int r, uint64_t n_r,
                           const uint32_t *__restrict__ idx, int from, int to, int b,
                           uint64_t *keys) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n_r;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t *row = rows + (uint64_t)idx[i] * r;
    uint64_t k = 0;
    for (int q = from; q < to; q++) k = (k << b) | (uint64_t)(uint32_t)row[q];
    keys[i] = k;
  }
}

__global__ void k_permute_rows(const int32_t *__restrict__ rows, const uint32_t *__restrict__ kap,
                               const uint32_t *__restrict__ cnt, int r, uint64_t n_r,
                               const uint32_t *__restrict__ idx, int32_t *rows_out,
                               uint32_t *kap_out, uint32_t *cnt_out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n_r;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t j = idx[i];
    for (int q = 0; q < r; q++) rows_out[(uint64_t)i * r + q] = rows[j * r + q];
    kap_out[i] = kap[j];
    if (cnt_out) cnt_out[i] = cnt[j];
  }
}

// ---- batched decomposition: the batch is one disjoint union (kappa is a
// property of each connected component, so the union's kappa of an r-clique
// equals its kappa in its own graph).
struct GraphDesc {
  const int64_t *rp;
  const int32_t *col;
  int32_t n;
  int32_t vo;  // first union id of the graph
  int64_t nnz;
  int64_t eo;  // first union arc of the graph
};

// last g in [0, count) with key[g] <= x (empty graphs share offsets; the
// last of equal offsets is the non-empty one that owns x)
template <class T>
__device__ __forceinline__ int owner_of(const T *__restrict__ key, int count, T x) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (key[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ void k_union_rows(const GraphDesc *__restrict__ gd, const int32_t *__restrict__ vo,
                             int count, int32_t n_total, int64_t nnz_total, int64_t *rp) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v <= n_total;
       v += (int64_t)gridDim.x * blockDim.x) {
    if (v == n_total) {
      rp[v] = nnz_total;
      continue;
    }
    const int g = owner_of<int32_t>(vo, count, (int32_t)v);
    rp[v] = gd[g].eo + gd[g].rp[v - gd[g].vo];
  }
}

__global__ void k_union_cols(const GraphDesc *__restrict__ gd, const int64_t *__restrict__ eo,
                             int count, int64_t nnz_total, int32_t *col, uint32_t *err) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz_total;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int g = owner_of<int64_t>(eo, count, i);
    const int32_t c = gd[g].col[i - gd[g].eo];
    if (c < 0 || c >= gd[g].n) {
      atomicOr(err, kErrGraph);
      col[i] = 0;
    } else {
      col[i] = c + gd[g].vo;
    }
  }
}

// canonical batch output: rows are already grouped by graph and ordered
// within it; only the ids become graph-local
__global__ void k_localise(const int32_t *__restrict__ rcl, const uint32_t *__restrict__ kap,
                           const uint32_t *__restrict__ cnt, int r, uint64_t n_r,
                           const int32_t *__restrict__ gid, const int32_t *__restrict__ vo,
                           int32_t *rcl_out, uint32_t *kap_out, uint32_t *cnt_out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n_r;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int g = gid[i];
    for (int q = 0; q < r; q++) rcl_out[i * r + q] = rcl[i * r + q] - vo[g];
    kap_out[i] = kap[i];
    if (cnt_out) cnt_out[i] = cnt[i];
  }
}

// graph of every output row (its first vertex's graph) and rows per graph
__global__ void k_row_graph(const int32_t *__restrict__ rcl, int r, uint64_t n_r,
                            const int32_t *__restrict__ vo, int count, int32_t *gid,
                            unsigned long long *per_graph) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n_r;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int g = owner_of<int32_t>(vo, count, rcl[i * r]);
    gid[i] = g;
    atomicAdd(&per_graph[g], 1ull);
  }
}

__global__ void k_regroup(const int32_t *__restrict__ rcl, const uint32_t *__restrict__ kap,
                          const uint32_t *__restrict__ cnt, int r, uint64_t n_r,
                          const int32_t *__restrict__ gid, const int32_t *__restrict__ vo,
                          const unsigned long long *__restrict__ off, unsigned long long *cursor,
                          int32_t *rcl_out, uint32_t *kap_out, uint32_t *cnt_out) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n_r;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int g = gid[i];
    const uint64_t at = off[g] + atomicAdd(&cursor[g], 1ull);
    for (int q = 0; q < r; q++) rcl_out[at * r + q] = rcl[i * r + q] - vo[g];
    kap_out[at] = kap[i];
    if (cnt_out) cnt_out[at] = cnt[i];
  }
}

uint64_t binom_u64(int n, int k) {
  uint64_t r = 1;
  for (int i = 1; i <= k; i++) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}

int bits_for(uint64_t maxval) {
  int b = 0;
  while (b < 64 && (maxval >> b) != 0) b++;
  return b;
}

// HIP events created once per plan (a run creates none).
struct EventSet {
  std::vector<hipEvent_t> ev;
  bool ok = true;
  void create(int n) {
    ev.assign((size_t)n, nullptr);
    for (auto &e : ev)
      if (hipEventCreate(&e) != hipSuccess) {
        e = nullptr;
        ok = false;
      }
  }
  ~EventSet() {
    for (auto &e : ev)
      if (e) hipEventDestroy(e);
  }
  hipEvent_t at(int i) const { return ok && i < (int)ev.size() ? ev[i] : nullptr; }
  void mark(int i, hipStream_t st) {
    if (hipEvent_t e = at(i)) hipEventRecord(e, st);
  }
  float between(int a, int b) const {
    float ms = 0;
    hipEvent_t x = at(a), y = at(b);
    if (x && y && hipEventElapsedTime(&ms, x, y) == hipSuccess) return ms;
    return 0;
  }
};

template <class T>
T read_dev(const T *p, hipStream_t st) {
  T h;
  hip_check(hipMemcpyAsync(&h, p, sizeof(T), hipMemcpyDeviceToHost, st), "read back");
  hip_check(hipStreamSynchronize(st), "synchronize");
  return h;
}

}  // namespace

WorkspaceScope::WorkspaceScope(void *base, uint64_t size) : prev(g_ws) {
  ws.base = (char *)base;
  ws.size = size;
  ws.used = 0;
  g_ws = &ws;
}

WorkspaceScope::~WorkspaceScope() { g_ws = prev; }

void hip_ok(hipError_t e, const char *what) { hip_check(e, what); }

void read_back(void *dst, const void *src, size_t bytes, hipStream_t st) {
  hip_check(hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, st), "read back");
  hip_check(hipStreamSynchronize(st), "synchronize");
}

void *dev_alloc(size_t bytes) {
  if (g_ws) {
    const uint64_t b = ws_block(bytes);
    if (g_ws->used + b > g_ws->size)
      fail(ND_ENOMEM, "workspace of %llu bytes exhausted (%llu used, %llu more asked)",
           (unsigned long long)g_ws->size, (unsigned long long)g_ws->used,
           (unsigned long long)b);
    void *p = g_ws->base + g_ws->used;
    g_ws->used += b;
    return p;
  }
  void *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMallocAsync(&p, bytes, g_stream);
  if (e != hipSuccess || !p) {
    hipGetLastError();
    fail(ND_ENOMEM, "device allocation of %zu bytes failed", bytes);
  }
  return p;
}

void dev_free(void *p) {
  if (!p) return;
  if (g_ws && (char *)p >= g_ws->base && (char *)p < g_ws->base + g_ws->size) return;
  hipFreeAsync(p, g_stream);
}

}  // namespace nd

using namespace nd;

struct nd_plan_s {
  hipStream_t st = nullptr;
  int device = 0;     // device current at creation
  int r = 0, s = 0;
  nd_options opt{};
  uint64_t budget = 0;
  OrientedGraph g;
  DevBuf<uint64_t> seg;
  DevBuf<Slot> slots;
  DevBuf<int32_t> v1;
  DevBuf<uint64_t> khi;  // second key words, when the key fields need more than 63 bits
  DevBuf<uint64_t> aseg;  // three levels: last-level table of each arc position
  DevBuf<int32_t> v2s;    // three levels: second vertex of each slot
  DevBuf<uint32_t> occ;
  DevBuf<Counters> ctr;
  DevBuf<unsigned long long> stats;  // kStatLines x kStatStride statistic lines
  DevBuf<unsigned long long> total;  // [0] sum of the counts, [1] largest count
  DevBuf<RoundCtl> rcb;              // device round state of the peel
  RoundCtl *mirror = nullptr;        // its pinned host copy
  FastIndex fx;
  bool fast = false;  // s = r+1 path (bitmaps + apex lists)
  int path = 0;       // peel path: 0 walker, 1 s = r+1 passes, 2 s >= r+2 passes
  uint64_t n_r = 0, n_slots = 0, held = 0;
  int bits = 1;
  bool wide = false;  // two-word r-clique keys
  int levels = 2;     // r-clique table levels: 2, or 3 (r >= 4)
  int runs = 0;
  bool traced = false;
  PeelSuspend susp;          // a peel stopped by a round that outgrew the workspace
  uint64_t susp_n_s = 0;     // its s-clique count
  bool susp_counts = false;  // its initial counts are kept (susp_cnt)
  std::vector<uint32_t> susp_cnt;
  uint64_t rec_need = 0;     // record capacity the next run's workspace provides at least
  uint32_t trace_need = 0;   // round-trace capacity likewise
  std::vector<uint64_t> round_sizes;
  std::vector<uint32_t> round_k;
  uint64_t k_advances = 0;
  float ms_create[3] = {0, 0, 0};
  EventSet ev_create;  // 4: plan creation phases
  EventSet ev_run;     // 5: run phases, 2: count kernels
  EventSet ev_peel;    // timing: 2 * kPeelMaxDepth around the update passes
  hipStream_t graph_stream = nullptr;  // graph_rounds: capture stream of queued rounds
  TableView table() const {
    const bool three = levels == 3;
    return TableView{bits,
                     seg.get(),
                     slots.get(),
                     v1.get(),
                     wide ? khi.get() : nullptr,
                     three ? aseg.get() : nullptr,
                     three ? v2s.get() : nullptr,
                     g.view()};
  }
  ~nd_plan_s() {
    if (mirror) hipHostFree(mirror);
    if (graph_stream) hipStreamDestroy(graph_stream);
  }
};

namespace nd {
namespace {

// Workspace bytes of one run of plan p with the given round capacities: the
// sum of ws_block() over every buffer the run carves (see run_impl).
uint64_t run_ws_bytes(const nd_plan_s *p, uint64_t rec_cap, uint32_t tcap) {
  uint64_t b = 0;
  const uint64_t n_r = p->n_r;
  if (!p->fast) b += count_scliques_ws_bytes(p->g);
  b += peel_ws_bytes(p->r, p->path, n_r, (uint64_t)p->g.nnz, rec_cap, tcap);
  if (p->opt.canonical && n_r > 1) {
    const int r = p->r, bits = p->bits;
    b += ws_buf<int32_t>(n_r * (uint64_t)r) + 2 * ws_buf<uint32_t>(n_r);  // staged outputs
    b += ws_buf<uint64_t>(n_r) + ws_buf<uint32_t>(n_r);                   // keys, order
    if (r * bits <= 64) {
      b += radix_sort_ws_bytes((int64_t)n_r, r * bits, 0, true);
    } else {
      const int h = (r + 1) / 2;
      b += radix_sort_ws_bytes((int64_t)n_r, (r - h) * bits, 0, true) +
           radix_sort_ws_bytes((int64_t)n_r, h * bits, 0, true);
    }
  }
  return b;
}

// bytes of records, for the record capacity a workspace leaves
uint64_t rec_cap_for(const nd_plan_s *p, uint64_t ws_bytes) {
  if (p->path == 0 || p->n_r == 0) return 0;
  uint64_t lo = 0, hi = 1;
  while (run_ws_bytes(p, hi, p->trace_need) <= ws_bytes && hi < (1ull << 40)) hi *= 2;
  while (lo + 1 < hi) {  // largest capacity whose layout fits
    const uint64_t mid = lo + (hi - lo) / 2;
    if (run_ws_bytes(p, mid, p->trace_need) <= ws_bytes) lo = mid;
    else hi = mid;
  }
  return lo;
}

uint64_t required_ws(const nd_plan_s *p) { return run_ws_bytes(p, p->rec_need, p->trace_need); }

}  // namespace
}  // namespace nd

template <class F>
static nd_status guarded(hipStream_t st, F &&f) {
  StreamScope scope(st);
  try {
    f();
    return ND_OK;
  } catch (const Failure &e) {
    return e.st;
  } catch (const std::bad_alloc &) {
    g_last_error = "host allocation failed";
    return ND_ENOMEM;
  } catch (...) {
    g_last_error = "unexpected internal error";
    return ND_EHIP;
  }
}

extern "C" {

const char *nd_status_str(nd_status st) {
  switch (st) {
    case ND_OK: return "ok";
    case ND_EINVAL: return "invalid argument";
    case ND_EGRAPH: return "malformed graph";
    case ND_EKEYWIDTH: return "r-clique key does not fit two 64-bit words";
    case ND_EOVERFLOW: return "count or size overflow";
    case ND_ENOMEM: return "out of device memory or budget";
    case ND_EHIP: return "HIP runtime error";
    case ND_ESTATE: return "wrong call order";
  }
  return "unknown status";
}

const char *nd_last_error(void) { return g_last_error.c_str(); }

nd_status nd_plan_create(const nd_csr *gin, int r, int s, const nd_options *opt,
                         uint64_t hbm_budget_bytes, void *hip_stream, nd_plan *out) {
  if (!out) {
    g_last_error = "out is null";
    return ND_EINVAL;
  }
  *out = nullptr;
  if (!gin) {
    g_last_error = "graph is null";
    return ND_EINVAL;
  }
  if (r < 1 || s <= r || s > ND_MAX_S) {
    g_last_error = "need 1 <= r < s <= ND_MAX_S";
    return ND_EINVAL;
  }
  if (gin->n < 0 || gin->nnz < 0 || (gin->n > 0 && !gin->row_ptr) ||
      (gin->nnz > 0 && !gin->col)) {
    g_last_error = "bad CSR header";
    return ND_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  nd_plan p = new (std::nothrow) nd_plan_s();
  if (!p) return ND_ENOMEM;
  nd_status rc = guarded(st, [&] {
    p->st = st;
    hip_check(hipGetDevice(&p->device), "get device");
    p->r = r;
    p->s = s;
    if (opt) p->opt = *opt;
    if (p->opt.load_factor <= 0.f) p->opt.load_factor = 0.5f;
    if (p->opt.load_factor > 0.9f) fail(ND_EINVAL, "load_factor must be <= 0.9");
    if (p->opt.orient != 0 && p->opt.orient != 1) fail(ND_EINVAL, "orient must be 0 or 1");
    if (p->opt.path != 0 && p->opt.path != 1) fail(ND_EINVAL, "path must be 0 or 1");
    if (p->opt.canonical != 0 && p->opt.canonical != 1) fail(ND_EINVAL, "canonical must be 0 or 1");
    if (p->opt.queue_depth < 0 || p->opt.queue_depth > kPeelMaxDepth)
      fail(ND_EINVAL, "queue_depth must be in 0..%d", kPeelMaxDepth);
    if (p->opt.contract != 0 && p->opt.contract != 1) fail(ND_EINVAL, "contract must be 0 or 1");
    if (p->opt.graph_rounds != 0 && p->opt.graph_rounds != 1)
      fail(ND_EINVAL, "graph_rounds must be 0 or 1");
    if (p->opt.levels != 0 && p->opt.levels != 2 && p->opt.levels != 3)
      fail(ND_EINVAL, "levels must be 0, 2 or 3");
    if (p->opt.levels == 3 && r < 4) fail(ND_EINVAL, "three-level tables need r >= 4");
    p->levels = p->opt.levels == 3 ? 3 : 2;
    p->fast = (s == r + 1) && r >= 2 && r <= 6 && p->opt.path == 0;
    p->path = p->fast ? 1 : (s >= r + 2 && p->opt.path == 0 ? 2 : 0);
    p->budget = hbm_budget_bytes;
    const int32_t n = gin->n;
    // every event, pinned buffer and device buffer a run uses belongs to the plan
    // or to the run's workspace, so a run itself allocates nothing
    p->ev_create.create(4);
    p->ev_run.create(7);
    if (p->opt.timing) p->ev_peel.create(2 * kPeelMaxDepth);
    if (p->opt.graph_rounds)
      hip_check(hipStreamCreateWithFlags(&p->graph_stream, hipStreamNonBlocking),
                "create the capture stream");
    if (hipHostMalloc((void **)&p->mirror, sizeof(RoundCtl), hipHostMallocDefault) != hipSuccess) {
      hipGetLastError();
      p->mirror = nullptr;
      fail(ND_ENOMEM, "pinned host allocation failed");
    }
    EventSet &tm = p->ev_create;
    tm.mark(0, st);
    p->ctr.reset(1);
    p->stats.reset((size_t)kStatLines * kStatStride);
    p->total.reset(2);
    p->rcb.reset(1);
    fill_u32((uint32_t *)p->ctr.get(), 0, sizeof(Counters) / 4, st);
    if (validate_csr(n, gin->nnz, gin->row_ptr, gin->col, p->ctr.get(), st))
      fail(ND_EGRAPH, "CSR is not a simple symmetric graph with sorted rows");
    tm.mark(1, st);
    int vb = bits_for(n > 1 ? (uint64_t)(n - 1) : 1);
    p->bits = vb < 1 ? 1 : vb;
    // r-clique keys: the vertices after the levels' own (r-1 with two
    // levels, r-2 with three), `bits` each, in one word, or in two when they
    // need more than 63 bits
    const int key_bits = (r - (p->levels - 1)) * p->bits;
    if (key_bits > 126) fail(ND_EKEYWIDTH, "r-clique key needs %d bits (limit 126)", key_bits);
    p->wide = key_bits > 63;
    const uint64_t fixed_bytes = ws_buf<Counters>(1) + ws_buf<unsigned long long>(
                                     (uint64_t)kStatLines * kStatStride) +
                                 ws_buf<unsigned long long>(2) + ws_buf<RoundCtl>(1);
    uint64_t graph_bytes = (uint64_t)(n + 1) * 8 * 2 + (uint64_t)gin->nnz * 4 + (uint64_t)n * 4;
    if (p->budget && graph_bytes > p->budget) fail(ND_ENOMEM, "graph exceeds the HBM budget");
    orient_relabel(n, gin->nnz, gin->row_ptr, gin->col, p->opt.orient, &p->g, st);
    tm.mark(2, st);
    // r-clique table: count per first vertex, capacities, prefix sum.  For
    // (3,4)-type plans the triangles of bitmap roots are placed by rank
    // (ordered within a root), so the bitmaps are built first.  Three-level
    // tables count per out-arc (v1, v2) instead and give each arc position
    // its own last-level table.
    const bool ranked = p->fast && r == 3;
    const bool three = p->levels == 3;
    const int64_t n_units = three ? p->g.nnz : (int64_t)n;  // last-level tables
    DevBuf<uint32_t> cnt(n_units + 1);
    uint64_t *useg = nullptr;
    if (ranked)  // the index counts the triangles per root on the way
      build_fast_index(p->g, &p->fx, p->ctr.get(), st, cnt.get());
    else if (three)
      count_rcliques_arcs(p->g, r, cnt.get(), st);
    else
      count_rcliques(p->g, r, cnt.get(), st);
    if (three) {
      p->seg.reset(1);  // the middle level is the CSR row itself
      p->aseg.reset((size_t)n_units + 1);
      useg = p->aseg.get();
    } else {
      p->seg.reset((size_t)n + 1);
      useg = p->seg.get();
    }
    fill_u64(useg + n_units, 0, 1, st);
    if (ranked)
      ranked_caps(p->g, &p->fx, cnt.get(), p->opt.load_factor, useg, st);
    else if (n_units > 0)
      hipLaunchKernelGGL(k_caps, dim3((unsigned)grid_for(n_units, 256)), dim3(256), 0, st,
                         n_units, r, p->opt.load_factor, cnt.get(), useg);
    scan_exclusive_u64(useg, useg, n_units + 1, st);
    fill_u64((uint64_t *)&p->ctr.get()->n_s, 0, 1, st);
    sum_u32(cnt.get(), n_units, (uint64_t *)&p->ctr.get()->n_s, st);
    p->n_slots = read_dev(useg + n_units, st);
    p->n_r = read_dev((uint64_t *)&p->ctr.get()->n_s, st);
    if (p->n_slots >= (1ull << 32) - 1)
      fail(ND_EOVERFLOW, "table needs %llu slots (limit 2^32-1)", (unsigned long long)p->n_slots);
    // round records carry the frontier position as a signed 32-bit int
    if (p->n_r > 0x7FFFFFFFull)
      fail(ND_EOVERFLOW, "%llu r-cliques (limit 2^31-1)", (unsigned long long)p->n_r);
    // round capacities the workspace provides (records only on the split paths)
    // round capacities the workspace provides.  A round's records are its
    // candidate s-cliques (at most the s-cliques its frontier still lies in);
    // the largest round of rMAT-18 (3,4) writes 4.8 n_r of them, so the
    // default leaves room for 8 n_r (s = r+1) or 4 n_r candidates with 16 n_r
    // out-arcs (s >= r+2).  A round that still needs more stops the run, and
    // the plan then reports the larger workspace.
    if (p->path != 0)
      p->rec_need = p->opt.record_cap
                        ? p->opt.record_cap
                        : std::max<uint64_t>((p->path == 1 ? 8 : 4) * p->n_r, 1ull << 18);
    // rounds <= n_r; 2^20 rounds (8 MB of trace) cover every measured peel
    p->trace_need = p->opt.trace_cap
                        ? p->opt.trace_cap
                        : (uint32_t)std::max<uint64_t>(1, std::min<uint64_t>(p->n_r, 1u << 20));
    uint64_t table_bytes =
        p->n_slots * (sizeof(Slot) + 4 + (p->wide ? 8 : 0) + (three ? 4 : 0)) +
        p->n_r * 4 * 5 + (three ? ((uint64_t)n_units + 1) * 8 : 0);
    p->held = graph_bytes + table_bytes + (uint64_t)(n + 1) * 8 + fixed_bytes;
    // the budget covers the plan and the workspace of its run; checked before
    // the table is allocated
    if (p->budget && p->held + required_ws(p) > p->budget)
      fail(ND_ENOMEM, "plan needs %llu bytes and its run a workspace of %llu, budget %llu",
           (unsigned long long)p->held, (unsigned long long)required_ws(p),
           (unsigned long long)p->budget);
    p->slots.reset(p->n_slots ? p->n_slots : 1);
    p->v1.reset(p->n_slots ? p->n_slots : 1);
    if (p->wide) p->khi.reset(p->n_slots ? p->n_slots : 1);
    if (three) p->v2s.reset(p->n_slots ? p->n_slots : 1);
    fill_slots(p->slots.get(), (int64_t)p->n_slots, st);
    fill_u32(&p->ctr.get()->err, 0, 1, st);
    if (ranked) {
      ranked_insert(p->g, p->fx, p->table(), st);
      insert_rcliques_heavy3(p->g, p->table(), p->ctr.get(), st);
    } else {
      insert_rcliques(p->g, r, p->table(), p->ctr.get(), st);
    }
    p->occ.reset(p->n_r ? p->n_r : 1);
    occupied_list(p->slots.get(), p->n_slots, p->occ.get(), st);
    uint32_t err = read_dev(&p->ctr.get()->err, st);
    if (err) fail(ND_EHIP, "r-clique table build failed (flags %u)", err);
    if (p->fast) {
      if (!ranked) build_fast_index(p->g, &p->fx, p->ctr.get(), st);
      build_slot_loc(p->g, r, p->table(), p->n_slots, &p->fx, st);
      p->held += p->fx.bm_words * 8 + p->fx.n_tri * 4 + (uint64_t)(gin->nnz + 1) * 8 +
                 p->n_slots * 8;
      if (r == 2) {  // (2,3) run state: bitmaps, apex lists, edge states, loss counters
        p->fx.alive.reset(p->fx.bm_words ? p->fx.bm_words : 1);
        p->fx.lvr.reset(p->fx.n_tri ? p->fx.n_tri : 1);
        p->fx.llen.reset((size_t)gin->nnz + 1);
        p->fx.arcst.reset((size_t)gin->nnz + 1);
        p->fx.lost.reset(n > 0 ? (size_t)n : 1);
        p->fx.deg_at.reset(n > 0 ? (size_t)n : 1);
        p->held += 8 * (p->fx.bm_words + 1) + 4 * (p->fx.n_tri + 1) + 5 * (uint64_t)(gin->nnz + 1) +
                   8 * (uint64_t)(n + 1);
      }
      if (r == 3) {  // liveness and frontier bits, reset by every run
        const uint64_t bw = p->fx.bm_words ? p->fx.bm_words : 1;
        const uint64_t aw = (p->fx.n_tri + 63) / 64 ? (p->fx.n_tri + 63) / 64 : 1;
        p->fx.alive.reset(bw);
        p->fx.front.reset(bw);
        p->fx.alive_apex.reset(aw);
        p->fx.front_apex.reset(aw);
        p->held += 16 * (bw + aw);
      }
      if (p->budget && p->held + required_ws(p) > p->budget)
        fail(ND_ENOMEM, "plan needs %llu bytes and its run a workspace of %llu, budget %llu",
             (unsigned long long)p->held, (unsigned long long)required_ws(p),
             (unsigned long long)p->budget);
    }
    tm.mark(3, st);
    hip_check(hipStreamSynchronize(st), "synchronize");
    hip_check(hipGetLastError(), "kernel launch");
    p->ms_create[0] = tm.between(0, 1);
    p->ms_create[1] = tm.between(1, 2);
    p->ms_create[2] = tm.between(2, 3);
  });
  if (rc != ND_OK) {
    {
      StreamScope scope(st);
      delete p;
    }
    return rc;
  }
  *out = p;
  return ND_OK;
}

nd_status nd_plan_sizes(nd_plan p, uint64_t *n_r, uint64_t *workspace_bytes,
                        uint64_t *plan_bytes) {
  if (!p) {
    g_last_error = "plan is null";
    return ND_EINVAL;
  }
  if (n_r) *n_r = p->n_r;
  if (workspace_bytes) *workspace_bytes = required_ws(p);
  if (plan_bytes) *plan_bytes = p->held;
  return ND_OK;
}

}  // extern "C"

namespace {

// The run (a4-a8) of plan p inside an active workspace scope: every buffer
// below is carved from the workspace in the order run_ws_bytes counts them.
void run_impl(nd_plan p, int32_t *rcl_dev, uint32_t *kappa_dev, uint32_t *counts_dev,
              nd_stats *stats) {
  hipStream_t st = p->st;
  const int r = p->r, s = p->s;
  Counters *dc = p->ctr.get();
  EventSet &tm = p->ev_run;  // 0..4 phases, 5/6 around the count listing
  const bool timing = p->opt.timing != 0;
  float count_kernel_ms = 0, peel_kernel_ms = 0;
  uint32_t count_launches = 0, peel_launches = 0;
  // what is left of the workspace (a batch run carves its own buffers first)
  const uint64_t rec_cap = rec_cap_for(p, g_ws->size - g_ws->used);
  const uint32_t tcap = p->trace_need;
  const bool canon = p->opt.canonical && p->n_r > 1;
  // A peel that stopped at a round the last workspace could not hold goes on
  // from that round: the slots, statistics and round control are the plan's,
  // the rest of its state was kept in host memory.  (Not when this run asks
  // for initial counts that run did not take.)
  const bool want_counts = counts_dev != nullptr;
  if (p->susp.on && want_counts && !p->susp_counts) p->susp.on = false;
  const bool resume = p->susp.on;
  tm.mark(0, st);
  if (!resume && p->runs > 0 && p->n_slots)  // a re-run starts from the table as built
    hipLaunchKernelGGL(k_reset_slots, dim3((unsigned)grid_for(p->n_slots, 256, 16384)),
                       dim3(256), 0, st, p->slots.get(), p->n_slots);
  p->runs++;
  p->traced = false;
  DevBuf<int32_t> rows_tmp;
  DevBuf<uint32_t> kap_tmp, cnt_tmp;
  if (canon) {
    rows_tmp.reset(p->n_r * (uint64_t)r);
    kap_tmp.reset(p->n_r);
    cnt_tmp.reset(p->n_r);
  }
  int32_t *rows_out = canon ? rows_tmp.get() : rcl_dev;
  uint32_t *kap_out = canon ? kap_tmp.get() : kappa_dev;
  uint32_t *cnt_out = canon ? cnt_tmp.get() : counts_dev;
  uint64_t n_s = p->susp_n_s;
  Counters hc{};
  if (resume) {
    if (cnt_out &&
        hipMemcpyAsync(cnt_out, p->susp_cnt.data(), 4 * p->n_r, hipMemcpyHostToDevice, st) !=
            hipSuccess)
      fail(ND_EHIP, "restore the initial counts");
    tm.mark(1, st);
  } else {
    // ---- count (Count-Func)
    fill_u32((uint32_t *)dc, 0, sizeof(Counters) / 4, st);
    fill_u64((uint64_t *)p->stats.get(), 0, (int64_t)kStatLines * kStatStride, st);
    if (p->fast) {
      if (timing) tm.mark(5, st);
      count_direct(p->g, r, p->table(), p->fx, p->occ.get(), p->n_r, dc, st);
      if (timing) tm.mark(6, st);
    } else {
      count_scliques(p->g, r, s, p->table(), dc, p->stats.get(), st,
                     timing ? tm.at(5) : nullptr, timing ? tm.at(6) : nullptr);
      stats_collect(p->stats.get(), dc, st);
      fill_u64((uint64_t *)p->stats.get(), 0, (int64_t)kStatLines * kStatStride, st);
    }
    unsigned long long *total = p->total.get();
    fill_u64((uint64_t *)total, 0, 2, st);
    if (p->n_slots)
      hipLaunchKernelGGL(k_sum_slot_counts, dim3((unsigned)grid_for(p->n_slots, 256 * 16, 4096)),
                         dim3(256), 0, st, p->slots.get(), p->n_slots, total);
    hc = read_dev(dc, st);
    if (hc.err) fail(ND_EHIP, "s-clique count failed (flags %u)", hc.err);
    if (timing) {
      count_kernel_ms = tm.between(5, 6);
      count_launches = 1;
    }
    const uint64_t sum = read_dev((uint64_t *)total, st);
    const uint64_t maxc = read_dev((uint64_t *)total + 1, st);
    const uint64_t per = binom_u64(s, r);
    // direct counting: every s-clique is counted once by each of its r-subsets
    n_s = p->fast ? sum / per : hc.n_s;
    if (p->fast && sum % per != 0) fail(ND_EHIP, "direct counts are inconsistent");
    if (sum != per * n_s) fail(ND_EOVERFLOW, "an s-clique count exceeds 32 bits");
    if (maxc + p->opt.debug_count_bias > 0xFFFFFFFFull)
      fail(ND_EOVERFLOW, "an s-clique count (%llu + bias %llu) exceeds 32 bits",
           (unsigned long long)maxc, (unsigned long long)p->opt.debug_count_bias);
    // outputs are staged for the canonical row order; the initial counts are
    // taken now, before the peel decrements them
    if (cnt_out) gather_counts(p->occ.get(), p->n_r, p->slots.get(), cnt_out, st);
    if (p->fast && r == 2) {  // (2,3): the listed adjacency starts as the graph's
      const uint64_t nnz = (uint64_t)p->g.nnz;
      if (p->fx.bm_words)
        hip_check(hipMemcpyAsync(p->fx.alive.get(), p->fx.bm.get(), 8 * p->fx.bm_words,
                                 hipMemcpyDeviceToDevice, st),
                  "copy bitmaps");
      if (p->fx.n_tri)
        hip_check(hipMemcpyAsync(p->fx.lvr.get(), p->fx.lval.get(), 4 * p->fx.n_tri,
                                 hipMemcpyDeviceToDevice, st),
                  "copy apex lists");
      if (nnz)
        hipLaunchKernelGGL(k_r2_init_arcs, dim3((unsigned)grid_for((int64_t)nnz, 256)),
                           dim3(256), 0, st, p->fx.lptr.get(), nnz, p->fx.llen.get(),
                           p->fx.arcst.get());
      if (p->g.n)
        hipLaunchKernelGGL(k_r2_init_vertices, dim3((unsigned)grid_for(p->g.n, 256)), dim3(256), 0,
                           st, p->g.rp.get(), p->g.n, p->fx.lost.get(), p->fx.deg_at.get());
    }
    if (p->fast && r == 3) {  // liveness bitmaps start as the adjacency bitmaps
      if (p->fx.bm_words)
        hip_check(hipMemcpyAsync(p->fx.alive.get(), p->fx.bm.get(), 8 * p->fx.bm_words,
                                 hipMemcpyDeviceToDevice, st),
                  "copy bitmaps");
      const uint64_t bw = p->fx.bm_words ? p->fx.bm_words : 1;
      const uint64_t aw = (p->fx.n_tri + 63) / 64 ? (p->fx.n_tri + 63) / 64 : 1;
      fill_u64(p->fx.alive_apex.get(), ~0ull, (int64_t)aw, st);  // every triangle alive
      fill_u64(p->fx.front.get(), 0, (int64_t)bw, st);            // no triangle in a frontier yet
      fill_u64(p->fx.front_apex.get(), 0, (int64_t)aw, st);
    }
    tm.mark(1, st);
  }  // fresh run
  // ---- bucket init + peel, driven by the device (the host polls the
  // round state every few rounds)
  PeelResult pr;
  DevBuf<uint32_t> kround;
  PeelState ps;
  ps.rc = p->rcb.get();
  ps.mirror = p->mirror;
  ps.ev = timing && p->ev_peel.ok && !p->ev_peel.ev.empty() ? p->ev_peel.ev.data() : nullptr;
  ps.queue_depth = p->opt.queue_depth ? p->opt.queue_depth : kPeelMaxDepth;
  // (2,3) graph contraction after every 2n peeled edges (Section 4.6)
  ps.contract_every = p->fast && r == 2 && p->opt.contract ? 2ull * (uint64_t)p->g.n : 0;
  // events recorded by graph nodes cannot be timed: timed runs launch plainly
  ps.graph_stream = timing ? nullptr : p->graph_stream;
  const uint32_t perr =
      peel_all(p->g, r, s, p->path, p->table(), p->fast ? &p->fx : nullptr, p->occ.get(), p->n_r,
               dc, p->stats.get(), ps, rec_cap, tcap, st, tm.at(2), &kround, &pr, &p->susp);
  if (perr & kErrCapacity) {
    if (p->susp.on && !resume) {  // keep what the next run needs besides the peel state
      p->susp_n_s = n_s;
      p->susp_counts = cnt_out != nullptr;
      p->susp_cnt.clear();
      if (cnt_out) {
        p->susp_cnt.resize(p->n_r);
        if (hipMemcpyAsync(p->susp_cnt.data(), cnt_out, 4 * p->n_r, hipMemcpyDeviceToHost, st) !=
                hipSuccess ||
            hipStreamSynchronize(st) != hipSuccess)
          p->susp.on = false;
      }
    }
    // the workspace was too small for one round: raise the requirement so
    // that nd_plan_sizes reports the size to run again with
    if (pr.need_rec > rec_cap)  // later rounds may need more: half again, at least double
      p->rec_need = std::max<uint64_t>(pr.need_rec + pr.need_rec / 2, 2 * rec_cap);
    if (pr.need_trace > tcap)  // rho is unknown: grow the trace 8-fold, to at least 4096
      p->trace_need = (uint32_t)std::min<uint64_t>(
          std::max<uint64_t>(std::max<uint64_t>(pr.need_trace, 8ull * tcap), 4096),
          std::max<uint64_t>(p->n_r, 1));
    fail(ND_ENOMEM,
         "a peel round needs %llu records (workspace holds %llu) or %llu round-trace entries "
         "(holds %u); run again with a workspace of %llu bytes",
         (unsigned long long)pr.need_rec, (unsigned long long)rec_cap,
         (unsigned long long)pr.need_trace, tcap, (unsigned long long)required_ws(p));
  }
  if (perr & kErrRuntime) fail(ND_EHIP, "HIP error in the peel loop: %s",
                               hipGetErrorString(hipGetLastError()));
  if (perr) fail(ND_EHIP, "peel failed (flags %u)", perr);
  if (!p->susp.lists.empty() || !p->susp_cnt.empty()) {  // a finished peel keeps nothing
    p->susp = PeelSuspend();
    std::vector<uint32_t>().swap(p->susp_cnt);
    p->susp_counts = false;
  }
  p->round_sizes = pr.sizes;
  p->round_k = pr.levels;
  p->k_advances = pr.advances;
  if (timing) {
    peel_kernel_ms = pr.apply_ms;
    peel_launches = pr.apply_launches;
  }
  tm.mark(3, st);
  // ---- emit (staged for the canonical row order)
  stats_collect(p->stats.get(), dc, st);
  emit(r, p->occ.get(), p->n_r, p->table(), p->g.new2old.get(), kround.get(),
       (uint32_t)p->round_k.size(), rows_out, kap_out, st);
  if (canon) {
    // rows in lexicographic order of their vertices: radix sort of packed
    // keys (two keys, low part first, when r vertices need more than 64 bits)
    const uint64_t n_r = p->n_r;
    const int b = p->bits;
    DevBuf<uint64_t> keys(n_r);
    DevBuf<uint32_t> idx(n_r);
    iota_u32(idx.get(), (int64_t)n_r, st);
    const dim3 g((unsigned)grid_for((int64_t)n_r, 256)), blk(256);
    if (r * b <= 64) {
      hipLaunchKernelGGL(k_row_keys, g, blk, 0, st, rows_tmp.get(), r, n_r, idx.get(), 0, r, b,
                         keys.get());
      radix_sort(keys.get(), idx.get(), (int64_t)n_r, r * b, st);
    } else {
      const int h = (r + 1) / 2;
      hipLaunchKernelGGL(k_row_keys, g, blk, 0, st, rows_tmp.get(), r, n_r, idx.get(), h, r, b,
                         keys.get());
      radix_sort(keys.get(), idx.get(), (int64_t)n_r, (r - h) * b, st);
      hipLaunchKernelGGL(k_row_keys, g, blk, 0, st, rows_tmp.get(), r, n_r, idx.get(), 0, h, b,
                         keys.get());
      radix_sort(keys.get(), idx.get(), (int64_t)n_r, h * b, st);
    }
    hipLaunchKernelGGL(k_permute_rows, g, blk, 0, st, rows_tmp.get(), kap_tmp.get(),
                       cnt_tmp.get(), r, n_r, idx.get(), rcl_dev, kappa_dev,
                       counts_dev ? counts_dev : nullptr);
  }
  tm.mark(4, st);
  hc = read_dev(dc, st);
  hip_check(hipGetLastError(), "kernel launch");
  if (hc.err) fail(ND_EHIP, "peel failed (flags %u)", hc.err);
  p->traced = true;
  if (stats) {
    memset(stats, 0, sizeof(*stats));
    stats->n_r = p->n_r;
    stats->n_s = n_s;
    stats->rounds = p->round_sizes.size();
    stats->k_advances = p->k_advances;
    stats->decrements = hc.decrements;
    stats->discoveries = hc.discoveries;
    stats->atomics = hc.atomics;
    stats->table_slots = p->n_slots;
    stats->max_kappa = p->round_k.empty() ? 0 : p->round_k.back();
    stats->max_out_degree = p->g.max_out;
    stats->ms[0] = p->ms_create[0];
    stats->ms[1] = p->ms_create[1];
    stats->ms[2] = p->ms_create[2];
    stats->ms[3] = tm.between(0, 1);
    stats->ms[4] = tm.between(1, 2);
    stats->ms[5] = tm.between(2, 3);
    stats->ms[6] = tm.between(3, 4);
    stats->ms[7] = p->ms_create[0] + p->ms_create[1] + p->ms_create[2] + tm.between(0, 4);
    stats->count_kernel_ms = count_kernel_ms;
    stats->peel_kernel_ms = peel_kernel_ms;
    stats->count_launches = count_launches;
    stats->peel_launches = peel_launches;
    stats->workspace_bytes = g_ws->used;
    stats->max_round_records = pr.max_rec;
    stats->max_round_arcs = pr.max_arcs;
    stats->contractions = pr.contractions;
    stats->key_words = p->wide ? 2 : 1;
  }
}

}  // namespace

extern "C" {

nd_status nd_run(nd_plan p, void *workspace_dev, uint64_t workspace_bytes, int32_t *rcl_dev,
                 uint32_t *kappa_dev, uint32_t *counts_dev, nd_stats *stats) {
  if (!p) {
    g_last_error = "plan is null";
    return ND_EINVAL;
  }
  if (p->n_r && (!rcl_dev || !kappa_dev)) {
    g_last_error = "output pointer is null";
    return ND_EINVAL;
  }
  const uint64_t need = required_ws(p);
  if (workspace_bytes < need || (need && !workspace_dev)) {
    char buf[200];
    snprintf(buf, sizeof(buf), "workspace of %llu bytes given, the run needs %llu",
             (unsigned long long)workspace_bytes, (unsigned long long)need);
    g_last_error = buf;
    return ND_ENOMEM;
  }
  if (((uintptr_t)workspace_dev & (kWsAlign - 1)) != 0) {
    g_last_error = "workspace must be 256-byte aligned";
    return ND_EINVAL;
  }
  if (p->budget && p->held + workspace_bytes > p->budget) {
    char buf[200];
    snprintf(buf, sizeof(buf), "plan %llu bytes + workspace %llu bytes exceed the budget %llu",
             (unsigned long long)p->held, (unsigned long long)workspace_bytes,
             (unsigned long long)p->budget);
    g_last_error = buf;
    return ND_ENOMEM;
  }
  return guarded(p->st, [&] {
    WorkspaceScope ws(workspace_dev, workspace_bytes);
    run_impl(p, rcl_dev, kappa_dev, counts_dev, stats);
  });
}

}  // extern "C"

// Workspace of nd_run_noalloc: one static device array, which every GPU the
// library runs on holds from load until the process ends.  In host code its
// name is only a stand-in; kernels get the device address that
// hipGetSymbolAddress returns for the current device, looked up once per
// device at that device's first nd_run_noalloc call.
static __device__ __align__(256) unsigned char scratch[ND_NOALLOC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// device address of `scratch` on the current device
void *scratch_on_device(int dev) {
  if (dev < 0 || dev >= kMaxDevices) fail(ND_EINVAL, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr) {
      hipGetLastError();
      fail(ND_EHIP, "hipGetSymbolAddress of the static workspace failed: %s",
           hipGetErrorString(e));
    }
    g_scratch_ptr[dev] = ptr;
  }
  return g_scratch_ptr[dev];
}

}  // namespace

extern "C" {

nd_status nd_run_noalloc(nd_plan p, int32_t *rcl_dev, uint32_t *kappa_dev, uint32_t *counts_dev,
                         nd_stats *stats) {
  if (!p) {
    g_last_error = "plan is null";
    return ND_EINVAL;
  }
  if (p->n_r && (!rcl_dev || !kappa_dev)) {
    g_last_error = "output pointer is null";
    return ND_EINVAL;
  }
  const uint64_t need = required_ws(p);
  if (need > ND_NOALLOC_WORKSPACE_BYTES) {
    char buf[200];
    snprintf(buf, sizeof(buf),
             "the run needs a workspace of %llu bytes; the static workspace holds %llu",
             (unsigned long long)need, (unsigned long long)ND_NOALLOC_WORKSPACE_BYTES);
    g_last_error = buf;
    return ND_ENOMEM;
  }
  if (p->budget && p->held + need > p->budget) {
    g_last_error = "plan and workspace exceed the budget";
    return ND_ENOMEM;
  }
  return guarded(p->st, [&] {
    int dev = -1;
    hip_check(hipGetDevice(&dev), "get device");
    if (dev != p->device) fail(ND_EINVAL, "call on the plan's device (%d, current %d)", p->device, dev);
    void *ws = scratch_on_device(dev);
    WorkspaceScope scope(ws, ND_NOALLOC_WORKSPACE_BYTES);
    run_impl(p, rcl_dev, kappa_dev, counts_dev, stats);
  });
}

nd_status nd_round_trace(nd_plan p, uint64_t *sizes_host, uint32_t *levels_host, uint64_t cap,
                         uint64_t *rounds) {
  if (!p) {
    g_last_error = "plan is null";
    return ND_EINVAL;
  }
  if (!p->traced) {
    g_last_error = "no successful nd_run on this plan";
    return ND_ESTATE;
  }
  uint64_t n = p->round_sizes.size();
  if (rounds) *rounds = n;
  uint64_t m = n < cap ? n : cap;
  for (uint64_t i = 0; i < m; i++) {
    if (sizes_host) sizes_host[i] = p->round_sizes[i];
    if (levels_host) levels_host[i] = p->round_k[i];
  }
  return ND_OK;
}

nd_status nd_plan_destroy(nd_plan p) {
  if (!p) return ND_OK;
  hipStream_t st = p->st;
  StreamScope scope(st);
  delete p;
  hipStreamSynchronize(st);
  return ND_OK;
}

struct nd_batch_s {
  hipStream_t st = nullptr;
  int r = 0, s = 0;
  int32_t count = 0, n_total = 0;
  int64_t nnz_total = 0;
  DevBuf<int64_t> rp;
  DevBuf<int32_t> col, vo;
  nd_plan plan = nullptr;
  uint64_t n_r = 0;
};

}  // extern "C"

namespace {

// bytes a batch run carves before the union plan's run: staged outputs,
// per-graph row counts and cursors, row graph ids
uint64_t batch_extra_ws(const nd_batch_s *b) {
  const uint64_t n1 = b->n_r ? b->n_r : 1;
  return ws_buf<int32_t>(b->n_r ? b->n_r * (uint64_t)b->r : 1) + 2 * ws_buf<uint32_t>(n1) +
         2 * ws_buf<unsigned long long>((uint64_t)b->count + 1) + ws_buf<int32_t>(n1);
}

}  // namespace

extern "C" {

nd_status nd_batch_create(const nd_csr *graphs, int32_t count, int r, int s,
                          const nd_options *opt, uint64_t hbm_budget_bytes, void *hip_stream,
                          nd_batch *out) {
  if (!out || (count > 0 && !graphs) || count < 0) {
    g_last_error = "bad batch arguments";
    return ND_EINVAL;
  }
  *out = nullptr;
  hipStream_t st = (hipStream_t)hip_stream;
  nd_batch b = new (std::nothrow) nd_batch_s();
  if (!b) return ND_ENOMEM;
  nd_status rc = guarded(st, [&] {
    b->st = st;
    b->r = r;
    b->s = s;
    b->count = count;
    std::vector<GraphDesc> gd((size_t)(count > 0 ? count : 1));
    std::vector<int32_t> vo((size_t)count + 1);
    std::vector<int64_t> eo((size_t)count + 1);
    int64_t nv = 0, ne = 0;
    for (int32_t g = 0; g < count; g++) {
      const nd_csr &c = graphs[g];
      if (c.n < 0 || c.nnz < 0 || (c.n > 0 && !c.row_ptr) || (c.nnz > 0 && !c.col))
        fail(ND_EINVAL, "graph %d has a bad CSR header", g);
      vo[g] = (int32_t)nv;
      eo[g] = ne;
      gd[g] = GraphDesc{c.row_ptr, c.col, c.n, (int32_t)nv, c.nnz, ne};
      nv += c.n;
      ne += c.nnz;
      if (nv > INT32_MAX - 1) fail(ND_EOVERFLOW, "the batch has more than 2^31 vertices");
    }
    vo[count] = (int32_t)nv;
    eo[count] = ne;
    b->n_total = (int32_t)nv;
    b->nnz_total = ne;
    b->rp.reset((size_t)nv + 1);
    b->col.reset(ne > 0 ? (size_t)ne : 1);
    b->vo.reset((size_t)count + 1);
    DevBuf<GraphDesc> gdd(gd.size());
    DevBuf<int64_t> eod((size_t)count + 1);
    DevBuf<uint32_t> err(1);
    fill_u32(err.get(), 0, 1, st);
    hip_check(hipMemcpyAsync(gdd.get(), gd.data(), sizeof(GraphDesc) * gd.size(),
                             hipMemcpyHostToDevice, st), "copy descriptors");
    hip_check(hipMemcpyAsync(b->vo.get(), vo.data(), 4 * vo.size(), hipMemcpyHostToDevice, st),
              "copy offsets");
    hip_check(hipMemcpyAsync(eod.get(), eo.data(), 8 * eo.size(), hipMemcpyHostToDevice, st),
              "copy offsets");
    if (count > 0) {
      hipLaunchKernelGGL(k_union_rows, dim3((unsigned)grid_for(nv + 1, 256)), dim3(256), 0, st,
                         gdd.get(), b->vo.get(), (int)count, (int32_t)nv, ne, b->rp.get());
      if (ne > 0)
        hipLaunchKernelGGL(k_union_cols, dim3((unsigned)grid_for(ne, 256)), dim3(256), 0, st,
                           gdd.get(), eod.get(), (int)count, ne, b->col.get(), err.get());
    } else {
      fill_u64((uint64_t *)b->rp.get(), 0, 1, st);
    }
    if (read_dev(err.get(), st)) fail(ND_EGRAPH, "a batch graph has a vertex id out of range");
    nd_csr u{(int32_t)nv, ne, b->rp.get(), b->col.get()};
    nd_status prc = nd_plan_create(&u, r, s, opt, hbm_budget_bytes, hip_stream, &b->plan);
    if (prc != ND_OK) throw Failure{prc};
    b->n_r = b->plan->n_r;
  });
  if (rc != ND_OK) {
    nd_batch_destroy(b);
    return rc;
  }
  *out = b;
  return ND_OK;
}

nd_status nd_batch_sizes(nd_batch b, uint64_t *n_r_total, int32_t *count,
                         uint64_t *workspace_bytes) {
  if (!b) {
    g_last_error = "batch is null";
    return ND_EINVAL;
  }
  if (n_r_total) *n_r_total = b->n_r;
  if (count) *count = b->count;
  if (workspace_bytes) *workspace_bytes = batch_extra_ws(b) + required_ws(b->plan);
  return ND_OK;
}

nd_status nd_batch_run(nd_batch b, void *workspace_dev, uint64_t workspace_bytes,
                       int32_t *rcliques_dev, uint32_t *kappa_dev, uint32_t *counts_dev,
                       uint64_t *row_offsets_host, nd_stats *stats) {
  if (!b || !row_offsets_host) {
    g_last_error = "batch or row_offsets is null";
    return ND_EINVAL;
  }
  if (b->n_r && (!rcliques_dev || !kappa_dev)) {
    g_last_error = "output pointer is null";
    return ND_EINVAL;
  }
  const uint64_t need = batch_extra_ws(b) + required_ws(b->plan);
  if (workspace_bytes < need || !workspace_dev) {
    char buf[200];
    snprintf(buf, sizeof(buf), "workspace of %llu bytes given, the batch run needs %llu",
             (unsigned long long)workspace_bytes, (unsigned long long)need);
    g_last_error = buf;
    return ND_ENOMEM;
  }
  if (((uintptr_t)workspace_dev & (kWsAlign - 1)) != 0) {
    g_last_error = "workspace must be 256-byte aligned";
    return ND_EINVAL;
  }
  nd_plan p = b->plan;
  if (p->budget && p->held + workspace_bytes > p->budget) {
    g_last_error = "plan and workspace exceed the budget";
    return ND_ENOMEM;
  }
  hipStream_t st = b->st;
  return guarded(st, [&] {
    WorkspaceScope ws(workspace_dev, workspace_bytes);
    const int r = b->r;
    const uint64_t n_r = b->n_r;
    const int count = b->count;
    DevBuf<int32_t> rcl(n_r ? n_r * r : 1);
    DevBuf<uint32_t> kap(n_r ? n_r : 1), cnt(n_r ? n_r : 1);
    DevBuf<unsigned long long> per((size_t)count + 1), cur((size_t)count + 1);
    DevBuf<int32_t> gid(n_r ? n_r : 1);
    run_impl(p, rcl.get(), kap.get(), counts_dev ? cnt.get() : nullptr, stats);
    fill_u64((uint64_t *)per.get(), 0, count + 1, st);
    fill_u64((uint64_t *)cur.get(), 0, count + 1, st);
    if (n_r && count > 0)
      hipLaunchKernelGGL(k_row_graph, dim3((unsigned)grid_for(n_r, 256)), dim3(256), 0, st,
                         rcl.get(), r, n_r, b->vo.get(), count, gid.get(), per.get());
    // row offsets: prefix sum of the per-graph row counts (count + 1 values)
    std::vector<uint64_t> off((size_t)count + 1);
    hip_check(hipMemcpyAsync(off.data(), per.get(), 8 * off.size(), hipMemcpyDeviceToHost, st),
              "copy row counts");
    hip_check(hipStreamSynchronize(st), "synchronize");
    uint64_t acc = 0;
    for (auto &x : off) {
      const uint64_t c = x;
      x = acc;
      acc += c;
    }
    hip_check(hipMemcpyAsync(per.get(), off.data(), 8 * off.size(), hipMemcpyHostToDevice, st),
              "copy row offsets");
    if (n_r && count > 0) {
      if (p->opt.canonical)  // rows sorted by union ids are grouped by graph already
        hipLaunchKernelGGL(k_localise, dim3((unsigned)grid_for(n_r, 256)), dim3(256), 0, st,
                           rcl.get(), kap.get(), cnt.get(), r, n_r, gid.get(), b->vo.get(),
                           rcliques_dev, kappa_dev, counts_dev ? counts_dev : nullptr);
      else
        hipLaunchKernelGGL(k_regroup, dim3((unsigned)grid_for(n_r, 256)), dim3(256), 0, st,
                           rcl.get(), kap.get(), cnt.get(), r, n_r, gid.get(), b->vo.get(),
                           per.get(), cur.get(), rcliques_dev, kappa_dev,
                           counts_dev ? counts_dev : nullptr);
    }
    hip_check(hipStreamSynchronize(st), "synchronize");
    hip_check(hipGetLastError(), "kernel launch");
    memcpy(row_offsets_host, off.data(), 8 * off.size());
  });
}

nd_status nd_batch_round_trace(nd_batch b, uint64_t *sizes_host, uint32_t *levels_host,
                               uint64_t cap, uint64_t *rounds) {
  if (!b || !b->plan) {
    g_last_error = "batch is null";
    return ND_EINVAL;
  }
  return nd_round_trace(b->plan, sizes_host, levels_host, cap, rounds);
}

nd_status nd_batch_destroy(nd_batch b) {
  if (!b) return ND_OK;
  hipStream_t st = b->st;
  if (b->plan) nd_plan_destroy(b->plan);
  {
    StreamScope scope(st);
    delete b;
  }
  hipStreamSynchronize(st);
  return ND_OK;
}

nd_status nd_batch_autotune(const nd_csr *graphs, int32_t count, int r, int s,
                            const nd_options *base, int32_t sample_count, void *hip_stream,
                            nd_options *best, nd_tune_report *report) {
  if (!best || (count > 0 && !graphs) || count < 0 || sample_count < 1) {
    g_last_error = "bad autotune arguments";
    return ND_EINVAL;
  }
  hipStream_t st = (hipStream_t)hip_stream;
  return guarded(st, [&] {
    // held-out sample: graphs spread evenly over the input
    const int32_t m = std::min(count, sample_count);
    std::vector<nd_csr> sample((size_t)std::max(m, 1));
    for (int32_t k = 0; k < m; k++) sample[k] = graphs[(int64_t)k * count / m];
    nd_options b0{};
    if (base) b0 = *base;
    b0.timing = 0;
    std::vector<nd_options> cand;
    for (int orient = 0; orient < 2; orient++)
      for (int depth : {8, 32})
        for (int graph = 0; graph < 2; graph++) {
          nd_options o = b0;
          o.orient = orient;
          o.queue_depth = depth;
          o.graph_rounds = graph;
          cand.push_back(o);
        }
    std::vector<float> ms(cand.size(), 0.f);
    auto one = [&](const nd_options &o) -> double {
      nd_batch b = nullptr;
      const auto t0 = std::chrono::steady_clock::now();
      nd_status rc = nd_batch_create(sample.data(), m, r, s, &o, 0, hip_stream, &b);
      if (rc != ND_OK) throw Failure{rc};
      uint64_t n_r = 0, wsb = 0;
      int32_t cnt = 0;
      nd_batch_sizes(b, &n_r, &cnt, &wsb);
      DevBuf<unsigned char> ws(wsb + kWsAlign);
      DevBuf<int32_t> rcl(n_r ? n_r * (uint64_t)r : 1);
      DevBuf<uint32_t> kap(n_r ? n_r : 1);
      std::vector<uint64_t> off((size_t)cnt + 1);
      char *wp = (char *)ws.get();
      wp += (kWsAlign - ((uintptr_t)wp & (kWsAlign - 1))) & (kWsAlign - 1);
      rc = nd_batch_run(b, wp, wsb, rcl.get(), kap.get(), nullptr, off.data(), nullptr);
      const auto t1 = std::chrono::steady_clock::now();
      nd_batch_destroy(b);
      if (rc != ND_OK) throw Failure{rc};
      return std::chrono::duration<double, std::milli>(t1 - t0).count();
    };
    one(cand[0]);  // warm-up: code objects, pool
    size_t bi = 0;
    for (size_t i = 0; i < cand.size(); i++) {
      ms[i] = (float)std::min(one(cand[i]), one(cand[i]));
      if (ms[i] < ms[bi]) bi = i;
    }
    *best = cand[bi];
    if (base) best->timing = base->timing;
    if (report) {
      memset(report, 0, sizeof(*report));
      report->candidates = (int32_t)std::min<size_t>(cand.size(), ND_TUNE_MAX);
      report->best = (int32_t)bi;
      report->sample_graphs = m;
      for (int32_t i = 0; i < report->candidates; i++) {
        report->opt[i] = cand[i];
        report->ms[i] = ms[i];
      }
    }
  });
}

nd_status nd_release_cached(void) {
  return guarded(nullptr, [&] {
    hip_check(hipDeviceSynchronize(), "synchronize");
    int dev = 0;
    hip_check(hipGetDevice(&dev), "get device");
    hipMemPool_t pool;
    hip_check(hipDeviceGetDefaultMemPool(&pool, dev), "get pool");
    hip_check(hipMemPoolTrimTo(pool, 0), "trim pool");
  });
}

}  // extern "C"
