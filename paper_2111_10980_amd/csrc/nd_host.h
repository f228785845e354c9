// Host-side launch interfaces shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include <vector>

#include "nd_internal.h"

namespace nd {

// Device memory from the library's caching pool (never hipMalloc directly),
// or, while a workspace is active on the calling thread, carved from it.
void *dev_alloc(size_t bytes);
void dev_free(void *p);

// Caller-owned device workspace.  While a WorkspaceScope is alive on a
// thread, every dev_alloc of that thread takes the next 256-byte aligned
// block of the workspace (blocks are never reused within the scope and
// dev_free of a block does nothing); a request past the end fails with
// ND_ENOMEM.  The workspace a run needs is therefore the sum of ws_block()
// over every buffer it allocates, which the sizing functions below add up.
constexpr uint64_t kWsAlign = 256;
inline uint64_t ws_block(uint64_t bytes) {
  if (bytes == 0) bytes = 16;
  return (bytes + kWsAlign - 1) & ~(kWsAlign - 1);
}
// bytes one DevBuf<T>(count) takes from a workspace (none for count 0)
template <class T>
inline uint64_t ws_buf(uint64_t count) {
  return count ? ws_block(count * sizeof(T)) : 0;
}
struct Workspace {
  char *base = nullptr;
  uint64_t size = 0, used = 0;
};
struct WorkspaceScope {
  Workspace ws;
  Workspace *prev;
  WorkspaceScope(void *base, uint64_t size);
  ~WorkspaceScope();
  WorkspaceScope(const WorkspaceScope &) = delete;
  WorkspaceScope &operator=(const WorkspaceScope &) = delete;
};

// Scratch buffer that returns to the pool when it goes out of scope.
template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  DevBuf() = default;
  explicit DevBuf(size_t count) { reset(count); }
  DevBuf(const DevBuf &) = delete;
  DevBuf &operator=(const DevBuf &) = delete;
  DevBuf(DevBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
  DevBuf &operator=(DevBuf &&o) noexcept {
    if (this != &o) {
      release();
      p = o.p; n = o.n; o.p = nullptr; o.n = 0;
    }
    return *this;
  }
  ~DevBuf() { release(); }
  void reset(size_t count) {
    release();
    n = count;
    p = count ? (T *)dev_alloc(count * sizeof(T)) : nullptr;
  }
  void release() {
    if (p) dev_free(p);
    p = nullptr;
    n = 0;
  }
  T *get() const { return p; }
};

struct OutOfMemory {};

// Raises the library's error (ND_ENOMEM for out-of-memory, else ND_EHIP,
// with `what` and HIP's message) when e is not hipSuccess.
void hip_ok(hipError_t e, const char *what);
// Copies bytes from device memory to the host on stream st and waits for
// the copy; a failed copy or wait raises the library's error instead of
// leaving dst uninitialised.
void read_back(void *dst, const void *src, size_t bytes, hipStream_t st);

// ---- primitives (nd_prims.hip)
void fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t st);
void fill_u64(uint64_t *p, uint64_t v, int64_t n, hipStream_t st);
void fill_slots(Slot *p, int64_t n, hipStream_t st);
void iota_u32(uint32_t *p, int64_t n, hipStream_t st);
void widen_u32_to_u64(const uint32_t *a, uint64_t *b, int64_t n, hipStream_t st);
// exclusive prefix sum, in place allowed; n elements
void scan_exclusive_u64(const uint64_t *in, uint64_t *out, int64_t n, hipStream_t st);
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int64_t n, hipStream_t st);
// stable LSD radix sort of keys by bits [lo_bit, bits), optional values
void radix_sort(uint64_t *keys, uint32_t *vals, int64_t n, int bits, hipStream_t st,
                int lo_bit = 0);
// sum of a u32 array into *out (device u64, accumulated)
void sum_u32(const uint32_t *p, int64_t n, uint64_t *out, hipStream_t st);
uint32_t max_u32_host(const uint32_t *p, int64_t n, hipStream_t st);
// workspace bytes one call allocates
uint64_t scan_ws_bytes(int64_t n, size_t elem);
uint64_t radix_sort_ws_bytes(int64_t n, int bits, int lo_bit, bool vals);

// ---- graph (nd_graph.hip)
struct OrientedGraph {
  int32_t n = 0;
  int64_t nnz = 0;
  DevBuf<int64_t> rp, up;
  DevBuf<int32_t> col;
  DevBuf<int32_t> new2old;  // rank -> original id
  uint32_t max_out = 0;
  GraphView view() const { return GraphView{n, rp.get(), col.get(), up.get()}; }
};
// returns 0 or kErrGraph
uint32_t validate_csr(int32_t n, int64_t nnz, const int64_t *rp, const int32_t *col,
                      Counters *dctr, hipStream_t st);
void orient_relabel(int32_t n, int64_t nnz, const int64_t *rp, const int32_t *col, int mode,
                    OrientedGraph *og, hipStream_t st);

// ---- cliques (nd_clique.hip)
// count the r-cliques rooted at each vertex (lowest rank), into cnt[n]
void count_rcliques(const OrientedGraph &g, int r, uint32_t *cnt, hipStream_t st);
// r >= 4: r-cliques per out-arc (v1, v2), indexed by arc position (nnz + 1 entries)
void count_rcliques_arcs(const OrientedGraph &g, int r, uint32_t *cnt, hipStream_t st);
void insert_rcliques(const OrientedGraph &g, int r, const TableView &T, Counters *dctr,
                     hipStream_t st);
// ev0/ev1 (nullable) are recorded around the listing kernels only
void count_scliques(const OrientedGraph &g, int r, int s, const TableView &T, Counters *dctr,
                    unsigned long long *stats, hipStream_t st, hipEvent_t ev0 = nullptr,
                    hipEvent_t ev1 = nullptr);
// workspace bytes count_scliques allocates
uint64_t count_scliques_ws_bytes(const OrientedGraph &g);
// sum the statistic lines into dctr->decrements, discoveries, n_s (adds)
void stats_collect(unsigned long long *stats, Counters *dctr, hipStream_t st);

// every triangle (x<y<z) writes key (arc(y,z) << xbits | x) at cursor[x]++
void list_apex_keys(const OrientedGraph &g, uint64_t *cursor, uint64_t *keys, int xbits,
                    Counters *dctr, hipStream_t st);

// ---- s = r+1 path (nd_fast.hip): per-root adjacency bitmaps and apex lists
struct FastView {
  const uint64_t *__restrict__ bm_off;  // n: word offset of root v's bitmap rows
  const uint64_t *__restrict__ bm;      // symmetric rows, d x ceil(d/64) words per root
  const uint64_t *__restrict__ lptr;    // nnz+1: apex list of the arc at col position e
  const int32_t *__restrict__ lval;     // apex vertices, ascending within a list
  uint64_t *alive;                      // r = 3: bitmap copy, a triangle's bits cleared
                                        // after the round that peels it (else null)
  uint64_t *alive_apex;                 // r = 3: one bit per apex-list entry (= per
                                        // triangle), cleared with the triangle (else null)
  uint64_t *front;                      // r = 3: bitmap layout, bits of the triangles
                                        // of the current frontier (else null)
  uint64_t *front_apex;                 // r = 3: apex-entry bits of the same (else null)
  const uint32_t *__restrict__ rowpre;  // r = 3 ranked table: per out-arc (v, N+(v)[i]) the
                                        // triangles of v's bitmap rows before i (else null)
  // r = 2 (the (2,3) peel), else null: the run's copy of the apex lists,
  // compacted by graph contraction, with each list's live length; one state
  // byte per arc position (alive / in the frontier / peeled); per vertex the
  // incident edges peeled since its last contraction and its degree then
  int32_t *lvr;
  uint32_t *llen;
  uint8_t *arcst;
  uint32_t *lost;
  uint32_t *deg_at;
};
struct FastIndex {
  DevBuf<uint64_t> bm_off, bm, lptr, alive, alive_apex, front, front_apex;
  DevBuf<uint32_t> rowpre;
  DevBuf<int32_t> lvr;                    // r = 2 run state (see FastView)
  DevBuf<uint32_t> llen, lost, deg_at;
  DevBuf<uint8_t> arcst;
  DevBuf<uint64_t> loc;  // per slot: local indices of v2..vr in N+(v1), 9 bits each
  DevBuf<int32_t> lval;
  uint64_t bm_words = 0, n_tri = 0;
  FastView view() const {
    return FastView{bm_off.get(),  bm.get(),         lptr.get(),  lval.get(),
                    alive.get(),   alive_apex.get(), front.get(), front_apex.get(),
                    rowpre.n ? rowpre.get() : nullptr,
                    lvr.get(),     llen.get(),       arcst.get(), lost.get(),
                    deg_at.get()};
  }
};
// tri_per_root (nullable, n entries) receives the triangles rooted at each
// vertex, which the apex lists are laid out by
void build_fast_index(const OrientedGraph &g, FastIndex *fx, Counters *dctr, hipStream_t st,
                      uint32_t *tri_per_root = nullptr);
// r = 3 ranked table.  A triangle (v, a, b) whose root v keeps a bitmap sits
// at seg[v] + its rank among the bits of v's bitmap above the diagonal
// (row-major), so the triangles of one bitmap row are contiguous; roots
// without a bitmap keep a hashed segment.  ranked_caps writes the segment
// capacities (before the prefix sum) and fills fx->rowpre; ranked_insert
// writes the keys of the bitmap roots' triangles.
void ranked_caps(const OrientedGraph &g, FastIndex *fx, const uint32_t *tri_per_root, float lf,
                 uint64_t *cap, hipStream_t st);
void ranked_insert(const OrientedGraph &g, const FastIndex &fx, const TableView &T,
                   hipStream_t st);
// r = 3: insert the triangles of the roots without a bitmap (> 512 out-neighbours)
void insert_rcliques_heavy3(const OrientedGraph &g, const TableView &T, Counters *dctr,
                            hipStream_t st);
// count(R) = |common neighbourhood of R| written straight into each slot
void count_direct(const OrientedGraph &g, int r, const TableView &T, const FastIndex &fx,
                  const uint32_t *occ, uint64_t n_r, Counters *dctr, hipStream_t st);
void build_slot_loc(const OrientedGraph &g, int r, const TableView &T, uint64_t n_slots,
                    FastIndex *fx, hipStream_t st);
// ---- peel loop (nd_peel.hip)
struct PeelResult {
  std::vector<uint64_t> sizes;   // |A_t| per round
  std::vector<uint32_t> levels;  // k per round
  uint32_t advances = 0;         // level advances
  float apply_ms = 0;            // update-pass kernel time (timing only)
  uint32_t apply_launches = 0;
  uint64_t need_rec = 0;         // kErrCapacity: record capacity the halted round needs
  uint64_t need_trace = 0;       // kErrCapacity: round-trace capacity needed
  uint64_t max_rec = 0, max_arcs = 0;  // largest per-round record / out-arc totals
  uint32_t contractions = 0;           // r = 2: graph contraction passes
};
constexpr int kPeelMaxDepth = 32;      // rounds queued between two reads of the state
constexpr uint64_t kArcsPerRecord = 4; // s >= r+2: out-arc capacity per record slot
// Plan-owned state of the peel loop (no device allocation happens in a
// run): the device round control block, its pinned host mirror, with timing
// 2 * kPeelMaxDepth events (else null), the queue depth and, for graph
// replay of queued rounds, the capture stream.
struct PeelState {
  uint64_t contract_every = 0;           // r = 2: contract after this many peeled edges (0 = never)
  RoundCtl *rc = nullptr;
  RoundCtl *mirror = nullptr;
  hipEvent_t *ev = nullptr;
  int queue_depth = kPeelMaxDepth;       // most rounds queued between two state reads
  hipStream_t graph_stream = nullptr;    // non-null: queued rounds replayed from captured
                                         // graphs, captured on this (plan-owned) stream
};
// Workspace bytes peel_all allocates with the given capacities.
uint64_t peel_ws_bytes(int r, int path, uint64_t n_r, uint64_t nnz, uint64_t rec_cap,
                       uint32_t trace_cap);
// The peel's state between rounds that lives in the workspace (bucket
// lists, round trace, r = 2 edge states), kept in host memory when a round
// outgrew the workspace, together with the round control block as it
// stopped.  Everything else the peel carries from round to round is
// plan-owned (slot counts and stamps, liveness bits, statistics), so a run
// with a larger workspace continues at the round that stopped.
struct PeelSuspend {
  bool on = false;
  RoundCtl rc{};
  std::vector<uint32_t> lists;       // the live lists: frontier, window, high (nF + nW + nH)
  std::vector<uint32_t> tsize, tk;   // the rounds done
  std::vector<uint8_t> dead;         // s >= r+2, r = 2: per-arc edge states
};

// Whole bucketed peel (Algorithm 2 after the count) on the device.  path: 0
// the one-wave walker, 1 the s = r+1 expand/apply passes (needs fx), 2 the
// flattened s >= r+2 passes.  rec_cap records (and kArcsPerRecord * rec_cap
// out-arcs) per round and trace_cap rounds; a round that needs more stops the
// peel with kErrCapacity and the capacity it needs in res.  With sus, a round
// that outgrew the records or out-arcs leaves the state in *sus, and a call
// with sus->on continues from it instead of starting the peel.  kround
// receives the level of every round (for emit).  Returns 0 or kErr* bits.
uint32_t peel_all(const OrientedGraph &g, int r, int s, int path, const TableView &T,
                  const FastIndex *fx, const uint32_t *occ, uint64_t n_r, Counters *dc,
                  unsigned long long *stats, const PeelState &ps, uint64_t rec_cap,
                  uint32_t trace_cap, hipStream_t st, hipEvent_t ev_first,
                  DevBuf<uint32_t> *kround, PeelResult *res, PeelSuspend *sus);
void occupied_list(const Slot *slots, uint64_t n_slots, uint32_t *occ, hipStream_t st);
void gather_counts(const uint32_t *occ, uint64_t n_r, const Slot *slots, uint32_t *out,
                   hipStream_t st);
void emit(int r, const uint32_t *occ, uint64_t n_r, const TableView &T, const int32_t *new2old,
          const uint32_t *kround, uint32_t nrounds, int32_t *rcl_out, uint32_t *kappa_out,
          hipStream_t st);

}  // namespace nd
