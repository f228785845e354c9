// Serving loop: continuous batching of (graph, r, s) decomposition jobs.
//
// A fixed pool of worker threads, each with its own HIP stream, takes jobs
// from one FIFO queue.  Admission is by the device-memory budget, in two
// steps.  A job at the head of the queue starts its plan when a worker is
// idle and its estimate fits what is left of the budget.  The estimate is
// computed from the graph's size, scaled by the largest ratio of exact to
// estimated bytes seen so far for its (r, s).  Once the plan exists, the job
// holds exactly its plan's bytes, its run's workspace and its outputs
// (nd_plan_sizes).  When that exact figure does not fit, the job destroys
// its plan and waits at the head of the queue for the exact figure.  A job
// larger than the whole budget runs alone.  An admitted job keeps its plan
// (oriented graph, r-clique table, bucket state) on the device until its
// last round.  The rounds of the jobs in flight interleave on the GPU
// through their streams.  A job that arrives while others run starts as
// soon as a slot and memory are free, instead of waiting for the GPU to
// drain.  Results stay on the device until the caller releases them, and
// their bytes count against the budget until then.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/nd.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
  uint64_t id = 0;
  nd_csr g{};
  int r = 0, s = 0;
  nd_options opt{};
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit
  uint64_t est_raw = 0;        // size-only estimate
  uint64_t exact = 0;          // plan + workspace + outputs, once known
  uint64_t held = 0;           // bytes counted against the budget right now
  uint64_t out_bytes = 0;      // outputs, counted until release
  nd_status st = ND_OK;
  std::string err;
  bool done = false;
  uint64_t n_r = 0;
  int32_t *rcl = nullptr;
  uint32_t *kappa = nullptr;
  hipStream_t stream = nullptr;  // stream its outputs were allocated on
  nd_stats stats{};
  uint32_t requeues = 0;
  Clock::time_point t_submit, t_start, t_end;
};

// Device bytes a job may hold at its peak, from its size alone: the relabeled
// graph and its indexes, sort buffers, and a table and lists proportional to
// the arcs (n_r is unknown until the table is built).
uint64_t estimate(const nd_csr &g, int r) {
  const uint64_t m = (uint64_t)(g.nnz > 0 ? g.nnz : 0), n = (uint64_t)(g.n > 0 ? g.n : 0);
  const uint64_t per_arc = r <= 1 ? 48 : (r == 2 ? 96 : 192);
  return (64ull << 20) + 40 * n + per_arc * m;
}

}  // namespace

struct nd_server_s {
  int device = 0;
  uint64_t budget = 0, in_use = 0;
  bool stop = false;
  uint64_t next_id = 1;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Job *> queue;
  std::unordered_map<uint64_t, Job *> jobs;
  std::vector<std::thread> workers;
  std::vector<hipStream_t> streams;
  int running = 0;
  double scale[ND_MAX_S + 1][ND_MAX_S + 1];  // exact / estimate seen per (r, s)
  nd_server_s() {
    for (auto &row : scale)
      for (auto &x : row) x = 1.0;
  }
  // bytes the head job asks for at admission (under mu)
  uint64_t want(const Job *j) const {
    if (j->exact) return j->exact;
    const double x = (double)j->est_raw * scale[j->r][j->s];
    return x > 1.8e19 ? UINT64_MAX : (uint64_t)x;
  }
  // whether `extra` more bytes fit the budget (under mu); alone = no other job holds memory
  bool fits(uint64_t extra, bool alone) const {
    return budget == 0 || in_use + extra <= budget || alone;
  }
};

// Runs one admitted job on stream st.  Returns false when the job gave its
// memory back and went to the head of the queue again (its exact figure did
// not fit the budget).
static bool run_job(nd_server sv, Job *j, hipStream_t st) {
  if (j->ready && hipStreamWaitEvent(st, j->ready, 0) != hipSuccess) {
    hipGetLastError();
    j->st = ND_EHIP;
    j->err = "cannot order the job after the submitting stream";
    return true;
  }
  nd_plan plan = nullptr;
  void *ws = nullptr;
  j->st = nd_plan_create(&j->g, j->r, j->s, &j->opt, 0, st, &plan);
  for (int attempt = 0; j->st == ND_OK; attempt++) {
    uint64_t ws_bytes = 0, plan_bytes = 0;
    nd_plan_sizes(plan, &j->n_r, &ws_bytes, &plan_bytes);
    const uint64_t n1 = j->n_r ? j->n_r : 1;
    j->out_bytes = n1 * (uint64_t)j->r * 4 + n1 * 4;
    const uint64_t exact = plan_bytes + ws_bytes + j->out_bytes;
    bool fit;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      if (!j->exact && j->est_raw) {  // learn how far off the size-only estimate was
        const double ratio = (double)exact / (double)j->est_raw;
        double &sc = sv->scale[j->r][j->s];
        sc = std::min(64.0, std::max(sc, ratio));
      }
      fit = exact <= j->held || sv->fits(exact - j->held, sv->running == 1);
      if (fit) {
        sv->in_use = sv->in_use - j->held + exact;
        j->held = exact;
      }
      j->exact = exact;
    }
    if (!fit) {
      // free the plan first, then give the reservation back and wait at the
      // head of the queue for the exact figure
      nd_plan_destroy(plan);
      if (ws) hipFreeAsync(ws, st);
      if (j->rcl) hipFreeAsync(j->rcl, st);
      if (j->kappa) hipFreeAsync(j->kappa, st);
      j->rcl = nullptr;
      j->kappa = nullptr;
      hipStreamSynchronize(st);
      {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->in_use -= j->held;
        j->held = 0;
        j->requeues++;
        sv->running--;
        sv->queue.push_front(j);
      }
      sv->cv_work.notify_all();
      return false;
    }
    sv->cv_work.notify_all();  // a smaller exact figure frees budget for others
    if (ws) hipFreeAsync(ws, st);
    ws = nullptr;
    if (!j->rcl) {
      if (hipMallocAsync((void **)&j->rcl, n1 * (size_t)j->r * 4, st) != hipSuccess ||
          hipMallocAsync((void **)&j->kappa, n1 * 4, st) != hipSuccess) {
        hipGetLastError();
        j->st = ND_ENOMEM;
        j->err = "output allocation failed";
        break;
      }
      j->stream = st;
    }
    if (hipMallocAsync(&ws, ws_bytes ? ws_bytes : 256, st) != hipSuccess) {
      hipGetLastError();
      ws = nullptr;
      j->st = ND_ENOMEM;
      j->err = "workspace allocation failed";
      break;
    }
    j->st = nd_run(plan, ws, ws_bytes, j->rcl, j->kappa, nullptr, &j->stats);
    uint64_t again = 0;
    nd_plan_sizes(plan, nullptr, &again, nullptr);
    // a round outgrew the workspace: the plan now reports a larger one
    if (j->st == ND_ENOMEM && again > ws_bytes && attempt < 4) {
      j->st = ND_OK;
      continue;
    }
    break;
  }
  if (j->st != ND_OK && j->err.empty()) j->err = nd_last_error();
  if (ws) hipFreeAsync(ws, st);
  if (plan) nd_plan_destroy(plan);
  hipStreamSynchronize(st);
  return true;
}

static void worker_main(nd_server sv, int w) {
  hipSetDevice(sv->device);
  hipStream_t st = sv->streams[w];
  for (;;) {
    Job *j = nullptr;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_work.wait(lk, [&] {
        if (sv->stop) return true;
        if (sv->queue.empty()) return false;
        // FIFO admission by the memory budget; an oversized job runs alone
        return sv->fits(sv->want(sv->queue.front()), sv->running == 0);
      });
      if (sv->stop && sv->queue.empty()) return;
      if (sv->queue.empty()) continue;
      j = sv->queue.front();
      sv->queue.pop_front();
      j->held = sv->want(j);
      sv->in_use += j->held;
      sv->running++;
    }
    if (j->requeues == 0) j->t_start = Clock::now();
    if (!run_job(sv, j, st)) continue;  // back in the queue with its exact figure
    j->t_end = Clock::now();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      // the outputs stay counted until the job is released
      const uint64_t keep = j->st == ND_OK ? std::min(j->out_bytes, j->held) : 0;
      sv->in_use -= j->held - keep;
      j->held = keep;
      sv->running--;
      j->done = true;
    }
    sv->cv_done.notify_all();
    sv->cv_work.notify_all();
  }
}

extern "C" {

nd_status nd_server_create(int32_t workers, uint64_t hbm_budget_bytes, nd_server *out) {
  if (!out || workers < 1 || workers > 64) return ND_EINVAL;
  *out = nullptr;
  nd_server sv = new (std::nothrow) nd_server_s();
  if (!sv) return ND_ENOMEM;
  if (hipGetDevice(&sv->device) != hipSuccess) {
    delete sv;
    return ND_EHIP;
  }
  sv->budget = hbm_budget_bytes;
  for (int w = 0; w < workers; w++) {
    hipStream_t st = nullptr;
    if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
      for (hipStream_t x : sv->streams) hipStreamDestroy(x);
      delete sv;
      return ND_EHIP;
    }
    sv->streams.push_back(st);
  }
  for (int w = 0; w < workers; w++) sv->workers.emplace_back(worker_main, sv, w);
  *out = sv;
  return ND_OK;
}

nd_status nd_server_submit(nd_server sv, const nd_csr *g, int r, int s, const nd_options *opt,
                           void *hip_stream, uint64_t *job) {
  if (!sv || !g || !job) return ND_EINVAL;
  if (r < 1 || s <= r || s > ND_MAX_S) return ND_EINVAL;
  Job *j = new (std::nothrow) Job();
  if (!j) return ND_ENOMEM;
  j->g = *g;
  j->r = r;
  j->s = s;
  if (opt) j->opt = *opt;
  j->est_raw = estimate(*g, r);
  j->t_submit = Clock::now();
  // the job's first kernel waits for the work that produced the graph
  if (hipEventCreateWithFlags(&j->ready, hipEventDisableTiming) != hipSuccess ||
      hipEventRecord(j->ready, (hipStream_t)hip_stream) != hipSuccess) {
    hipGetLastError();
    if (j->ready) hipEventDestroy(j->ready);
    delete j;
    return ND_EHIP;
  }
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
      hipEventDestroy(j->ready);
      delete j;
      return ND_ESTATE;
    }
    j->id = sv->next_id++;
    sv->jobs[j->id] = j;
    sv->queue.push_back(j);
    *job = j->id;
  }
  sv->cv_work.notify_all();
  return ND_OK;
}

nd_status nd_server_wait(nd_server sv, uint64_t job, int32_t timeout_ms, int32_t *done) {
  if (!sv || !done) return ND_EINVAL;
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->jobs.find(job);
  if (it == sv->jobs.end()) return ND_EINVAL;
  Job *j = it->second;
  if (timeout_ms < 0) sv->cv_done.wait(lk, [&] { return j->done; });
  else sv->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return j->done; });
  *done = j->done ? 1 : 0;
  return ND_OK;
}

nd_status nd_server_result(nd_server sv, uint64_t job, uint64_t *n_r, const int32_t **rcliques_dev,
                           const uint32_t **kappa_dev, nd_stats *stats, double *queue_ms,
                           double *service_ms) {
  if (!sv) return ND_EINVAL;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->jobs.find(job);
  if (it == sv->jobs.end()) return ND_EINVAL;
  Job *j = it->second;
  if (!j->done) return ND_ESTATE;
  if (j->st != ND_OK) return j->st;
  if (n_r) *n_r = j->n_r;
  if (rcliques_dev) *rcliques_dev = j->rcl;
  if (kappa_dev) *kappa_dev = j->kappa;
  if (stats) *stats = j->stats;
  using ms = std::chrono::duration<double, std::milli>;
  if (queue_ms) *queue_ms = ms(j->t_start - j->t_submit).count();
  if (service_ms) *service_ms = ms(j->t_end - j->t_start).count();
  return ND_OK;
}

nd_status nd_server_copy(nd_server sv, uint64_t job, int32_t *rcliques_dst, uint32_t *kappa_dst) {
  if (!sv) return ND_EINVAL;
  Job *j = nullptr;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(job);
    if (it == sv->jobs.end()) return ND_EINVAL;
    j = it->second;
    if (!j->done) return ND_ESTATE;
    if (j->st != ND_OK) return j->st;
  }
  if (j->n_r == 0) return ND_OK;
  if (!rcliques_dst || !kappa_dst) return ND_EINVAL;
  if (hipMemcpyAsync(rcliques_dst, j->rcl, j->n_r * (size_t)j->r * 4, hipMemcpyDeviceToDevice,
                     j->stream) != hipSuccess ||
      hipMemcpyAsync(kappa_dst, j->kappa, j->n_r * 4, hipMemcpyDeviceToDevice, j->stream) !=
          hipSuccess ||
      hipStreamSynchronize(j->stream) != hipSuccess) {
    hipGetLastError();
    return ND_EHIP;
  }
  return ND_OK;
}

nd_status nd_server_release(nd_server sv, uint64_t job) {
  if (!sv) return ND_EINVAL;
  Job *j = nullptr;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->jobs.find(job);
    if (it == sv->jobs.end()) return ND_EINVAL;
    j = it->second;
    if (!j->done) return ND_ESTATE;
    sv->jobs.erase(it);
    sv->in_use -= j->held;  // the outputs
    j->held = 0;
  }
  sv->cv_work.notify_all();
  if (j->rcl) hipFreeAsync(j->rcl, j->stream);
  if (j->kappa) hipFreeAsync(j->kappa, j->stream);
  if (j->stream) hipStreamSynchronize(j->stream);
  if (j->ready) hipEventDestroy(j->ready);
  delete j;
  return ND_OK;
}

nd_status nd_server_destroy(nd_server sv) {
  if (!sv) return ND_OK;
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->stop = true;
  }
  sv->cv_work.notify_all();
  for (auto &t : sv->workers) t.join();
  for (auto &kv : sv->jobs) {
    Job *j = kv.second;
    if (j->rcl) hipFreeAsync(j->rcl, j->stream);
    if (j->kappa) hipFreeAsync(j->kappa, j->stream);
    if (j->stream) hipStreamSynchronize(j->stream);
    if (j->ready) hipEventDestroy(j->ready);
    delete j;
  }
  for (hipStream_t st : sv->streams) hipStreamDestroy(st);
  delete sv;
  return ND_OK;
}

}  // extern "C"
