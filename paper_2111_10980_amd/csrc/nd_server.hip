// Serving loop: continuous batching of (graph, r, s) decomposition jobs.
//
// A fixed pool of worker threads, each with its own HIP stream, takes jobs
// from one FIFO queue.  A job is admitted when a worker is idle and its
// device-memory estimate fits the remaining budget (a job larger than the
// whole budget runs alone).  An admitted job keeps its plan — oriented
// graph, r-clique table, bucket state — on the device until its last round,
// and the rounds of the jobs in flight interleave on the GPU through their
// streams; a job that arrives while others run starts as soon as a slot and
// memory are free, instead of waiting for the GPU to drain.  Results stay on
// the device until the caller releases them.
#include <hip/hip_runtime.h>
#include <string.h>

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
  uint64_t est = 0;
  nd_status st = ND_OK;
  std::string err;
  bool done = false;
  uint64_t n_r = 0;
  int32_t *rcl = nullptr;
  uint32_t *kappa = nullptr;
  hipStream_t stream = nullptr;  // stream its outputs were allocated on
  nd_stats stats{};
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
};

static void run_job(Job *j, hipStream_t st) {
  nd_plan plan = nullptr;
  j->st = nd_plan_create(&j->g, j->r, j->s, &j->opt, 0, st, &plan);
  if (j->st == ND_OK) {
    uint64_t bytes = 0;
    nd_plan_sizes(plan, &j->n_r, &bytes);
    const size_t rb = (size_t)(j->n_r ? j->n_r : 1) * (size_t)j->r * 4;
    const size_t kb = (size_t)(j->n_r ? j->n_r : 1) * 4;
    if (hipMallocAsync((void **)&j->rcl, rb, st) != hipSuccess ||
        hipMallocAsync((void **)&j->kappa, kb, st) != hipSuccess) {
      hipGetLastError();
      j->st = ND_ENOMEM;
      j->err = "output allocation failed";
    } else {
      j->stream = st;
      j->st = nd_run(plan, j->rcl, j->kappa, nullptr, &j->stats);
    }
  }
  if (j->st != ND_OK && j->err.empty()) j->err = nd_last_error();
  if (plan) nd_plan_destroy(plan);
  hipStreamSynchronize(st);
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
        const Job *h = sv->queue.front();
        // FIFO admission by the memory budget; an oversized job runs alone
        return sv->budget == 0 || sv->in_use + h->est <= sv->budget || sv->running == 0;
      });
      if (sv->stop && sv->queue.empty()) return;
      if (sv->queue.empty()) continue;
      j = sv->queue.front();
      sv->queue.pop_front();
      sv->in_use += j->est;
      sv->running++;
    }
    j->t_start = Clock::now();
    run_job(j, st);
    j->t_end = Clock::now();
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      sv->in_use -= j->est;
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
                           uint64_t *job) {
  if (!sv || !g || !job) return ND_EINVAL;
  if (r < 1 || s <= r || s > ND_MAX_S) return ND_EINVAL;
  Job *j = new (std::nothrow) Job();
  if (!j) return ND_ENOMEM;
  j->g = *g;
  j->r = r;
  j->s = s;
  if (opt) j->opt = *opt;
  j->est = estimate(*g, r);
  j->t_submit = Clock::now();
  {
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->stop) {
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
  }
  if (j->rcl) hipFreeAsync(j->rcl, j->stream);
  if (j->kappa) hipFreeAsync(j->kappa, j->stream);
  if (j->stream) hipStreamSynchronize(j->stream);
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
    delete j;
  }
  for (hipStream_t st : sv->streams) hipStreamDestroy(st);
  delete sv;
  return ND_OK;
}

}  // extern "C"
