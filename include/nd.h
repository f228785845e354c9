/*
 * nd.h -- C ABI of the MI355X (gfx950) (r,s) nucleus decomposition library.
 *
 * The operation (Shi, Dhulipala, Shun, "Theoretically and Practically
 * Efficient Parallel Nucleus Decomposition", Section 2, "(r,s) nucleus
 * decomposition problem"): given a simple undirected graph G and 1 <= r < s,
 * compute for every r-clique R of G its (r,s)-clique core number kappa(R),
 * the largest c such that R belongs to a set X of r-cliques in which every
 * member lies in at least c s-cliques whose r-subsets are all in X.  The
 * library follows Algorithm 2 ("arb-nucleus-decomp"): orient G, count the
 * s-cliques containing each r-clique (Count-Func), then peel the minimum
 * bucket round by round, re-listing the s-cliques of every peeled r-clique
 * and decrementing the other r-cliques in them (Update / Update-Func).
 *
 * Conventions of every entry point:
 *   - All pointers named *_dev are DEVICE pointers on the current HIP device;
 *     the caller owns them.  Host pointers are named *_host or are structs.
 *   - Memory: a plan owns its device state (relabeled graph, r-clique table,
 *     index, round control) until nd_plan_destroy.  Everything a run needs
 *     beyond that comes from a caller-owned device workspace whose exact size
 *     nd_plan_sizes reports; nd_run itself allocates nothing.
 *   - Work is enqueued on the stream given at plan creation and runs in
 *     stream order; entry points that return sizes or statistics synchronise
 *     that stream before returning.
 *   - Every entry point returns nd_status; nothing throws across the ABI.
 *     On error the outputs are unspecified, nd_last_error() holds a detail
 *     string for the calling thread, and a plan stays destroyable.
 *   - A plan is not thread-safe; separate plans are independent.
 */
#ifndef ND_H
#define ND_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ND_OK = 0,
  ND_EINVAL = 1,     /* bad argument: r < 1, s <= r, s > ND_MAX_S, null pointer, ... */
  ND_EGRAPH = 2,     /* CSR is not simple/symmetric/sorted, or ids out of range */
  ND_EKEYWIDTH = 3,  /* (r-1) * ceil(log2 n) > 126: an r-clique key does not fit two words */
  ND_EOVERFLOW = 4,  /* an s-clique count exceeds UINT32_MAX, the table exceeds 2^32-1 slots,
                        or the graph has more than 2^31-1 r-cliques */
  ND_ENOMEM = 5,     /* device memory budget exceeded or allocation failed */
  ND_EHIP = 6,       /* a HIP runtime call failed */
  ND_ESTATE = 7      /* entry point called in the wrong order */
} nd_status;

#define ND_MAX_S 8

/* Simple undirected graph in CSR form, DEVICE pointers, caller-owned.
 * row_ptr[n+1] (int64, row_ptr[0] = 0, row_ptr[n] = nnz), col[nnz] (int32);
 * each undirected edge appears in both rows; rows strictly ascending, no
 * self-loops (paper Section 2, "Graph Storage": CSR). */
typedef struct {
  int32_t n;
  int64_t nnz;
  const int64_t *row_ptr;
  const int32_t *col;
} nd_csr;

/* Options; zero-initialised = defaults. */
typedef struct {
  int32_t orient;        /* 0 = degree order (ties by id), 1 = exact core (degeneracy) order */
  int32_t timing;        /* 1 = time the count-listing and peel kernels with HIP events */
  float load_factor;     /* r-clique table load factor in (0, 0.9]; 0 = 0.5 */
  int32_t path;          /* 0 = auto; 1 = force the one-wave generic walker (Count-Func
                            atomics; each peeled r-clique's s-cliques listed by one wave
                            with edge tests) for every (r, s) */
  int32_t canonical;     /* 1 = output rows in lexicographic order of their vertices
                            (original ids); 0 = library order */
  uint32_t trace_cap;    /* round-trace capacity the workspace provides at first;
                            0 = min(n_r, 2^20) */
  uint64_t record_cap;   /* per-round record capacity the workspace provides at first
                            (s = r+1 and s >= r+2 paths); 0 = max(8 n_r, 2^18) for
                            s = r+1, max(4 n_r, 2^18) for s >= r+2 */
  uint64_t debug_count_bias; /* debug: the 32-bit range check of the initial counts sees
                                every count raised by this amount, so a bias above
                                UINT32_MAX - (largest count) makes nd_run return
                                ND_EOVERFLOW; 0 = off (results are never changed) */
  int32_t queue_depth;   /* most peel rounds queued between two reads of the device round
                            state, 1..32; 0 = 32 */
  int32_t contract;      /* (2,3) only: 1 = graph contraction (Section 4.6: after every 2n
                            peeled edges, the listed adjacency of each vertex that lost a
                            quarter of its neighbours since its last contraction is
                            filtered of its peeled edges); 0 = off (default: measured
                            slower on rMAT-18, since each triangle is listed once anyway) */
  int32_t graph_rounds;  /* 1 = the rounds queued after the first of each batch are
                            captured once into a HIP graph (per queue depth and grid
                            class) and replayed with one launch; 0 = plain launches.
                            Ignored with timing (events recorded by graph nodes cannot
                            be timed) */
  int32_t levels;        /* r-clique table levels (Section 4.1): 0 or 2 = two (an array over
                            the first vertex v1, hashed last-level tables keyed by the other
                            r-1 vertices); 3 = three, r >= 4 only (v1, then its out-arc to v2
                            found in v1's sorted row, hashed last-level tables per arc keyed
                            by the other r-2 vertices) */
} nd_options;

typedef struct {
  uint64_t n_r;          /* r-cliques */
  uint64_t n_s;          /* s-cliques */
  uint64_t rounds;       /* peeling rounds rho (Section 3.2, peeling complexity) */
  uint64_t k_advances;   /* times the level k moved to a new minimum bucket */
  uint64_t decrements;   /* count decrements applied while peeling */
  uint64_t discoveries;  /* (peeled r-clique, s-clique) pairs listed while peeling */
  uint64_t table_slots;  /* capacity of the r-clique table */
  uint32_t max_kappa;
  uint32_t max_out_degree; /* of the orientation */
  float ms[8];           /* phase times: 0 validate, 1 orient+relabel, 2 table,
                            3 count, 4 bucket init, 5 peel loop, 6 emit, 7 total (of this
                            call: a run that resumed a stopped peel counts no count phase
                            and only its own rounds) */
  float count_kernel_ms; /* with options.timing: time of the s-clique count kernels */
  float peel_kernel_ms;  /* with options.timing: summed time of every round's update
                            (apply) kernel -- k_apply3 / k_apply / k_gen_apply / k_peel --
                            alone, not the round's other passes */
  uint32_t count_launches;
  uint32_t peel_launches; /* with options.timing: update kernels timed (one per round) */
  uint64_t atomics;      /* returning atomic decrements issued: a decrement of a count that
                            is already at or below the level (Algorithm 2 clamps it to k)
                            is counted in decrements but needs no memory operation */
  uint64_t workspace_bytes;   /* workspace bytes the run carved */
  uint64_t max_round_records; /* largest number of records one peel round wrote */
  uint64_t max_round_arcs;    /* s >= r+2: largest number of out-arcs one round walked */
  uint32_t contractions;      /* (2,3): graph contraction passes */
  uint32_t key_words;         /* 64-bit words per r-clique key: 1, or 2 when the r-1
                                 vertex fields of ceil(log2 n) bits need more than 63 */
} nd_stats;

typedef struct nd_plan_s *nd_plan; /* opaque, library-owned */

/* Validate the graph (a1), orient and relabel it (a2: Section 2
 * "O(alpha)-Orientation", Section 4.4 "Graph Relabeling") and build the
 * two-level r-clique table (a3: Sections 4.1-4.3, contiguous last-level
 * tables, slot position = r-clique index).  A last-level key packs the
 * r-clique's other r-1 vertices, ceil(log2 n) bits each, into one 64-bit word,
 * or into two when they need more than 63 bits (ND_EKEYWIDTH beyond 126).  hbm_budget_bytes bounds the
 * plan's device memory plus the workspace its run needs (0 = no budget): a
 * plan that would exceed it fails with ND_ENOMEM once n_r is known, before
 * the table is allocated.  On success *out owns device memory until
 * nd_plan_destroy. */
nd_status nd_plan_create(const nd_csr *g, int r, int s, const nd_options *opt,
                         uint64_t hbm_budget_bytes, void *hip_stream, nd_plan *out);

/* Number of r-cliques (rows of the output), the exact workspace bytes nd_run
 * needs, and the device bytes the plan holds.  Any argument may be NULL. */
nd_status nd_plan_sizes(nd_plan p, uint64_t *n_r, uint64_t *workspace_bytes,
                        uint64_t *plan_bytes);

/* Count (Algorithm 2 Count-Func), bucket and peel (Algorithm 2 main loop,
 * Update, Update-Func), then emit (Algorithm 2 returns every r-clique with
 * its bucket).  workspace_dev: DEVICE, caller-owned, 256-byte aligned, at
 * least the workspace_bytes nd_plan_sizes reports (a larger one leaves more
 * room for round records); its contents are scratch, overwritten by the run.
 * Outputs (DEVICE, caller-owned):
 *   rcliques_dev[n_r * r]  int32: row i = the vertices (original ids,
 *                          ascending) of r-clique i; rows in library order,
 *                          or lexicographic with options.canonical;
 *   kappa_dev[n_r]         uint32: nucleus number of row i;
 *   counts_dev[n_r]        uint32, may be NULL: initial s-clique count of row i.
 * stats (host) may be NULL.  Every r-clique of G is a row, including those in
 * no s-clique (kappa 0).  Errors: ND_ENOMEM before any kernel when the
 * workspace is smaller than required or plan + workspace exceed the budget;
 * ND_ENOMEM after the peel started when one round needs more records (or
 * round-trace entries) than the workspace holds -- the plan then reports
 * the larger requirement through nd_plan_sizes and may be run again;
 * ND_EOVERFLOW when a count does not fit 32 bits.  After ND_ENOMEM for
 * records or out-arcs the plan keeps the peel's state (in host memory),
 * and the next nd_run on it goes on from the round that stopped; the rows,
 * kappa and counts of the whole peel are written by the run that finishes
 * (initial counts as the stopped run took them; a resumed run that asks
 * for counts the stopped run did not take starts again).  Otherwise a plan
 * may be run any number of times; each run starts again from the table. */
nd_status nd_run(nd_plan p, void *workspace_dev, uint64_t workspace_bytes, int32_t *rcliques_dev,
                 uint32_t *kappa_dev, uint32_t *counts_dev, nd_stats *stats);

/* Bytes of the static device workspace nd_run_noalloc uses (64 MiB). */
#define ND_NOALLOC_WORKSPACE_BYTES (64ull << 20)

/* nd_run for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same run, with the workspace taken from one static device array of
 * ND_NOALLOC_WORKSPACE_BYTES that the library holds on every GPU it runs on
 * until the process ends, instead of a caller buffer.  It calls no hipMalloc,
 * hipFree or other allocating routine.  Arguments and outputs as nd_run;
 * call it with the plan's device current.  Errors: ND_ENOMEM when the plan
 * needs a larger workspace than the static one (nd_plan_sizes tells), or
 * when a round outgrows it as in nd_run; ND_EINVAL on another device.
 * Every call on a GPU shares that GPU's array and leaves its contents
 * behind (a run overwrites everything it reads): calls that overlap on one
 * GPU -- from several threads, or on several streams without ordering --
 * race and must not be issued. */
nd_status nd_run_noalloc(nd_plan p, int32_t *rcliques_dev, uint32_t *kappa_dev,
                         uint32_t *counts_dev, nd_stats *stats);

/* Round sizes |A_t| and levels k_t of the last successful nd_run (host
 * arrays of capacity cap); *rounds receives rho.  Either array may be NULL. */
nd_status nd_round_trace(nd_plan p, uint64_t *sizes_host, uint32_t *levels_host, uint64_t cap,
                         uint64_t *rounds);

nd_status nd_plan_destroy(nd_plan p);

/* ---- Batched decomposition of many independent graphs ------------------
 * The batch is decomposed as one disjoint union: kappa of an r-clique is
 * determined by its connected component (the definition in Section 2 only
 * involves s-cliques that contain it), so every graph's result equals its
 * own decomposition while all graphs share each kernel launch and every
 * peeling round.  Graphs are CSRs as in nd_plan_create (DEVICE pointers,
 * caller-owned, may be freed after nd_batch_create returns); count may be 0
 * and graphs may be empty. */
typedef struct nd_batch_s *nd_batch;

nd_status nd_batch_create(const nd_csr *graphs, int32_t count, int r, int s,
                          const nd_options *opt, uint64_t hbm_budget_bytes, void *hip_stream,
                          nd_batch *out);

/* Total rows over all graphs (sum of their r-clique counts), the count, and
 * the exact workspace bytes nd_batch_run needs.  Any argument may be NULL. */
nd_status nd_batch_sizes(nd_batch b, uint64_t *n_r_total, int32_t *count,
                         uint64_t *workspace_bytes);

/* Runs the decomposition with a caller-owned DEVICE workspace as in nd_run.
 * Outputs are grouped by graph: the rows of graph g are
 * [row_offsets_host[g], row_offsets_host[g+1]) (host array of count+1), with
 * vertex ids local to graph g (ascending within a row); rows within a graph
 * are in no particular order, or lexicographic with options.canonical.
 * rcliques_dev[n_r_total * r], kappa_dev[n_r_total], counts_dev (nullable)
 * as in nd_run.  Errors as nd_run; may be run again. */
nd_status nd_batch_run(nd_batch b, void *workspace_dev, uint64_t workspace_bytes,
                       int32_t *rcliques_dev, uint32_t *kappa_dev, uint32_t *counts_dev,
                       uint64_t *row_offsets_host, nd_stats *stats);

/* Rounds of the shared peel (every graph's rounds interleaved). */
nd_status nd_batch_round_trace(nd_batch b, uint64_t *sizes_host, uint32_t *levels_host,
                               uint64_t cap, uint64_t *rounds);

nd_status nd_batch_destroy(nd_batch b);

/* Schedule autotuner for batched decompositions.  Decomposes a held-out
 * sample of the graphs -- at most sample_count of them, spread evenly over
 * the input -- as one batch under each candidate setting and returns the
 * fastest setting in *best (base's other fields are kept; base may be NULL).
 * Candidates: orientation (degree order, core order) x queue depth (8, 32)
 * x replay of queued rounds from captured graphs (off, on).  Each candidate
 * is timed, host clock around plan creation and run, as the better of two
 * runs after a warm-up.  report (nullable) receives every candidate with its
 * time and the index of the best.  Graphs as in nd_batch_create; device
 * memory comes from the library's pool and is returned; the sample's
 * results are discarded. */
#define ND_TUNE_MAX 16
typedef struct {
  int32_t candidates;
  int32_t best;
  int32_t sample_graphs;
  nd_options opt[ND_TUNE_MAX];
  float ms[ND_TUNE_MAX];
} nd_tune_report;

nd_status nd_batch_autotune(const nd_csr *graphs, int32_t count, int r, int s,
                            const nd_options *base, int32_t sample_count, void *hip_stream,
                            nd_options *best, nd_tune_report *report);

/* ---- Serving: continuous batching of (graph, r, s) jobs ----------------
 * A pool of `workers` threads, each with its own HIP stream on the device
 * current at creation, takes jobs from one FIFO queue.  Admission is by
 * hbm_budget_bytes (0 = no budget): a job starts its plan when a worker is
 * idle and an estimate from its size fits what is left of the budget; once
 * its plan exists the job holds exactly the plan's bytes plus its run's
 * workspace and outputs (nd_plan_sizes).  A job whose exact figure does not
 * fit gives its plan back and waits at the head of the queue for that
 * figure; a job larger than the whole budget runs alone.  Jobs that arrive
 * while others run are admitted as slots and memory free up, and their peel
 * rounds interleave on the GPU.  The caller keeps each submitted graph's
 * device memory alive until the job is done.  Results stay on the device
 * until nd_server_release. */
typedef struct nd_server_s *nd_server;

nd_status nd_server_create(int32_t workers, uint64_t hbm_budget_bytes, nd_server *out);

/* Queue one decomposition; *job receives its id.  opt may be NULL.
 * hip_stream is the stream that produced the graph (NULL = the null
 * stream): the job's first kernel waits for everything enqueued on it
 * before this call. */
nd_status nd_server_submit(nd_server sv, const nd_csr *g, int r, int s, const nd_options *opt,
                           void *hip_stream, uint64_t *job);

/* Wait up to timeout_ms (-1 = without limit); *done = 1 once the job ended. */
nd_status nd_server_wait(nd_server sv, uint64_t job, int32_t timeout_ms, int32_t *done);

/* Outputs of a finished job (library-owned DEVICE arrays as in nd_run:
 * rcliques [n_r * r], kappa [n_r]), its statistics, and the time it waited
 * in the queue and spent running.  Returns the job's own status if it failed. */
nd_status nd_server_result(nd_server sv, uint64_t job, uint64_t *n_r,
                           const int32_t **rcliques_dev, const uint32_t **kappa_dev,
                           nd_stats *stats, double *queue_ms, double *service_ms);

/* Copy a finished job's outputs into caller-owned device buffers of
 * n_r * r int32 and n_r uint32 and wait for the copy. */
nd_status nd_server_copy(nd_server sv, uint64_t job, int32_t *rcliques_dst, uint32_t *kappa_dst);

/* Free a finished job's outputs. */
nd_status nd_server_release(nd_server sv, uint64_t job);

/* Finish the queued jobs, stop the workers, free everything. */
nd_status nd_server_destroy(nd_server sv);

/* Free the library's cached device blocks (its allocator keeps freed blocks
 * for reuse by later plans). */
nd_status nd_release_cached(void);

const char *nd_status_str(nd_status st);
const char *nd_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* ND_H */
