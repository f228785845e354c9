/*
 * CPU ORACLE for (r,s) nucleus decomposition -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential, deliberately slow and obviously correct.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * file's library; the product path never does.  It shares no code, header,
 * table or helper with the GPU library.
 *
 * What it computes (paper Section 2, definition of the (r,s)-clique core
 * number, and Algorithm 2 "arb-nucleus-decomp"):
 *   - every r-clique of the simple undirected input graph, as a sorted tuple
 *     of original vertex ids, kept in one lexicographically sorted array whose
 *     position is the r-clique's index (lookup = binary search);
 *   - its initial s-clique count: every s-clique is enumerated once and each
 *     of its C(s,r) r-subsets gets +1 (Algorithm 2, Count-Func);
 *   - its nucleus number kappa by bulk-round peeling (Algorithm 2 main loop
 *     with Update / Update-Func), and, as an independent second algorithm,
 *     by one-at-a-time peeling (the classical sequential peel the paper's
 *     related-work section attributes to Matula and Beck for k-cores).
 *
 * Readings taken where the paper is silent (each is listed in the design
 * notes):
 *   - r-cliques in no s-clique are in T with count 0 and get kappa 0.
 *   - "subtract 1/a" (Update-Func) is realised exactly with integers: of the
 *     a r-subsets of S peeled in the same round, only the one with the
 *     smallest index decrements the live subsets of S, each by 1.
 *   - "previously peeled" = stamped in an earlier round; a round is every
 *     live r-clique whose count is <= the current level k, where
 *     k = max(k, min live count) (the bucket of Section 2 "Parallel
 *     Bucketing" always extracts the minimum bucket; counts that fall below
 *     k are clamped to k, so they are peeled in the next round at level k).
 *   - The dense bucket array of the sequential variant (Section 3.2
 *     "Discussion", appendix A) is used as the bucket structure: one doubly
 *     linked list per count value.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_S 8
#define ORC_LIVE UINT32_MAX

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_EGRAPH = 2, ORC_ENOMEM = 5 };

typedef struct {
  int32_t n;
  const int64_t *rp;
  const int32_t *col;
} ograph;

typedef struct {
  int r, s;
  int64_t n_r;       /* number of r-cliques */
  int32_t *tup;      /* n_r * r vertex ids, rows sorted, rows in lex order */
  int64_t *first;    /* n+1: rows whose first vertex is v are [first[v], first[v+1]) */
  uint64_t *count0;  /* initial s-clique counts */
  uint64_t *count;   /* working counts */
  uint32_t *stamp;   /* round in which the r-clique was peeled, or ORC_LIVE */
  uint64_t *kappa;   /* nucleus numbers */
  uint64_t n_s;      /* number of s-cliques */
  uint64_t rounds;
  uint64_t *round_size; /* |A_t| per round */
  uint64_t *round_k;    /* level k of each round */
  uint64_t round_cap;
  uint64_t discoveries; /* (R, S) pairs found while peeling */
  uint64_t decrements;  /* total count decrements */
  uint64_t max_kappa;
  /* combinations: all r-subsets of {0..s-1}, lexicographic */
  int ncomb;
  int comb[70][ORC_MAX_S];
} ores;

/* ---------------------------------------------------------------- graph -- */

static int validate(const ograph *g) {
  if (g->n < 0) return ORC_EINVAL;
  if (g->n == 0) return ORC_OK;
  if (!g->rp || (g->rp[g->n] > 0 && !g->col)) return ORC_EINVAL;
  if (g->rp[0] != 0) return ORC_EGRAPH;
  for (int32_t v = 0; v < g->n; v++) {
    if (g->rp[v + 1] < g->rp[v]) return ORC_EGRAPH;
    for (int64_t i = g->rp[v]; i < g->rp[v + 1]; i++) {
      int32_t u = g->col[i];
      if (u < 0 || u >= g->n || u == v) return ORC_EGRAPH;
      if (i > g->rp[v] && g->col[i - 1] >= u) return ORC_EGRAPH;
    }
  }
  /* symmetry: every arc has its reverse (checked by binary search) */
  for (int32_t v = 0; v < g->n; v++) {
    for (int64_t i = g->rp[v]; i < g->rp[v + 1]; i++) {
      int32_t u = g->col[i];
      int64_t lo = g->rp[u], hi = g->rp[u + 1];
      int found = 0;
      while (lo < hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (g->col[mid] == v) { found = 1; break; }
        if (g->col[mid] < v) lo = mid + 1; else hi = mid;
      }
      if (!found) return ORC_EGRAPH;
    }
  }
  return ORC_OK;
}

static int adjacent(const ograph *g, int32_t u, int32_t v) {
  int64_t lo = g->rp[u], hi = g->rp[u + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    if (g->col[mid] == v) return 1;
    if (g->col[mid] < v) lo = mid + 1; else hi = mid;
  }
  return 0;
}

/* ------------------------------------------------------------ listing ---- */

/* Enumerate every c-clique {x_0 < x_1 < ... < x_{c-1}} whose vertices are
 * drawn from the sorted candidate array cand (all of them adjacent to the
 * vertices already in cur[0..depth)), in lexicographic order. */
typedef void (*clique_fn)(void *ctx, const int32_t *clique);

static void enum_rec(const ograph *g, int c, int32_t *cur, int depth,
                     const int32_t *cand, int64_t ncand, clique_fn fn, void *ctx) {
  if (depth == c) { fn(ctx, cur); return; }
  int32_t *next = (int32_t *)malloc(sizeof(int32_t) * (size_t)(ncand > 0 ? ncand : 1));
  for (int64_t i = 0; i < ncand; i++) {
    int32_t x = cand[i];
    cur[depth] = x;
    int64_t nn = 0;
    if (depth + 1 < c)
      for (int64_t j = i + 1; j < ncand; j++)
        if (adjacent(g, x, cand[j])) next[nn++] = cand[j];
    enum_rec(g, c, cur, depth + 1, next, nn, fn, ctx);
  }
  free(next);
}

/* All c-cliques of the graph, lexicographic. */
static void enum_cliques(const ograph *g, int c, clique_fn fn, void *ctx) {
  int32_t cur[ORC_MAX_S];
  for (int32_t v = 0; v < g->n; v++) {
    cur[0] = v;
    if (c == 1) { fn(ctx, cur); continue; }
    /* candidates: neighbours greater than v */
    int64_t lo = g->rp[v], hi = g->rp[v + 1], nn = 0;
    int32_t *cand = (int32_t *)malloc(sizeof(int32_t) * (size_t)(hi - lo + 1));
    for (int64_t i = lo; i < hi; i++)
      if (g->col[i] > v) cand[nn++] = g->col[i];
    enum_rec(g, c, cur, 1, cand, nn, fn, ctx);
    free(cand);
  }
}

/* ------------------------------------------------------------- table ----- */

typedef struct { ores *res; int64_t fill; int counting; } build_ctx;

static void rclique_cb(void *vctx, const int32_t *cl) {
  build_ctx *b = (build_ctx *)vctx;
  if (!b->counting) memcpy(b->res->tup + (size_t)b->fill * b->res->r, cl, sizeof(int32_t) * b->res->r);
  b->fill++;
}

static int tuple_cmp(const int32_t *a, const int32_t *b, int r) {
  for (int i = 0; i < r; i++) {
    if (a[i] < b[i]) return -1;
    if (a[i] > b[i]) return 1;
  }
  return 0;
}

/* index of the sorted r-tuple R, or -1 */
static int64_t lookup(const ores *res, const int32_t *R) {
  int64_t lo = res->first[R[0]], hi = res->first[R[0] + 1];
  while (lo < hi) {
    int64_t mid = lo + (hi - lo) / 2;
    int c = tuple_cmp(res->tup + (size_t)mid * res->r, R, res->r);
    if (c == 0) return mid;
    if (c < 0) lo = mid + 1; else hi = mid;
  }
  return -1;
}

/* ------------------------------------------------------------- count ----- */

typedef struct { ores *res; int bad; } count_ctx;

static void sclique_cb(void *vctx, const int32_t *S) {
  count_ctx *c = (count_ctx *)vctx;
  ores *res = c->res;
  res->n_s++;
  int32_t R[ORC_MAX_S];
  for (int q = 0; q < res->ncomb; q++) {
    for (int i = 0; i < res->r; i++) R[i] = S[res->comb[q][i]];
    int64_t idx = lookup(res, R);
    if (idx < 0) { c->bad = 1; return; }
    res->count0[idx] += 1; /* Count-Func: +1 on T[R] for every r-subset */
  }
}

static void make_combs(ores *res) {
  int r = res->r, s = res->s, idx[ORC_MAX_S];
  for (int i = 0; i < r; i++) idx[i] = i;
  res->ncomb = 0;
  for (;;) {
    memcpy(res->comb[res->ncomb++], idx, sizeof(int) * r);
    int i = r - 1;
    while (i >= 0 && idx[i] == s - r + i) i--;
    if (i < 0) break;
    idx[i]++;
    for (int j = i + 1; j < r; j++) idx[j] = idx[j - 1] + 1;
  }
}

/* ----------------------------------------------------------- buckets ----- */

/* Dense bucket array: one doubly linked list per count value. */
typedef struct {
  uint64_t nb;
  int64_t *head;
  int64_t *next, *prev;
  uint64_t *key; /* bucket an item currently sits in */
} bucketq;

static int bq_init(bucketq *q, uint64_t nb, int64_t n_items) {
  q->nb = nb;
  q->head = (int64_t *)malloc(sizeof(int64_t) * nb);
  q->next = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_items + 1));
  q->prev = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_items + 1));
  q->key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n_items + 1));
  if (!q->head || !q->next || !q->prev || !q->key) return ORC_ENOMEM;
  for (uint64_t b = 0; b < nb; b++) q->head[b] = -1;
  return ORC_OK;
}

static void bq_free(bucketq *q) {
  free(q->head); free(q->next); free(q->prev); free(q->key);
}

static void bq_insert(bucketq *q, int64_t x, uint64_t b) {
  q->key[x] = b;
  q->prev[x] = -1;
  q->next[x] = q->head[b];
  if (q->head[b] >= 0) q->prev[q->head[b]] = x;
  q->head[b] = x;
}

static void bq_remove(bucketq *q, int64_t x) {
  uint64_t b = q->key[x];
  if (q->prev[x] >= 0) q->next[q->prev[x]] = q->next[x]; else q->head[b] = q->next[x];
  if (q->next[x] >= 0) q->prev[q->next[x]] = q->prev[x];
}

/* ------------------------------------------------------------- peel ------ */

/* Enumerate every s-clique that contains the r-clique R: the remaining
 * s-r vertices form a clique inside I = intersection of N(v), v in R
 * (Algorithm 2, Update). */
typedef void (*sfn)(void *ctx, const int32_t *S);

typedef struct {
  const ograph *g;
  const int32_t *R;
  int r, s;
  sfn fn;
  void *ctx;
} ext_ctx;

static void ext_cb(void *vctx, const int32_t *Q) {
  ext_ctx *e = (ext_ctx *)vctx;
  int32_t S[ORC_MAX_S];
  /* merge the two sorted tuples */
  int i = 0, j = 0, k = 0, q = e->s - e->r;
  while (i < e->r || j < q) {
    if (j >= q || (i < e->r && e->R[i] < Q[j])) S[k++] = e->R[i++];
    else S[k++] = Q[j++];
  }
  e->fn(e->ctx, S);
}

static void sets_containing(const ograph *g, const int32_t *R, int r, int s, sfn fn, void *ctx) {
  /* I = N(R[0]) intersected with N(R[1]), ... (sorted merge) */
  int64_t len = g->rp[R[0] + 1] - g->rp[R[0]];
  int32_t *I = (int32_t *)malloc(sizeof(int32_t) * (size_t)(len + 1));
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(len + 1));
  memcpy(I, g->col + g->rp[R[0]], sizeof(int32_t) * (size_t)len);
  for (int t = 1; t < r; t++) {
    const int32_t *b = g->col + g->rp[R[t]];
    int64_t lb = g->rp[R[t] + 1] - g->rp[R[t]], i = 0, j = 0, nn = 0;
    while (i < len && j < lb) {
      if (I[i] == b[j]) { tmp[nn++] = I[i]; i++; j++; }
      else if (I[i] < b[j]) i++;
      else j++;
    }
    memcpy(I, tmp, sizeof(int32_t) * (size_t)nn);
    len = nn;
  }
  ext_ctx e = {g, R, r, s, fn, ctx};
  int32_t cur[ORC_MAX_S];
  enum_rec(g, s - r, cur, 0, I, len, ext_cb, &e);
  free(I);
  free(tmp);
}

typedef struct {
  ores *res;
  bucketq *q;
  int64_t self;   /* index of the peeled r-clique R */
  uint32_t t;     /* current round */
  uint64_t k;     /* current level */
  int single;     /* one-at-a-time variant */
  int bad;
} upd_ctx;

/* Update-Func for one s-clique S found from the peeled r-clique R = self. */
static void update_cb(void *vctx, const int32_t *S) {
  upd_ctx *u = (upd_ctx *)vctx;
  ores *res = u->res;
  int32_t R[ORC_MAX_S];
  int64_t idx[70];
  res->discoveries++;
  int64_t owner = INT64_MAX;
  for (int c = 0; c < res->ncomb; c++) {
    for (int i = 0; i < res->r; i++) R[i] = S[res->comb[c][i]];
    idx[c] = lookup(res, R);
    if (idx[c] < 0) { u->bad = 1; return; }
    uint32_t st = res->stamp[idx[c]];
    if (st != ORC_LIVE && st < u->t) return;           /* S destroyed earlier */
    if (st == u->t && idx[c] < owner) owner = idx[c];  /* peeled this round */
  }
  if (owner != u->self) return; /* exactly one peeled subset applies S's -1 */
  for (int c = 0; c < res->ncomb; c++) {
    int64_t x = idx[c];
    if (res->stamp[x] != ORC_LIVE) continue;
    if (res->count[x] == 0) { u->bad = 1; return; }
    res->count[x] -= 1;
    res->decrements++;
    uint64_t nb = res->count[x] > u->k ? res->count[x] : u->k;
    bq_remove(u->q, x);
    bq_insert(u->q, x, nb);
  }
}

static int push_round(ores *res, uint64_t size, uint64_t k) {
  if (res->rounds == res->round_cap) {
    uint64_t cap = res->round_cap ? 2 * res->round_cap : 64;
    uint64_t *a = (uint64_t *)realloc(res->round_size, sizeof(uint64_t) * cap);
    if (!a) return ORC_ENOMEM;
    res->round_size = a;
    uint64_t *b = (uint64_t *)realloc(res->round_k, sizeof(uint64_t) * cap);
    if (!b) return ORC_ENOMEM;
    res->round_k = b;
    res->round_cap = cap;
  }
  res->round_size[res->rounds] = size;
  res->round_k[res->rounds] = k;
  res->rounds++;
  return ORC_OK;
}

static int peel(const ograph *g, ores *res, int single) {
  uint64_t maxc = 0;
  for (int64_t i = 0; i < res->n_r; i++) {
    res->count[i] = res->count0[i];
    res->stamp[i] = ORC_LIVE;
    if (res->count0[i] > maxc) maxc = res->count0[i];
  }
  bucketq q;
  if (bq_init(&q, maxc + 1, res->n_r) != ORC_OK) { bq_free(&q); return ORC_ENOMEM; }
  for (int64_t i = res->n_r - 1; i >= 0; i--) bq_insert(&q, i, res->count[i]);
  uint64_t k = 0, finished = 0;
  uint32_t t = 0;
  int64_t *A = (int64_t *)malloc(sizeof(int64_t) * (size_t)(res->n_r + 1));
  int32_t Rv[ORC_MAX_S];
  int rc = ORC_OK;
  while (finished < (uint64_t)res->n_r) {
    while (q.head[k] < 0) k++; /* minimum non-empty bucket; never below k */
    int64_t na = 0;
    if (single) {
      /* pop one r-clique of the minimum bucket */
      int64_t x = q.head[k];
      bq_remove(&q, x);
      A[na++] = x;
    } else {
      /* the whole bucket is this round's A; later arrivals go to the next */
      for (int64_t x = q.head[k]; x >= 0; x = q.next[x]) A[na++] = x;
      q.head[k] = -1;
    }
    for (int64_t i = 0; i < na; i++) {
      res->stamp[A[i]] = t;
      res->kappa[A[i]] = k;
      if (k > res->max_kappa) res->max_kappa = k;
    }
    finished += (uint64_t)na;
    if (!single) {
      rc = push_round(res, (uint64_t)na, k);
      if (rc) break;
    }
    /* Update: every peeled R re-lists its s-cliques */
    upd_ctx u = {res, &q, 0, t, k, single, 0};
    /* sort A by index so the run is reproducible */
    for (int64_t i = 1; i < na; i++) {
      int64_t x = A[i], j = i - 1;
      while (j >= 0 && A[j] > x) { A[j + 1] = A[j]; j--; }
      A[j + 1] = x;
    }
    for (int64_t i = 0; i < na; i++) {
      u.self = A[i];
      memcpy(Rv, res->tup + (size_t)A[i] * res->r, sizeof(int32_t) * res->r);
      sets_containing(g, Rv, res->r, res->s, update_cb, &u);
      if (u.bad) { rc = ORC_EINVAL; break; }
    }
    if (rc) break;
    t++;
  }
  if (single) res->rounds = 0;
  free(A);
  bq_free(&q);
  return rc;
}

/* ------------------------------------------------------------ driver ----- */

void ndo_free(ores *res);

int ndo_decompose(int32_t n, const int64_t *row_ptr, const int32_t *col, int r, int s,
                  int single, ores **out) {
  *out = NULL;
  if (r < 1 || s <= r || s > ORC_MAX_S) return ORC_EINVAL;
  ograph g = {n, row_ptr, col};
  int rc = validate(&g);
  if (rc) return rc;
  ores *res = (ores *)calloc(1, sizeof(ores));
  if (!res) return ORC_ENOMEM;
  res->r = r;
  res->s = s;
  make_combs(res);
  /* 1. all r-cliques, lexicographic */
  build_ctx b = {res, 0, 1};
  enum_cliques(&g, r, rclique_cb, &b);
  res->n_r = b.fill;
  res->tup = (int32_t *)malloc(sizeof(int32_t) * (size_t)(res->n_r * r + 1));
  res->first = (int64_t *)calloc((size_t)n + 2, sizeof(int64_t));
  res->count0 = (uint64_t *)calloc((size_t)res->n_r + 1, sizeof(uint64_t));
  res->count = (uint64_t *)calloc((size_t)res->n_r + 1, sizeof(uint64_t));
  res->stamp = (uint32_t *)calloc((size_t)res->n_r + 1, sizeof(uint32_t));
  res->kappa = (uint64_t *)calloc((size_t)res->n_r + 1, sizeof(uint64_t));
  if (!res->tup || !res->first || !res->count0 || !res->count || !res->stamp || !res->kappa) {
    ndo_free(res);
    return ORC_ENOMEM;
  }
  b.fill = 0;
  b.counting = 0;
  enum_cliques(&g, r, rclique_cb, &b);
  /* first-vertex offsets */
  for (int64_t i = 0; i < res->n_r; i++) res->first[res->tup[(size_t)i * r] + 1]++;
  for (int32_t v = 0; v < n; v++) res->first[v + 1] += res->first[v];
  /* 2. initial counts: every s-clique adds 1 to each of its r-subsets */
  count_ctx c = {res, 0};
  enum_cliques(&g, s, sclique_cb, &c);
  if (c.bad) { ndo_free(res); return ORC_EINVAL; }
  /* 3. peel */
  rc = peel(&g, res, single);
  if (rc) { ndo_free(res); return rc; }
  *out = res;
  return ORC_OK;
}

/* Initial counts only (no peel). */
int ndo_count(int32_t n, const int64_t *row_ptr, const int32_t *col, int r, int s, ores **out) {
  *out = NULL;
  if (r < 1 || s <= r || s > ORC_MAX_S) return ORC_EINVAL;
  ograph g = {n, row_ptr, col};
  int rc = validate(&g);
  if (rc) return rc;
  ores *res = (ores *)calloc(1, sizeof(ores));
  if (!res) return ORC_ENOMEM;
  res->r = r;
  res->s = s;
  make_combs(res);
  build_ctx b = {res, 0, 1};
  enum_cliques(&g, r, rclique_cb, &b);
  res->n_r = b.fill;
  res->tup = (int32_t *)malloc(sizeof(int32_t) * (size_t)(res->n_r * r + 1));
  res->first = (int64_t *)calloc((size_t)n + 2, sizeof(int64_t));
  res->count0 = (uint64_t *)calloc((size_t)res->n_r + 1, sizeof(uint64_t));
  if (!res->tup || !res->first || !res->count0) { ndo_free(res); return ORC_ENOMEM; }
  b.fill = 0;
  b.counting = 0;
  enum_cliques(&g, r, rclique_cb, &b);
  for (int64_t i = 0; i < res->n_r; i++) res->first[res->tup[(size_t)i * r] + 1]++;
  for (int32_t v = 0; v < n; v++) res->first[v + 1] += res->first[v];
  count_ctx c = {res, 0};
  enum_cliques(&g, s, sclique_cb, &c);
  if (c.bad) { ndo_free(res); return ORC_EINVAL; }
  *out = res;
  return ORC_OK;
}

/* Validation alone (same rules as the decomposition). */
int ndo_validate(int32_t n, const int64_t *row_ptr, const int32_t *col) {
  ograph g = {n, row_ptr, col};
  return validate(&g);
}

/* The s-cliques containing one given r-clique (sorted original ids), counted
 * directly: (s-r)-cliques inside the common neighbourhood. */
typedef struct { uint64_t n; } cnt_ctx;
static void cnt_cb(void *vctx, const int32_t *S) { (void)S; ((cnt_ctx *)vctx)->n++; }

uint64_t ndo_count_one(int32_t n, const int64_t *row_ptr, const int32_t *col, int r, int s,
                       const int32_t *R) {
  (void)n;
  ograph g = {n, row_ptr, col};
  cnt_ctx c = {0};
  sets_containing(&g, R, r, s, cnt_cb, &c);
  return c.n;
}

/* Local certificate for one r-clique R given a kappa assignment of all
 * r-cliques (looked up through `kap_of`, a sorted table passed in as tuples):
 * returns the number of s-cliques S containing R whose other r-subsets all
 * have kappa >= c, for c = threshold. */
typedef struct {
  const ograph *g;
  int r, s;
  const int32_t *tab;     /* sorted r-tuples */
  const int64_t *first;   /* first-vertex offsets over the table */
  const uint32_t *kap;    /* kappa per table row */
  const int32_t *self;    /* the r-clique whose support is measured */
  uint64_t threshold;
  uint64_t hits;
  int ncomb;
  int comb[70][ORC_MAX_S];
  int bad;
} cert_ctx;

static void cert_cb(void *vctx, const int32_t *S) {
  cert_ctx *c = (cert_ctx *)vctx;
  int32_t R[ORC_MAX_S];
  for (int q = 0; q < c->ncomb; q++) {
    for (int i = 0; i < c->r; i++) R[i] = S[c->comb[q][i]];
    if (tuple_cmp(R, c->self, c->r) == 0) continue;
    int64_t lo = c->first[R[0]], hi = c->first[R[0] + 1], at = -1;
    while (lo < hi) {
      int64_t mid = lo + (hi - lo) / 2;
      int cmp = tuple_cmp(c->tab + (size_t)mid * c->r, R, c->r);
      if (cmp == 0) { at = mid; break; }
      if (cmp < 0) lo = mid + 1; else hi = mid;
    }
    if (at < 0) { c->bad = 1; return; }
    if (c->kap[at] < c->threshold) return;
  }
  c->hits++;
}

int64_t ndo_support_at(int32_t n, const int64_t *row_ptr, const int32_t *col, int r, int s,
                       const int32_t *tab, const int64_t *first, const uint32_t *kap,
                       const int32_t *R, uint64_t threshold) {
  ograph g = {n, row_ptr, col};
  cert_ctx c;
  memset(&c, 0, sizeof(c));
  c.g = &g; c.r = r; c.s = s; c.tab = tab; c.first = first; c.kap = kap; c.self = R;
  c.threshold = threshold;
  ores tmp;
  memset(&tmp, 0, sizeof(tmp));
  tmp.r = r; tmp.s = s;
  make_combs(&tmp);
  c.ncomb = tmp.ncomb;
  memcpy(c.comb, tmp.comb, sizeof(c.comb));
  sets_containing(&g, R, r, s, cert_cb, &c);
  if (c.bad) return -1;
  return (int64_t)c.hits;
}

/* ----------------------------------------------------------- accessors --- */

int64_t ndo_n_r(const ores *res) { return res->n_r; }
uint64_t ndo_n_s(const ores *res) { return res->n_s; }
uint64_t ndo_rounds(const ores *res) { return res->rounds; }
uint64_t ndo_discoveries(const ores *res) { return res->discoveries; }
uint64_t ndo_decrements(const ores *res) { return res->decrements; }
uint64_t ndo_max_kappa(const ores *res) { return res->max_kappa; }

void ndo_copy(const ores *res, int32_t *tup, uint64_t *count0, uint64_t *kappa) {
  if (tup) memcpy(tup, res->tup, sizeof(int32_t) * (size_t)(res->n_r * res->r));
  if (count0) memcpy(count0, res->count0, sizeof(uint64_t) * (size_t)res->n_r);
  if (kappa && res->kappa) memcpy(kappa, res->kappa, sizeof(uint64_t) * (size_t)res->n_r);
}

/* Counts after peeling (the initial count minus every decrement received). */
void ndo_copy_final(const ores *res, uint64_t *count) {
  if (count && res->count) memcpy(count, res->count, sizeof(uint64_t) * (size_t)res->n_r);
}

void ndo_copy_rounds(const ores *res, uint64_t *size, uint64_t *k) {
  if (size) memcpy(size, res->round_size, sizeof(uint64_t) * (size_t)res->rounds);
  if (k) memcpy(k, res->round_k, sizeof(uint64_t) * (size_t)res->rounds);
}

void ndo_free(ores *res) {
  if (!res) return;
  free(res->tup); free(res->first); free(res->count0); free(res->count);
  free(res->stamp); free(res->kappa); free(res->round_size); free(res->round_k);
  free(res);
}
