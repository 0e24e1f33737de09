/*
 * Deterministic graph builder for the synthetic workloads (input preparation).
 *
 * The paper searches a fixed out-degree directed graph built with the Vamana
 * algorithm: per node, a greedy search over the current graph collects
 * candidates, and a pruning rule keeps at most R diverse out-neighbours
 * (Appendix A "search" and "pruning"; Appendix C settings: alpha = 1.2 for
 * Euclidean distance, 0.95 for inner product).  Euclidean pruning drops a
 * candidate c when an already kept neighbour s has alpha * d(s,c) <= d(p,c).
 * For inner product the rule is read as <p,c> <= alpha * <s,c> (alpha < 1
 * then relaxes pruning the way alpha > 1 does for distances).  On unit-norm
 * data both metrics rank identically (d^2 = 2 - 2<a,b>).
 *
 * The graph is an input shared by the search implementations under test; it
 * is not part of the search method.  Determinism independent of the thread
 * count comes from batch-synchronous insertion: points are inserted in a
 * seeded random order in batches whose sizes double up to a cap; inside a
 * batch every search sees the graph frozen at the start of the batch, each
 * node's new edge list is computed independently, and reverse edges are
 * applied per target in sorted source order.
 *
 * Vectors are float16; inner products accumulate in float32 in a fixed order.
 * Rows of the adjacency hold the valid neighbours first, then 0xFFFFFFFF.
 */
#include <immintrin.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>
#include <time.h>

#define SENT 0xFFFFFFFFu

/* vectors are float16 (IEEE binary16 bits); products accumulate in float32
 * over 16 fixed lanes, then a fixed reduction */
static inline float dotf(const uint16_t *a, const uint16_t *b, int n) {
  __m512 acc = _mm512_setzero_ps();
  int i = 0;
  for (; i + 16 <= n; i += 16) {
    __m512 x = _mm512_cvtph_ps(_mm256_loadu_si256((const __m256i *)(a + i)));
    __m512 y = _mm512_cvtph_ps(_mm256_loadu_si256((const __m256i *)(b + i)));
    acc = _mm512_fmadd_ps(x, y, acc);
  }
  float t = _mm512_reduce_add_ps(acc);
  for (; i < n; ++i) t += _cvtsh_ss(a[i]) * _cvtsh_ss(b[i]);
  return t;
}

typedef struct {
  float s;
  uint32_t id;
} cand_t;

/* Similarity used by search and pruning.  metric 0 (Euclidean): s(a,b) =
 * -||a-b||^2 computed as 2<a,b> - |a|^2 - |b|^2; metric 1: s(a,b) = <a,b>. */
typedef struct {
  const uint16_t *X;
  const float *nrm; /* squared norms (metric 0) */
  int dim, metric;
} space_t;

static inline float sim(const space_t *sp, const uint16_t *qa, float qn, uint32_t b) {
  float d = dotf(qa, sp->X + (size_t)b * sp->dim, sp->dim);
  if (sp->metric == 0) return 2.f * d - qn - sp->nrm[b];
  return d;
}

/* prune test: is c (similarity sc to the pruned node) made redundant by the
 * kept neighbour with similarity ssc to c? */
static inline int dominated(const space_t *sp, float sc, float ssc, float alpha) {
  if (sp->metric == 0) return alpha * alpha * (-ssc) <= -sc;
  return sc <= alpha * ssc;
}

/* total order: larger similarity first, then smaller id */
static inline int better(float as, uint32_t aid, float bs, uint32_t bid) {
  return as > bs || (as == bs && aid < bid);
}

static int cmp_cand(const void *a, const void *b) {
  const cand_t *x = (const cand_t *)a, *y = (const cand_t *)b;
  if (better(x->s, x->id, y->s, y->id)) return -1;
  if (better(y->s, y->id, x->s, x->id)) return 1;
  return 0;
}

typedef struct {
  /* visited set: open addressing with a generation stamp per slot */
  uint32_t *hkey, *hstamp;
  uint32_t hmask, stamp;
  /* beam */
  float *ls;
  uint32_t *lid;
  uint8_t *lexp;
  /* visited list with similarities */
  cand_t *vis;
  size_t nvis, cvis;
  /* scratch for pruning */
  cand_t *pool;
  size_t cpool;
  uint32_t *fresh;
} scratch_t;

static void scratch_init(scratch_t *w, int L, int R) {
  w->hmask = (1u << 17) - 1;
  w->hkey = (uint32_t *)calloc(w->hmask + 1, sizeof(uint32_t));
  w->hstamp = (uint32_t *)calloc(w->hmask + 1, sizeof(uint32_t));
  w->stamp = 0;
  w->ls = (float *)malloc(sizeof(float) * (L + 1));
  w->lid = (uint32_t *)malloc(sizeof(uint32_t) * (L + 1));
  w->lexp = (uint8_t *)malloc(L + 1);
  w->cvis = 4096;
  w->vis = (cand_t *)malloc(sizeof(cand_t) * w->cvis);
  w->cpool = 4096;
  w->pool = (cand_t *)malloc(sizeof(cand_t) * w->cpool);
  w->fresh = (uint32_t *)malloc(sizeof(uint32_t) * (R > 64 ? R : 64));
}

static void scratch_free(scratch_t *w) {
  free(w->hkey); free(w->hstamp); free(w->ls); free(w->lid); free(w->lexp);
  free(w->vis); free(w->pool); free(w->fresh);
}

static inline uint32_t hmix(uint32_t x) {
  x ^= x >> 16; x *= 0x7feb352dU; x ^= x >> 15; x *= 0x846ca68bU; x ^= x >> 16;
  return x;
}

/* returns 1 if id was newly inserted, 0 if already present */
static inline int visit(scratch_t *w, uint32_t id) {
  uint32_t h = hmix(id) & w->hmask;
  for (;;) {
    if (w->hstamp[h] != w->stamp) {
      w->hstamp[h] = w->stamp;
      w->hkey[h] = id;
      return 1;
    }
    if (w->hkey[h] == id) return 0;
    h = (h + 1) & w->hmask;
  }
}

static void vis_push(scratch_t *w, float s, uint32_t id) {
  if (w->nvis == w->cvis) {
    w->cvis *= 2;
    w->vis = (cand_t *)realloc(w->vis, sizeof(cand_t) * w->cvis);
  }
  w->vis[w->nvis].s = s;
  w->vis[w->nvis].id = id;
  w->nvis++;
}

/* best-first beam search with window L from the entry; fills w->vis */
static void greedy(scratch_t *w, const space_t *sp, const uint32_t *adj, int R,
                   uint32_t entry, const uint16_t *q, float qn, int L) {
  const uint16_t *X = sp->X;
  const int dim = sp->dim;
  w->stamp++;
  if (w->stamp == 0) { /* wrapped: clear stamps */
    memset(w->hstamp, 0, sizeof(uint32_t) * (w->hmask + 1));
    w->stamp = 1;
  }
  w->nvis = 0;
  int cnt = 0;
  visit(w, entry);
  float s0 = sim(sp, q, qn, entry);
  vis_push(w, s0, entry);
  w->ls[0] = s0; w->lid[0] = entry; w->lexp[0] = 0; cnt = 1;
  if ((uint64_t)w->nvis * 2 > w->hmask) return;
  for (;;) {
    int i = 0;
    while (i < cnt && w->lexp[i]) ++i;
    if (i == cnt) break;
    w->lexp[i] = 1;
    const uint32_t *row = adj + (size_t)w->lid[i] * R;
    int nf = 0;
    for (int r = 0; r < R; ++r) {
      uint32_t nb = row[r];
      if (nb == SENT) break;
      if (!visit(w, nb)) continue;
      w->fresh[nf++] = nb;
      __builtin_prefetch(X + (size_t)nb * dim);
    }
    for (int f = 0; f < nf; ++f) {
      uint32_t nb = w->fresh[f];
      float s = sim(sp, q, qn, nb);
      vis_push(w, s, nb);
      if (cnt == L && !better(s, nb, w->ls[cnt - 1], w->lid[cnt - 1])) continue;
      int pos = cnt < L ? cnt : L - 1;
      while (pos > 0 && better(s, nb, w->ls[pos - 1], w->lid[pos - 1])) {
        w->ls[pos] = w->ls[pos - 1]; w->lid[pos] = w->lid[pos - 1];
        w->lexp[pos] = w->lexp[pos - 1];
        --pos;
      }
      w->ls[pos] = s; w->lid[pos] = nb; w->lexp[pos] = 0;
      if (cnt < L) ++cnt;
    }
    /* keep the visited table at most half full: 2^16 visits is far beyond
     * what a window of a few hundred needs */
    if ((uint64_t)w->nvis * 2 > w->hmask) break;
  }
}

/* Keep at most R of the candidates in w->pool[0..np) (similarities to p
 * already filled in) using the diversity rule; writes a padded row. */
static void prune(scratch_t *w, size_t np, const space_t *sp, uint32_t p,
                  float alpha, int R, int maxc, uint32_t *out) {
  const uint16_t *X = sp->X;
  const int dim = sp->dim;
  qsort(w->pool, np, sizeof(cand_t), cmp_cand);
  int nsel = 0;
  size_t seen = 0;
  uint32_t last = SENT;
  for (size_t i = 0; i < np && nsel < R; ++i) {
    uint32_t c = w->pool[i].id;
    if (c == p || c == last) continue; /* self or duplicate (adjacent after sort) */
    last = c;
    if ((int)seen >= maxc) break;
    ++seen;
    const uint16_t *xc = X + (size_t)c * dim;
    const float nc = sp->metric == 0 ? sp->nrm[c] : 0.f;
    int keep = 1;
    for (int j = 0; j < nsel; ++j) {
      if (dominated(sp, w->pool[i].s, sim(sp, xc, nc, out[j]), alpha)) {
        keep = 0;
        break;
      }
    }
    if (keep) out[nsel++] = c;
  }
  for (int j = nsel; j < R; ++j) out[j] = SENT;
}

static void pool_reserve(scratch_t *w, size_t n) {
  if (n > w->cpool) {
    while (w->cpool < n) w->cpool *= 2;
    w->pool = (cand_t *)realloc(w->pool, sizeof(cand_t) * w->cpool);
  }
}

static uint64_t splitmix(uint64_t *s) {
  uint64_t z = (*s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

typedef struct {
  uint32_t dst, src;
} edge_t;

static int cmp_edge(const void *a, const void *b) {
  const edge_t *x = (const edge_t *)a, *y = (const edge_t *)b;
  if (x->dst != y->dst) return x->dst < y->dst ? -1 : 1;
  if (x->src != y->src) return x->src < y->src ? -1 : 1;
  return 0;
}

/* entry = vector closest (L2) to the mean; ties to the lower id */
uint32_t lvg_medoid(const uint16_t *X, int64_t n, int32_t dim) {
  const int64_t CH = 4096;
  int64_t nch = (n + CH - 1) / CH;
  double *part = (double *)calloc((size_t)nch * dim, sizeof(double));
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nch; ++c) {
    double *acc = part + (size_t)c * dim;
    for (int64_t i = c * CH; i < n && i < (c + 1) * CH; ++i)
      for (int j = 0; j < dim; ++j) acc[j] += _cvtsh_ss(X[(size_t)i * dim + j]);
  }
  double *mean = (double *)calloc(dim, sizeof(double));
  for (int64_t c = 0; c < nch; ++c)
    for (int j = 0; j < dim; ++j) mean[j] += part[(size_t)c * dim + j];
  for (int j = 0; j < dim; ++j) mean[j] /= (double)n;
  double *bestd = (double *)malloc(sizeof(double) * nch);
  int64_t *besti = (int64_t *)malloc(sizeof(int64_t) * nch);
#pragma omp parallel for schedule(static)
  for (int64_t c = 0; c < nch; ++c) {
    double bd = INFINITY;
    int64_t bi = -1;
    for (int64_t i = c * CH; i < n && i < (c + 1) * CH; ++i) {
      double s = 0.0;
      for (int j = 0; j < dim; ++j) {
        double t = (double)_cvtsh_ss(X[(size_t)i * dim + j]) - mean[j];
        s += t * t;
      }
      if (s < bd) { bd = s; bi = i; }
    }
    bestd[c] = bd; besti[c] = bi;
  }
  double bd = INFINITY;
  int64_t bi = 0;
  for (int64_t c = 0; c < nch; ++c)
    if (bestd[c] < bd) { bd = bestd[c]; bi = besti[c]; }
  free(part); free(mean); free(bestd); free(besti);
  return (uint32_t)bi;
}

/*
 * Build the graph.  X: float16 bits [n][dim] row-major (host).  adj: [n][R] out.
 * alphas[npasses]: pruning factor per pass (first pass usually 1.0).
 * Returns the entry id, or -1 on bad arguments.
 */
int64_t lvg_build(const uint16_t *X, int64_t n, int32_t dim, int32_t metric, int32_t R,
                  int32_t L, int32_t maxc, const float *alphas, int32_t npasses,
                  double batch_frac, uint64_t seed, int32_t nthreads, uint32_t *adj) {
  if (!X || !adj || n < 1 || n >= (int64_t)SENT || dim < 1 || R < 1 || L < 1 ||
      npasses < 1 || !alphas || (metric != 0 && metric != 1))
    return -1;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  for (size_t i = 0; i < (size_t)n * R; ++i) adj[i] = SENT;
  if (n == 1) return 0;
  uint32_t entry = lvg_medoid(X, n, dim);
  float *nrm = (float *)malloc(sizeof(float) * n);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i)
    nrm[i] = dotf(X + (size_t)i * dim, X + (size_t)i * dim, dim);
  space_t space = {X, nrm, dim, metric};
  const space_t *sp = &space;

  uint32_t *perm = (uint32_t *)malloc(sizeof(uint32_t) * n);
  for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
  uint64_t st = seed;
  for (int64_t i = n - 1; i > 0; --i) {
    int64_t j = (int64_t)(splitmix(&st) % (uint64_t)(i + 1));
    uint32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
  int64_t maxb = (int64_t)(batch_frac * (double)n);
  if (maxb < 1) maxb = 1;
  uint32_t *newN = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)maxb * R);
  edge_t *E = (edge_t *)malloc(sizeof(edge_t) * (size_t)maxb * R);
  int64_t *gstart = (int64_t *)malloc(sizeof(int64_t) * ((size_t)maxb * R + 1));

  int nt = omp_get_max_threads();
  scratch_t *ws = (scratch_t *)malloc(sizeof(scratch_t) * nt);
  for (int t = 0; t < nt; ++t) scratch_init(&ws[t], L, R);

  double last_report = 0.0;
  {
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    last_report = ts.tv_sec + 1e-9 * ts.tv_nsec;
  }
  for (int pass = 0; pass < npasses; ++pass) {
    float alpha = alphas[pass];
    int64_t start = 0, bs = pass == 0 ? 1 : maxb;
    while (start < n) {
      int64_t end = start + bs < n ? start + bs : n;
      int64_t B = end - start;
#pragma omp parallel for schedule(dynamic, 8)
      for (int64_t i = 0; i < B; ++i) {
        scratch_t *w = &ws[omp_get_thread_num()];
        uint32_t p = perm[start + i];
        const uint16_t *xp = X + (size_t)p * dim;
        greedy(w, sp, adj, R, entry, xp, nrm[p], L);
        pool_reserve(w, w->nvis + R);
        size_t np = 0;
        for (size_t v = 0; v < w->nvis; ++v) w->pool[np++] = w->vis[v];
        const uint32_t *row = adj + (size_t)p * R;
        for (int r = 0; r < R && row[r] != SENT; ++r) {
          w->pool[np].id = row[r];
          w->pool[np].s = sim(sp, xp, nrm[p], row[r]);
          ++np;
        }
        prune(w, np, sp, p, alpha, R, maxc, newN + (size_t)i * R);
      }
      size_t ne = 0;
      for (int64_t i = 0; i < B; ++i) {
        uint32_t p = perm[start + i];
        memcpy(adj + (size_t)p * R, newN + (size_t)i * R, sizeof(uint32_t) * R);
        for (int r = 0; r < R; ++r) {
          uint32_t j = newN[(size_t)i * R + r];
          if (j == SENT) break;
          E[ne].dst = j; E[ne].src = p; ++ne;
        }
      }
      qsort(E, ne, sizeof(edge_t), cmp_edge);
      int64_t ng = 0;
      for (size_t e = 0; e < ne; ++e)
        if (e == 0 || E[e].dst != E[e - 1].dst) gstart[ng++] = (int64_t)e;
      gstart[ng] = (int64_t)ne;
#pragma omp parallel for schedule(dynamic, 16)
      for (int64_t g = 0; g < ng; ++g) {
        scratch_t *w = &ws[omp_get_thread_num()];
        uint32_t j = E[gstart[g]].dst;
        uint32_t *row = adj + (size_t)j * R;
        int deg = 0;
        while (deg < R && row[deg] != SENT) ++deg;
        int64_t cnt = gstart[g + 1] - gstart[g];
        pool_reserve(w, (size_t)deg + cnt);
        /* union of the current row and new sources, preserving row order */
        size_t np = 0;
        for (int r = 0; r < deg; ++r) { w->pool[np].id = row[r]; ++np; }
        for (int64_t e = gstart[g]; e < gstart[g + 1]; ++e) {
          uint32_t s = E[e].src;
          int dup = 0;
          for (int r = 0; r < deg; ++r)
            if (row[r] == s) { dup = 1; break; }
          if (!dup && s != j) { w->pool[np].id = s; ++np; }
        }
        if ((int64_t)np <= R) {
          for (size_t r = 0; r < np; ++r) row[r] = w->pool[r].id;
          for (int r = (int)np; r < R; ++r) row[r] = SENT;
        } else {
          const uint16_t *xj = X + (size_t)j * dim;
          for (size_t r = 0; r < np; ++r)
            w->pool[r].s = sim(sp, xj, nrm[j], w->pool[r].id);
          prune(w, np, sp, j, alpha, R, maxc, w->fresh);
          memcpy(row, w->fresh, sizeof(uint32_t) * R);
        }
      }
      start = end;
      if (n >= 200000) { /* progress on long builds, about every 20 s */
        struct timespec ts;
        clock_gettime(CLOCK_MONOTONIC, &ts);
        double now = ts.tv_sec + 1e-9 * ts.tv_nsec;
        if (now - last_report > 20.0) {
          fprintf(stderr, "graph build: pass %d/%d, %lld of %lld inserted\n", pass + 1, npasses,
                  (long long)start, (long long)n);
          fflush(stderr);
          last_report = now;
        }
      }
      bs = bs * 2 < maxb ? bs * 2 : maxb;
    }
  }
  for (int t = 0; t < nt; ++t) scratch_free(&ws[t]);
  free(ws); free(perm); free(newN); free(E); free(gstart); free(nrm);
  return (int64_t)entry;
}

/* mark everything reachable from s that is not marked yet; returns the count */
static int64_t bfs_mark(const uint32_t *adj, int64_t n, int32_t R, uint32_t s, uint8_t *mark,
                        uint32_t *q) {
  int64_t h = 0, t = 0;
  if (mark[s]) return 0;
  mark[s] = 1;
  q[t++] = s;
  while (h < t) {
    uint32_t u = q[h++];
    for (int r = 0; r < R; ++r) {
      uint32_t v = adj[(size_t)u * R + r];
      if (v == SENT) break;
      if (v < (uint64_t)n && !mark[v]) { mark[v] = 1; q[t++] = v; }
    }
  }
  return t;
}

/*
 * Make every node reachable from the entry.  Unreachable nodes are visited in
 * increasing id; for each one still unreachable, a greedy search from the
 * entry (which only walks reachable nodes) ranks reachable candidates, and
 * the most similar one with a free slot gets an edge to it (the most similar
 * one overall has its last edge replaced if none has a free slot).  Repeats
 * until a full BFS reaches everything (bounded).  Returns the number of
 * edges added.
 */
int64_t lvg_repair(const uint16_t *X, int64_t n, int32_t dim, int32_t metric, int32_t R, int32_t L,
                   uint32_t entry, uint32_t *adj) {
  uint8_t *mark = (uint8_t *)malloc((size_t)n);
  uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * n);
  float *nrm = (float *)malloc(sizeof(float) * n);
  for (int64_t i = 0; i < n; ++i) nrm[i] = dotf(X + (size_t)i * dim, X + (size_t)i * dim, dim);
  space_t space = {X, nrm, dim, metric};
  scratch_t w;
  scratch_init(&w, L, R);
  int64_t added = 0;
  for (int round = 0; round < 8; ++round) {
    memset(mark, 0, (size_t)n);
    if (bfs_mark(adj, n, R, entry, mark, q) == n) break;
    for (int64_t u = 0; u < n; ++u) {
      if (mark[u]) continue;
      const uint16_t *xu = X + (size_t)u * dim;
      greedy(&w, &space, adj, R, entry, xu, nrm[u], L);
      pool_reserve(&w, w.nvis);
      for (size_t v = 0; v < w.nvis; ++v) w.pool[v] = w.vis[v];
      qsort(w.pool, w.nvis, sizeof(cand_t), cmp_cand);
      int64_t pick = -1;
      for (size_t v = 0; v < w.nvis && pick < 0; ++v) {
        uint32_t c = w.pool[v].id;
        if (c == (uint32_t)u || !mark[c]) continue;
        if (adj[(size_t)c * R + R - 1] == SENT) pick = c;
      }
      if (pick < 0) {
        for (size_t v = 0; v < w.nvis && pick < 0; ++v)
          if (w.pool[v].id != (uint32_t)u && mark[w.pool[v].id]) pick = w.pool[v].id;
        if (pick < 0) pick = entry;
        adj[(size_t)pick * R + R - 1] = (uint32_t)u;
      } else {
        uint32_t *row = adj + (size_t)pick * R;
        int deg = 0;
        while (deg < R && row[deg] != SENT) ++deg;
        row[deg] = (uint32_t)u;
      }
      ++added;
      bfs_mark(adj, n, R, (uint32_t)u, mark, q);
    }
  }
  scratch_free(&w);
  free(mark); free(q); free(nrm);
  return added;
}

/* number of nodes reachable from entry (BFS); marks reach[i] = 1 */
int64_t lvg_reachable(const uint32_t *adj, int64_t n, int32_t R, uint32_t entry,
                      uint8_t *reach) {
  memset(reach, 0, (size_t)n);
  uint32_t *q = (uint32_t *)malloc(sizeof(uint32_t) * n);
  int64_t h = 0, t = 0;
  q[t++] = entry;
  reach[entry] = 1;
  while (h < t) {
    uint32_t u = q[h++];
    for (int r = 0; r < R; ++r) {
      uint32_t v = adj[(size_t)u * R + r];
      if (v == SENT) break;
      if (v < (uint64_t)n && !reach[v]) { reach[v] = 1; q[t++] = v; }
    }
  }
  free(q);
  return t;
}
