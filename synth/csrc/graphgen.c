/*
 * Seeded synthetic graph generators (directed Chung-Lu, R-MAT) and the
 * canonical CSR writer.
 *
 * These produce the inputs that both the CPU oracle and the GPU library
 * read. Nothing here performs any step of the PageRank method: no prefix
 * sums of weights, no walks, no counting. Every random value is a pure
 * function of (seed, stream, index) through a splitmix64-style hash, so the
 * output does not depend on the thread count.
 *
 * Canonical CSR: edges sorted by (src, dst, w); multi-edges and self-loops
 * are kept.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---- counter-based input hash (Steele et al., splitmix64 finalizer) ---- */
static inline uint64_t sm_mix(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}
static inline uint64_t gg_hash(uint64_t seed, uint64_t stream, uint64_t idx) {
  uint64_t z = sm_mix(seed + 0x9E3779B97F4A7C15ULL * (stream + 1));
  return sm_mix(z ^ (idx * 0xD6E8FEB86659FD93ULL + 0x632BE59BD9B4E019ULL));
}
static inline double gg_unit(uint64_t h) { /* uniform in [0, 1) */
  return (double)(h >> 11) * (1.0 / 9007199254740992.0);
}
/* first index i in cdf[0..len) with cdf[i] > u; cdf is nondecreasing and
 * cdf[len-1] is treated as +inf so the result is always < len. */
static inline uint32_t gg_search(const double* cdf, uint32_t len, double u) {
  uint32_t lo = 0, hi = len - 1;
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (cdf[mid] > u) hi = mid; else lo = mid + 1;
  }
  return lo;
}

typedef struct {
  int kind; /* 0 chung-lu, 1 rmat */
  uint64_t seed;
  uint64_t e0, e1;
  /* chung-lu */
  const double* cdf_out; const double* cdf_in; uint32_t n;
  /* rmat */
  uint32_t scale; uint32_t ta, tab, tabc; const uint32_t* perm;
  /* weights: table==NULL -> uniform in [1, wmax]; else cdf over [1, wlen] */
  const double* wcdf; uint32_t wlen; uint32_t wmax;
  uint32_t* src; uint32_t* dst; uint32_t* w;
} gen_job;

static void* gen_worker(void* arg) {
  gen_job* j = (gen_job*)arg;
  for (uint64_t e = j->e0; e < j->e1; ++e) {
    uint32_t s, d;
    if (j->kind == 0) {
      s = gg_search(j->cdf_out, j->n, gg_unit(gg_hash(j->seed, 1, e)));
      d = gg_search(j->cdf_in, j->n, gg_unit(gg_hash(j->seed, 2, e)));
    } else {
      s = 0; d = 0;
      for (uint32_t lvl = 0; lvl < j->scale; lvl += 2) {
        uint64_t h = gg_hash(j->seed, 3 + lvl / 2, e);
        for (uint32_t k = 0; k < 2 && lvl + k < j->scale; ++k) {
          uint32_t r = (uint32_t)(h >> (32 * k));
          uint32_t bit = j->scale - 1 - (lvl + k);
          if (r < j->ta) { /* top-left */ }
          else if (r < j->tab) d |= 1u << bit;
          else if (r < j->tabc) s |= 1u << bit;
          else { s |= 1u << bit; d |= 1u << bit; }
        }
      }
      if (j->perm) { s = j->perm[s]; d = j->perm[d]; }
    }
    uint64_t hw = gg_hash(j->seed, 64, e);
    uint32_t wt;
    if (j->wcdf) wt = 1 + gg_search(j->wcdf, j->wlen, gg_unit(hw));
    else wt = 1 + (uint32_t)(((hw >> 32) * (uint64_t)j->wmax) >> 32);
    j->src[e] = s; j->dst[e] = d; j->w[e] = wt;
  }
  return NULL;
}

static void run_jobs(gen_job* proto, uint64_t m, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  pthread_t th[64]; gen_job jobs[64];
  for (int t = 0; t < nthreads; ++t) {
    jobs[t] = *proto;
    jobs[t].e0 = m * (uint64_t)t / (uint64_t)nthreads;
    jobs[t].e1 = m * (uint64_t)(t + 1) / (uint64_t)nthreads;
    pthread_create(&th[t], NULL, gen_worker, &jobs[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
}

/* Seeded Fisher-Yates permutation of [0, n). */
void gg_permutation(uint32_t n, uint64_t seed, uint32_t* perm) {
  for (uint32_t i = 0; i < n; ++i) perm[i] = i;
  for (uint32_t i = n; i > 1; --i) {
    uint64_t h = gg_hash(seed, 99, i);
    uint32_t k = (uint32_t)(((h >> 32) * (uint64_t)i) >> 32); /* in [0, i) */
    uint32_t t = perm[i - 1]; perm[i - 1] = perm[k]; perm[k] = t;
  }
}

/* Directed Chung-Lu edge list: m independent (src, dst) draws from the
 * given out/in cumulative distributions over n nodes. */
void gg_chung_lu_edges(uint32_t n, uint64_t m, const double* cdf_out,
                       const double* cdf_in, const double* wcdf, uint32_t wlen,
                       uint32_t wmax, uint64_t seed, int nthreads,
                       uint32_t* src, uint32_t* dst, uint32_t* w) {
  gen_job j; memset(&j, 0, sizeof j);
  j.kind = 0; j.seed = seed; j.n = n; j.cdf_out = cdf_out; j.cdf_in = cdf_in;
  j.wcdf = wcdf; j.wlen = wlen; j.wmax = wmax; j.src = src; j.dst = dst; j.w = w;
  run_jobs(&j, m, nthreads);
}

/* R-MAT edge list (Chakrabarti et al.): per level one of four quadrants with
 * probabilities a, b, c, d given as 32-bit thresholds; perm (optional)
 * relabels vertices. */
void gg_rmat_edges(uint32_t scale, uint64_t m, uint32_t ta, uint32_t tab,
                   uint32_t tabc, const uint32_t* perm, const double* wcdf,
                   uint32_t wlen, uint32_t wmax, uint64_t seed, int nthreads,
                   uint32_t* src, uint32_t* dst, uint32_t* w) {
  gen_job j; memset(&j, 0, sizeof j);
  j.kind = 1; j.seed = seed; j.scale = scale; j.ta = ta; j.tab = tab; j.tabc = tabc;
  j.perm = perm; j.wcdf = wcdf; j.wlen = wlen; j.wmax = wmax;
  j.src = src; j.dst = dst; j.w = w;
  run_jobs(&j, m, nthreads);
}

/* ---- canonical CSR: counting sort by src, then sort each row by (dst, w) ---- */
static int cmp_u64(const void* a, const void* b) {
  uint64_t x = *(const uint64_t*)a, y = *(const uint64_t*)b;
  return (x > y) - (x < y);
}

typedef struct {
  uint32_t r0, r1;
  const uint64_t* off; uint64_t* key; uint32_t* col; uint32_t* w;
} row_job;

static void* row_worker(void* arg) {
  row_job* j = (row_job*)arg;
  for (uint32_t r = j->r0; r < j->r1; ++r) {
    uint64_t a = j->off[r], b = j->off[r + 1];
    if (b - a > 1) qsort(j->key + a, (size_t)(b - a), sizeof(uint64_t), cmp_u64);
    for (uint64_t e = a; e < b; ++e) {
      j->col[e] = (uint32_t)(j->key[e] >> 32);
      j->w[e] = (uint32_t)(j->key[e] & 0xFFFFFFFFu);
    }
  }
  return NULL;
}

/* Builds row_offsets[n+1], col[m], w_out[m] from an edge list.
 * Returns 0 on success, -1 on allocation failure or a src/dst >= n. */
int gg_build_csr(uint32_t n, uint64_t m, const uint32_t* src,
                 const uint32_t* dst, const uint32_t* w, int nthreads,
                 uint64_t* off, uint32_t* col, uint32_t* w_out) {
  for (uint64_t e = 0; e < m; ++e)
    if (src[e] >= n || dst[e] >= n) return -1;
  memset(off, 0, sizeof(uint64_t) * ((size_t)n + 1));
  for (uint64_t e = 0; e < m; ++e) off[src[e] + 1]++;
  for (uint32_t v = 0; v < n; ++v) off[v + 1] += off[v];
  uint64_t* cur = (uint64_t*)malloc(sizeof(uint64_t) * ((size_t)n + 1));
  uint64_t* key = (uint64_t*)malloc(sizeof(uint64_t) * (m ? m : 1));
  if (!cur || !key) { free(cur); free(key); return -1; }
  memcpy(cur, off, sizeof(uint64_t) * ((size_t)n + 1));
  for (uint64_t e = 0; e < m; ++e)
    key[cur[src[e]]++] = ((uint64_t)dst[e] << 32) | w[e];
  free(cur);
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  pthread_t th[64]; row_job jobs[64];
  /* split rows so each thread gets about m / nthreads edges */
  uint32_t r = 0;
  for (int t = 0; t < nthreads; ++t) {
    uint64_t target = m * (uint64_t)(t + 1) / (uint64_t)nthreads;
    uint32_t r1 = r;
    if (t == nthreads - 1) r1 = n;
    else while (r1 < n && off[r1 + 1] <= target) ++r1;
    jobs[t].r0 = r; jobs[t].r1 = r1; jobs[t].off = off; jobs[t].key = key;
    jobs[t].col = col; jobs[t].w = w_out;
    pthread_create(&th[t], NULL, row_worker, &jobs[t]);
    r = r1;
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  free(key);
  return 0;
}
