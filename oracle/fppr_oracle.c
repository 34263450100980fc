/*
 * CPU oracle (test infrastructure only; see oracle.h for the definitions it
 * follows and for who may call it).
 *
 * Deliberately plain: one walk at a time, one binary search per pick, qsort
 * for counting. Threads split the source list; every output slot belongs to
 * one source, so results do not depend on the thread count.
 */
#include "oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

struct or_graph {
  uint32_t n;
  uint64_t m;
  const uint64_t* off; /* row_offsets[n+1] */
  const uint32_t* col; /* col[m] */
  uint64_t* P;         /* inclusive prefix of w within each row */
};

struct or_pool {
  uint32_t S, L, K, T;
  uint64_t seed;
  uint64_t n_small;
  uint32_t* small_rank; /* [n], UINT32_MAX when not small */
  uint64_t* entry;      /* [n_small * K] */
};

/* ---------------------------------------------------------------------- */
/* Philox4x32-10: ten rounds of the Philox S-box on a 128-bit counter with a
 * 64-bit key bumped by the Weyl constants between rounds (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11). */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * c0;
    uint64_t p1 = (uint64_t)M1 * c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, uint32_t a, uint32_t b, uint32_t c, uint32_t d, uint32_t x[4]) {
  uint32_t ctr[4] = {a, b, c, d};
  uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
  or_philox4x32_10(ctr, key, x);
}

/* Coin of Algorithm 2 ("terminate if q <= alpha") on 32-bit integers:
 * P(x2 < T) = T / 2^32. */
uint32_t or_alpha_threshold(double alpha) {
  if (!(alpha > 0.0 && alpha < 1.0)) return 0;
  double t = floor(alpha * 4294967296.0 + 0.5);
  if (t < 1.0) t = 1.0;
  if (t > 4294967295.0) t = 4294967295.0;
  return (uint32_t)t;
}

/* ---------------------------------------------------------------------- */
/* Routing probability r(s,t) = w(s,t)/W (Sec. 2.1) realised on integers:
 * X uniform on [0, W) from 64 random bits, then the first prefix above X. */
static uint64_t scaled_draw(uint32_t x0, uint32_t x1, uint64_t W) {
  unsigned __int128 r = ((unsigned __int128)(((uint64_t)x1 << 32) | x0)) * W;
  return (uint64_t)(r >> 64);
}

/* First index j in [0, deg) with P[j] > X (P strictly increasing, P[deg-1] > X).
 * When `lines` is given, adds the number of distinct 64-byte lines of the
 * prefix array that the probes touch (row starts at element row_base). */
static uint32_t upper_bound(const uint64_t* P, uint32_t deg, uint64_t X, uint64_t row_base,
                            uint64_t* lines) {
  uint32_t lo = 0, hi = deg - 1;
  uint64_t seen[64];
  int nseen = 0;
  while (lo < hi) {
    uint32_t mid = lo + (hi - lo) / 2;
    if (lines) {
      uint64_t line = (row_base + mid) / 8;
      int dup = 0;
      for (int i = 0; i < nseen; ++i) dup |= (seen[i] == line);
      if (!dup) { seen[nseen++] = line; ++*lines; }
    }
    if (P[mid] > X) hi = mid; else lo = mid + 1;
  }
  return lo;
}

uint32_t or_pick(const uint64_t* P, uint32_t deg, uint32_t x0, uint32_t x1) {
  uint64_t X = scaled_draw(x0, x1, P[deg - 1]);
  return upper_bound(P, deg, X, 0, NULL);
}

static uint32_t ceil_log2(uint64_t d) {
  uint32_t c = 0;
  while (((uint64_t)1 << c) < d) ++c;
  return c;
}

/* ---------------------------------------------------------------------- */
or_graph* or_graph_new(uint32_t n, uint64_t m, const uint64_t* row_offsets, const uint32_t* col,
                       const uint32_t* w) {
  if (n == 0 || !row_offsets) return NULL;
  if (row_offsets[0] != 0 || row_offsets[n] != m) return NULL;
  for (uint32_t v = 0; v < n; ++v)
    if (row_offsets[v + 1] < row_offsets[v]) return NULL;
  for (uint64_t e = 0; e < m; ++e)
    if (col[e] >= n || w[e] == 0) return NULL;
  or_graph* g = (or_graph*)calloc(1, sizeof(or_graph));
  g->n = n;
  g->m = m;
  g->off = row_offsets;
  g->col = col;
  g->P = (uint64_t*)malloc(sizeof(uint64_t) * (m ? m : 1));
  for (uint32_t v = 0; v < n; ++v) {
    uint64_t acc = 0;
    for (uint64_t e = row_offsets[v]; e < row_offsets[v + 1]; ++e) {
      acc += w[e];
      g->P[e] = acc;
    }
  }
  return g;
}

void or_graph_free(or_graph* g) {
  if (!g) return;
  free(g->P);
  free(g);
}

void or_graph_prefix(const or_graph* g, uint64_t* out) { memcpy(out, g->P, sizeof(uint64_t) * g->m); }

static inline uint32_t degree(const or_graph* g, uint32_t v) {
  return (uint32_t)(g->off[v + 1] - g->off[v]);
}

/* One plain pick at a node with out-neighbours. */
static uint32_t plain_next(const or_graph* g, uint32_t v, uint32_t x0, uint32_t x1, uint64_t* lines) {
  uint64_t off = g->off[v];
  uint32_t deg = degree(g, v);
  const uint64_t* P = g->P + off;
  uint64_t X = scaled_draw(x0, x1, P[deg - 1]);
  uint32_t j = upper_bound(P, deg, X, off, lines);
  return g->col[off + j];
}

/* ---------------------------------------------------------------------- */
/* Short walks for small nodes (Sec. 4.2, "big moves"): the paper expands the
 * exact multi-step distribution of each small node; here each small node
 * keeps K sampled walks of at most L plain steps, each carrying the same
 * termination mark as a big move. A pool walk stops on its coin (mark
 * terminated), after L steps (mark active), or on arriving at a node without
 * out-neighbours (mark active: the restart to the main walk's head happens on
 * the main walk's next move). */
typedef struct {
  const or_graph* g;
  or_pool* p;
  uint32_t v0, v1;
} pool_job;

static void* pool_worker(void* arg) {
  pool_job* jb = (pool_job*)arg;
  const or_graph* g = jb->g;
  or_pool* p = jb->p;
  for (uint32_t v = jb->v0; v < jb->v1; ++v) {
    uint32_t rank = p->small_rank[v];
    if (rank == UINT32_MAX) continue;
    for (uint32_t j = 0; j < p->K; ++j) {
      uint32_t cur = v, steps = 0, mark = 0;
      for (uint32_t t = 0; t < p->L; ++t) {
        uint32_t x[4];
        draw(p->seed, j, t, v, 1, x);
        cur = plain_next(g, cur, x[0], x[1], NULL);
        steps += 1;
        if (x[2] < p->T) { mark = OR_POOL_TERM; break; }
        if (degree(g, cur) == 0) break;
      }
      p->entry[(uint64_t)rank * p->K + j] =
          (uint64_t)cur | ((uint64_t)steps << 32) | ((uint64_t)mark << 48);
    }
  }
  return NULL;
}

static int clamp_threads(int t) { return t < 1 ? 1 : (t > 256 ? 256 : t); }

or_pool* or_pool_new(const or_graph* g, uint32_t S, uint32_t L, uint32_t K, uint32_t T, uint64_t seed,
                     int nthreads) {
  if (!g || L == 0 || K == 0 || (K & (K - 1)) || T == 0 || S == 0) return NULL;
  or_pool* p = (or_pool*)calloc(1, sizeof(or_pool));
  p->S = S; p->L = L; p->K = K; p->T = T; p->seed = seed;
  p->small_rank = (uint32_t*)malloc(sizeof(uint32_t) * g->n);
  uint64_t ns = 0;
  for (uint32_t v = 0; v < g->n; ++v) {
    uint32_t d = degree(g, v);
    p->small_rank[v] = (d >= 1 && d <= S) ? (uint32_t)ns++ : UINT32_MAX;
  }
  p->n_small = ns;
  p->entry = (uint64_t*)malloc(sizeof(uint64_t) * (ns * K ? ns * K : 1));
  nthreads = clamp_threads(nthreads);
  pthread_t th[256];
  pool_job jobs[256];
  for (int t = 0; t < nthreads; ++t) {
    jobs[t].g = g; jobs[t].p = p;
    jobs[t].v0 = (uint32_t)((uint64_t)g->n * t / nthreads);
    jobs[t].v1 = (uint32_t)((uint64_t)g->n * (t + 1) / nthreads);
    pthread_create(&th[t], NULL, pool_worker, &jobs[t]);
  }
  for (int t = 0; t < nthreads; ++t) pthread_join(th[t], NULL);
  return p;
}

void or_pool_free(or_pool* p) {
  if (!p) return;
  free(p->small_rank);
  free(p->entry);
  free(p);
}

uint64_t or_pool_small_count(const or_pool* p) { return p->n_small; }

void or_pool_entries(const or_pool* p, uint64_t* out) {
  memcpy(out, p->entry, sizeof(uint64_t) * p->n_small * p->K);
}

/* ---------------------------------------------------------------------- */
/* One walk from source s (Sec. 2.1 and Algorithm 2): every move first picks
 * the next node, then tosses the termination coin, so a walk has length at
 * least one. A node without out-neighbours sends the walk back to its head.
 * With a pool, a move at a small node takes one pool entry instead (Sec. 4.2:
 * a terminated big move ends the walk, an active one continues from its end). */
static uint32_t walk(const or_graph* g, const or_pool* pool, uint32_t T, uint64_t seed, uint32_t s,
                     uint32_t i, uint32_t* len_out, or_stats* st) {
  uint32_t tail = s, len = 0, m = 0;
  for (;;) {
    uint32_t x[4];
    draw(seed, i, m, s, 0, x);
    uint32_t deg = degree(g, tail);
    int stop;
    if (deg == 0) {
      tail = s;
      len += 1;
      stop = x[2] < T;
      st->dangling_moves++;
      st->lines += 1;
    } else if (pool && deg <= pool->S) {
      uint32_t slot = (uint32_t)(((uint64_t)x[0] * pool->K) >> 32);
      uint64_t e = pool->entry[(uint64_t)pool->small_rank[tail] * pool->K + slot];
      tail = (uint32_t)e;
      len += (uint32_t)((e >> 32) & 0xFFFF);
      stop = ((e >> 48) & 1) == OR_POOL_TERM;
      st->stitched_moves++;
      st->lines += 2;
    } else {
      uint64_t nl = 0;
      st->probe_log_sum += ceil_log2(deg);
      tail = plain_next(g, tail, x[0], x[1], &nl);
      len += 1;
      stop = x[2] < T;
      st->plain_moves++;
      st->lines += 2 + nl; /* record + col + distinct prefix lines probed */
    }
    m += 1;
    if (!stop && m == OR_MOVE_CAP) {
      st->capped++;
      stop = 1;
    }
    if (stop) break;
  }
  st->moves += m;
  st->steps += len;
  st->walks += 1;
  *len_out = len;
  return tail;
}

/* ---------------------------------------------------------------------- */
/* Aggregation: pi_hat(s,t) = (#walks from s ending at t) / omega, kept only
 * for endpoints some walk reached (Algorithm 2, final phase; Sec. 1). */
static uint64_t fmix64(uint64_t k) { /* MurmurHash3 64-bit finalizer */
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}

uint64_t or_digest_term(uint32_t s, uint32_t t, uint32_t count) {
  uint64_t h = fmix64(((uint64_t)s << 32) | t);
  return fmix64(h ^ ((uint64_t)count * 0x9E3779B97F4A7C15ULL));
}

static int cmp_u32(const void* a, const void* b) {
  uint32_t x = *(const uint32_t*)a, y = *(const uint32_t*)b;
  return (x > y) - (x < y);
}

/* ranking order: count descending, then node id ascending */
static int cmp_rank(const void* a, const void* b) {
  const uint32_t* x = (const uint32_t*)a;
  const uint32_t* y = (const uint32_t*)b;
  if (x[1] != y[1]) return x[1] > y[1] ? -1 : 1;
  return (x[0] > y[0]) - (x[0] < y[0]);
}

typedef struct {
  const or_graph* g;
  const or_pool* pool;
  uint32_t T, R, k;
  uint64_t seed;
  const uint32_t* sources;
  uint64_t n_src;
  uint32_t *n_distinct, *counts, *topk, *endpoints, *lengths;
  uint64_t* digest;
  uint64_t* next; /* shared block counter */
  or_stats st;
} run_job;

#define OR_BLOCK 16

static void* run_worker(void* arg) {
  run_job* jb = (run_job*)arg;
  uint32_t R = jb->R;
  uint32_t* ep = (uint32_t*)malloc(sizeof(uint32_t) * (R ? R : 1));
  uint32_t* runs = (uint32_t*)malloc(sizeof(uint32_t) * 2 * (R ? R : 1));
  for (;;) {
    uint64_t b = __atomic_fetch_add(jb->next, 1, __ATOMIC_RELAXED);
    uint64_t s0 = b * OR_BLOCK;
    if (s0 >= jb->n_src) break;
    uint64_t s1 = s0 + OR_BLOCK < jb->n_src ? s0 + OR_BLOCK : jb->n_src;
    for (uint64_t si = s0; si < s1; ++si) {
      uint32_t s = jb->sources ? jb->sources[si] : (uint32_t)si;
      for (uint32_t i = 0; i < R; ++i) {
        uint32_t len;
        ep[i] = walk(jb->g, jb->pool, jb->T, jb->seed, s, i, &len, &jb->st);
        if (jb->endpoints) jb->endpoints[si * R + i] = ep[i];
        if (jb->lengths) jb->lengths[si * R + i] = len;
      }
      qsort(ep, R, sizeof(uint32_t), cmp_u32);
      uint32_t nd = 0;
      for (uint32_t i = 0; i < R; ++i) {
        if (i == 0 || ep[i] != ep[i - 1]) {
          runs[2 * nd] = ep[i];
          runs[2 * nd + 1] = 0;
          ++nd;
        }
        runs[2 * (nd - 1) + 1] += 1;
      }
      if (jb->n_distinct) jb->n_distinct[si] = nd;
      if (jb->counts) {
        uint32_t* c = jb->counts + si * 2 * (uint64_t)R;
        memset(c, 0, sizeof(uint32_t) * 2 * R);
        memcpy(c, runs, sizeof(uint32_t) * 2 * nd);
      }
      if (jb->digest) {
        uint64_t d = 0;
        for (uint32_t r = 0; r < nd; ++r) d += or_digest_term(s, runs[2 * r], runs[2 * r + 1]);
        jb->digest[si] = d;
      }
      if (jb->topk && jb->k) {
        qsort(runs, nd, 2 * sizeof(uint32_t), cmp_rank);
        uint32_t* o = jb->topk + si * 2 * (uint64_t)jb->k;
        for (uint32_t r = 0; r < jb->k; ++r) {
          o[2 * r] = r < nd ? runs[2 * r] : 0xFFFFFFFFu;
          o[2 * r + 1] = r < nd ? runs[2 * r + 1] : 0;
        }
      }
    }
  }
  free(ep);
  free(runs);
  return NULL;
}

int or_run(const or_graph* g, const or_pool* pool, uint32_t T, uint64_t seed, uint32_t R,
           const uint32_t* sources, uint64_t n_src, uint32_t k, int nthreads, uint32_t* n_distinct,
           uint32_t* counts, uint32_t* topk, uint64_t* digest, uint32_t* endpoints, uint32_t* lengths,
           or_stats* stats) {
  if (!g || T == 0 || R == 0) return -1;
  if (!sources && n_src > g->n) return -1;
  if (sources)
    for (uint64_t i = 0; i < n_src; ++i)
      if (sources[i] >= g->n) return -1;
  if (pool && pool->T != T) return -1;
  nthreads = clamp_threads(nthreads);
  pthread_t th[256];
  run_job* jobs = (run_job*)calloc((size_t)nthreads, sizeof(run_job));
  uint64_t next = 0;
  for (int t = 0; t < nthreads; ++t) {
    run_job* jb = &jobs[t];
    jb->g = g; jb->pool = pool; jb->T = T; jb->R = R; jb->k = k; jb->seed = seed;
    jb->sources = sources; jb->n_src = n_src;
    jb->n_distinct = n_distinct; jb->counts = counts; jb->topk = topk; jb->digest = digest;
    jb->endpoints = endpoints; jb->lengths = lengths; jb->next = &next;
    pthread_create(&th[t], NULL, run_worker, jb);
  }
  or_stats tot;
  memset(&tot, 0, sizeof tot);
  for (int t = 0; t < nthreads; ++t) {
    pthread_join(th[t], NULL);
    const or_stats* s = &jobs[t].st;
    tot.walks += s->walks; tot.moves += s->moves; tot.steps += s->steps;
    tot.capped += s->capped; tot.dangling_moves += s->dangling_moves;
    tot.plain_moves += s->plain_moves; tot.stitched_moves += s->stitched_moves;
    tot.probe_log_sum += s->probe_log_sum; tot.lines += s->lines;
  }
  free(jobs);
  if (stats) *stats = tot;
  return 0;
}
