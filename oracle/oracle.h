/*
 * CPU oracle for fully edge-weighted personalized PageRank by Monte Carlo
 * walks (Lin, "Distributed Algorithms for Fully Personalized PageRank on
 * Large Graphs", WWW'19).
 *
 * TEST INFRASTRUCTURE ONLY. This code is plain, slow and written to be
 * checked against the paper by eye. Only the test suite, the smoke check and
 * the benchmark's CPU-baseline leg may load it. It shares no code, header,
 * table or constant with the GPU library; the two sides meet only in the
 * seeded input graphs.
 *
 * Definitions followed (paper sections):
 *  - routing probability r(s,t) = w(s,t) / sum_v w(s,v)     (Sec. 2.1)
 *  - walk: pick the next node with probability r, then stop there with
 *    probability alpha; at a node without out-neighbours restart from the
 *    walk's head                                            (Sec. 2.1, Ex. 1)
 *  - one move per active path per round, coin q <= alpha    (Algorithm 2)
 *  - estimate pi(s,t) = #walks from s ending at t / omega   (Sec. 2.1, Alg. 2)
 *  - big moves: multi-step moves for small nodes carrying a termination
 *    mark                                                    (Sec. 4.2)
 *
 * Integer realisation (the readings the GPU path implements too):
 *  - draws: Philox4x32-10 (Salmon et al., SC'11), key = (seed_lo, seed_hi),
 *    counter = (walk i, move m, source s, 0) for walk moves and
 *    (slot j, step t, node v, 1) for short-walk pool steps.
 *  - coin: terminate iff x2 < T_alpha, T_alpha = floor(alpha*2^32 + 1/2)
 *    clamped to [1, 2^32-1].
 *  - edge pick: X = floor(((x1*2^32 + x0) * W) / 2^64), the chosen edge is
 *    the first j with P[j] > X where P is the inclusive prefix of the row's
 *    integer weights and W its total.
 */
#ifndef FPPR_ORACLE_H
#define FPPR_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define OR_MOVE_CAP 65536u
#define OR_POOL_TERM 1u

typedef struct or_graph or_graph;
typedef struct or_pool or_pool;

typedef struct {
  uint64_t walks;          /* walks completed */
  uint64_t moves;          /* Philox-keyed iterations */
  uint64_t steps;          /* edges traversed incl. restarts and stitched steps */
  uint64_t capped;         /* walks stopped by the move cap */
  uint64_t dangling_moves; /* restart moves */
  uint64_t plain_moves;    /* weighted edge picks */
  uint64_t stitched_moves; /* pool entries taken */
  uint64_t probe_log_sum;  /* sum over plain moves of ceil(log2(deg)) */
  uint64_t lines;          /* distinct 64-byte lines touched, line model */
} or_stats;

/* Philox4x32-10 block function. */
void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

/* floor(alpha * 2^32 + 0.5) clamped to [1, 2^32-1]; 0 if alpha is not in (0,1). */
uint32_t or_alpha_threshold(double alpha);

/* Weighted pick on one row: P = inclusive prefix (deg entries), W = P[deg-1].
 * Returns the edge index. */
uint32_t or_pick(const uint64_t* P, uint32_t deg, uint32_t x0, uint32_t x1);

/* Graph: references the caller's CSR arrays (kept alive by the caller) and
 * computes its own prefix sums. NULL on invalid input. */
or_graph* or_graph_new(uint32_t n, uint64_t m, const uint64_t* row_offsets,
                       const uint32_t* col, const uint32_t* w);
void or_graph_free(or_graph* g);
/* Row prefix access for tests: copies P[0..m) into out. */
void or_graph_prefix(const or_graph* g, uint64_t* out);

/* Short-walk pool for the small nodes (1 <= deg <= S): K walks of at most L
 * plain steps each. Entry encoding (uint64): end | steps << 32 | mark << 48,
 * mark 1 = terminated, 0 = still active. Entries are ordered by small node
 * id, then slot. K must be a power of two. */
or_pool* or_pool_new(const or_graph* g, uint32_t S, uint32_t L, uint32_t K, uint32_t T,
                     uint64_t seed, int nthreads);
void or_pool_free(or_pool* p);
uint64_t or_pool_small_count(const or_pool* p);
void or_pool_entries(const or_pool* p, uint64_t* out);

/* Runs R walks from each source (sources == NULL: all nodes 0..n-1) and
 * aggregates. pool == NULL runs plain walks; else stitched walks.
 * Outputs (each may be NULL):
 *   n_distinct[n_src]        distinct endpoints per source
 *   counts[n_src][R][2]      (t, count) sorted by t, first n_distinct valid,
 *                            the rest zero
 *   topk[n_src][k][2]        (t, count) by count desc, t asc; padded with
 *                            (0xFFFFFFFF, 0)
 *   digest[n_src]            sum mod 2^64 of fmix(s, t, count) over counts
 *   endpoints[n_src][R]      endpoint of walk i
 *   lengths[n_src][R]        steps of walk i
 * Returns 0 on success, -1 on invalid arguments. */
int or_run(const or_graph* g, const or_pool* pool, uint32_t T, uint64_t seed, uint32_t R,
           const uint32_t* sources, uint64_t n_src, uint32_t k, int nthreads,
           uint32_t* n_distinct, uint32_t* counts, uint32_t* topk, uint64_t* digest,
           uint32_t* endpoints, uint32_t* lengths, or_stats* stats);

/* The per-source digest term (exposed so tests can recompute it). */
uint64_t or_digest_term(uint32_t s, uint32_t t, uint32_t count);

#ifdef __cplusplus
}
#endif
#endif
