/*
 * jet_oracle.h -- plain single-threaded CPU oracle for deterministic Jet refinement of a
 * partitioned hypergraph under the connectivity (lambda - 1) metric.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library.  Only the tests, the
 * smoke check and the benchmark's CPU-baseline leg may load it.  It shares no source, header,
 * table or helper with the GPU library; the two only consume the same seeded inputs.
 *
 * All pointers are host pointers.  Vertex and net weights: NULL means unit weight.
 * Blocks are numbered 0..k-1.
 */
#ifndef JET_ORACLE_H
#define JET_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t n, m;
  int64_t p;
  const int64_t *off;   /* [m+1] pins of net e are pins[off[e] .. off[e+1]) */
  const int32_t *pins;  /* [p] */
  const int32_t *nw;    /* [m] net weights or NULL */
  const int32_t *vw;    /* [n] vertex weights or NULL */
  int32_t k;
  double eps;
} jo_hg;

typedef struct {
  int32_t limit;                /* iterations without improvement before a temperature round ends */
  int32_t max_iters;            /* hard cap on iterations per temperature round */
  int32_t num_tau;              /* number of temperature rounds, 1..8 */
  float tau[8];                 /* temperatures in [0,1] */
  int32_t deadzone_ppm;         /* deadzone factor d times 1e6 */
  int32_t max_rebalance_rounds; /* cap on rebalancing rounds per call */
  int32_t rb_unweighted;        /* 0: rebalancing priority gain / c(v) or gain * c(v) (Section 4.3);
                                   1: the gain alone (the original Jet's priority, an ablation);
                                   2: the original Jet's bucket order of the loss, a bucket's
                                   vertices in ID order (an ablation) */
} jo_params;

typedef struct {
  int64_t km1_in, km1_out, lmax, max_block_weight;
  int32_t iterations, rebalance_rounds, balanced, moves_executed;
  int32_t tau_q_used[8];
} jo_stats;

typedef struct { /* one record per Jet iteration */
  int64_t km1;          /* after the iteration (after rebalancing) */
  int64_t overload;     /* max(0, max block weight - Lmax) after the iteration */
  int32_t n_cand;       /* |M| */
  int32_t n_moved;      /* |X|, moves kept by the afterburner */
  int32_t rb_rounds;    /* rebalancing rounds run in this iteration */
  int32_t rb_moved;     /* vertices moved by the rebalancer in this iteration */
} jo_trace;

/* connectivity metric sum_e w(e) (lambda(e) - 1), lambda counted from scratch */
int64_t jo_km1(const jo_hg *h, const int32_t *part);
/* pin counts phi[e*k + b] = |e intersect V_b| */
void jo_phi(const jo_hg *h, const int32_t *part, int32_t *phi);
/* block weights bw[b] */
void jo_block_weights(const jo_hg *h, const int32_t *part, int64_t *bw);
/* A = ceil(W/k), Lmax = floor((1+eps) A), DZ = ceil((1+eps) A - d eps A) */
void jo_limits(int64_t W, int32_t k, double eps, int32_t deadzone_ppm, int64_t *A, int64_t *lmax, int64_t *dz);
/* tau_q = floor(tau * 65536 + 0.5) */
int32_t jo_quantize_tau(float tau);
/* gain of moving v alone to block b, by recomputing the metric before and after (brute force) */
int64_t jo_gain_bruteforce(const jo_hg *h, const int32_t *part, int32_t v, int32_t b);

/* Move candidates: t[v] target (-1 if v has no adjacent foreign block), g[v] its gain,
 * inM[v] = 1 iff v is a candidate.  lock may be NULL. */
void jo_candidates(const jo_hg *h, const int32_t *part, const uint8_t *lock, int32_t tau_q, int32_t *t,
                   int32_t *g, uint8_t *inM);
/* Candidate test for the listed vertices only (spot checks on large inputs). */
void jo_candidates_sample(const jo_hg *h, const int32_t *part, const uint8_t *lock, int32_t tau_q,
                          const int32_t *verts, int64_t nverts, int32_t *t, int32_t *g, uint8_t *inM);
/* Hypergraph afterburner (per-net replay of the ordered candidates): recomputed gains rg[v]
 * (0 for non-candidates). */
void jo_afterburner(const jo_hg *h, const int32_t *part, const int32_t *t, const int32_t *g, const uint8_t *inM,
                    int32_t *rg);
/* The afterburner's plain definition: execute the candidates one by one in order and record each
 * move's metric change by full recomputation.  O(|M| p); small inputs only. */
void jo_afterburner_replay(const jo_hg *h, const int32_t *part, const int32_t *t, const int32_t *g,
                           const uint8_t *inM, int64_t *rg);

/* One rebalancing round from part: writes sel_target[v] (-1 if v is not moved) and applies the
 * moves to part.  Returns the number of moved vertices. */
int32_t jo_rebalance_round(const jo_hg *h, int32_t *part, int32_t deadzone_ppm, int32_t *sel_target);
/* The same round in another order (jo_params.rb_unweighted): 1 the original Jet rebalancer's
 * priority (the gain alone), 2 its bucket order of the loss; the weights still count towards the
 * amount to move. */
int32_t jo_rebalance_round_w(const jo_hg *h, int32_t *part, int32_t deadzone_ppm, int32_t order,
                             int32_t *sel_target);
/* Rebalancing rounds until balanced, a round selects nothing, or the cap.  0 = balanced, 1 = not. */
int jo_rebalance(const jo_hg *h, int32_t *part, const jo_params *prm, jo_stats *st);
/* Full Jet refinement (all temperature rounds).  trace may be NULL; at most trace_cap records are
 * written; *trace_len receives the number of iterations.  0 = balanced result, 1 = not. */
int jo_refine(const jo_hg *h, int32_t *part, const jo_params *prm, jo_stats *st, jo_trace *trace,
              int32_t trace_cap, int32_t *trace_len);

/* Minimum metric over all 2-way partitions satisfying the balance constraint (n <= 24). */
int64_t jo_bruteforce_2way(const jo_hg *h);

/* ---- synchronous clustering of the coarsening phase (Section 6, Algorithm 4; coarsen_oracle.c) ---- */

/* Sub-round sizes of the prefix-doubling schedule for n vertices: initial_single sub-rounds of one
 * vertex, then 2, 4, 8, ... up to max(1, n / cap_div).  Writes min(count, max_sizes) sizes (sizes
 * may be NULL) and returns the number of sub-rounds, -1 for bad arguments. */
int64_t jo_coarsen_schedule(int32_t n, int32_t initial_single, int32_t cap_div, int32_t *sizes, int64_t max_sizes);
/* One sub-round over the vertices B[0..nb) of the clustering label[n] / cw[n] (cluster weights by
 * label), maximum cluster weight wmax: T[n] receives the targets after swap prevention (-1 outside
 * B and for no target; T[x] = x where x stays for its swap partner); approved moves are applied to
 * label and cw.  Returns the number of moved vertices. */
int32_t jo_coarsen_subround(const jo_hg *h, int32_t *label, int64_t *cw, const int32_t *B, int32_t nb, int64_t wmax,
                            int32_t *T);
/* The whole clustering pass over the vertex order order[n] (a permutation): label[n] receives
 * every vertex's cluster label.  Returns the number of clusters, -1 for a bad order or schedule. */
int32_t jo_coarsen(const jo_hg *h, const int32_t *order, int64_t wmax, int32_t initial_single, int32_t cap_div,
                   int32_t *label);

/* ---- flow-based refinement (Section 5; flow_oracle.c) ---- */

typedef struct {
  int64_t old_cut, new_cut;  /* the pair's induced cut before, and after (old_cut if not replaced) */
  int32_t iterations;        /* maximum-flow computations of the piercing loop */
  int32_t region_a, region_b; /* region vertices of each block */
  int32_t moved;             /* vertices that changed block */
} jo_flow_pair_stats;

typedef struct {
  int64_t km1_in, km1_out;
  int32_t rounds, matchings, pairs, accepted, flow_calls, moved;
} jo_flow_stats;

/* Region of the pair (a, b) for alpha: region[v] = 1 (block a's side), 2 (b's side), 0 outside.
 * Returns the number of region vertices, -1 on a bad argument. */
int32_t jo_flow_region(const jo_hg *h, const int32_t *part, int32_t a, int32_t b, int32_t alpha, int8_t *region);
/* Maximum flow of the pair's Lawler network with terminals term[v] (vertices of a and b: 0 free,
 * 1 source, 2 sink), and the residual reachable sets S_r (in_sr) and T_r (in_tr) over the vertices. */
int64_t jo_flow_mincut(const jo_hg *h, const int32_t *part, int32_t a, int32_t b, const int8_t *term,
                       uint8_t *in_sr, uint8_t *in_tr);
/* Two-way refinement of blocks a and b (Algorithm 3), part updated in place.  1 if replaced. */
int32_t jo_flow_pair(const jo_hg *h, int32_t *part, int32_t a, int32_t b, int32_t alpha, jo_flow_pair_stats *st);
/* k-way flow refinement with the matching schedule (Section 5.2), part updated in place. */
int32_t jo_flow_refine(const jo_hg *h, int32_t *part, int32_t alpha, int32_t max_rounds, jo_flow_stats *st);

#ifdef __cplusplus
}
#endif
#endif
