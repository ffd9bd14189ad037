/*
 * jet.h -- C ABI of the MI355X (gfx950) library for deterministic Jet refinement of a k-way
 * partitioned hypergraph under the connectivity (lambda - 1) metric.
 *
 * Method: "Deterministic Parallel High-Quality Hypergraph Partitioning" (arXiv 2504.12013),
 * Section 4 (Deterministic Jet Refinement): Algorithm 1 (the Jet loop), Section 4.1 (move
 * candidates with temperature tau, locking, rollback), Section 4.2 / Algorithm 2 (hypergraph
 * afterburner), Section 4.3 (deterministic rebalancing).  Definitions from Section 2.
 *
 * Conventions for every entry point:
 *  - Array arguments are DEVICE pointers (HIP / ROCm device memory) unless marked [host].
 *  - Every call is ordered on the HIP stream given to jet_init (passed as void*, NULL = the null
 *    stream).  Calls that fill [host] outputs synchronise that stream before returning; the others
 *    return as soon as their work is enqueued unless stated otherwise.
 *  - Blocks are numbered 0..k-1.  A partition is int32 part[n] with 0 <= part[v] < k.
 *  - Results depend only on the inputs and parameters (bit-identical across runs, streams and
 *    launch configurations).  All partition arithmetic is exact integer arithmetic.
 *  - Return value: JET_OK (0), JET_IMBALANCED (1, the call completed with a valid partition that
 *    violates the balance constraint), or a negative error code.  Nothing throws across the ABI.
 *    On an error the output partition is not defined unless stated otherwise.
 *  - A context is not thread safe: calls on one context must not overlap.
 */
#ifndef JET_H
#define JET_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define JET_OK 0
#define JET_IMBALANCED 1
#define JET_EINVAL (-1)     /* bad argument: sizes, NULL pointer, k outside [2,128], eps outside
                               (0,1), non-increasing offsets, empty net, pin or part out of range,
                               repeated pin in a net, weight < 1, bad params */
#define JET_ENOMEM (-2)     /* device or host allocation failed */
#define JET_EHIP (-3)       /* a HIP runtime call failed; jet_last_error() has the message */
#define JET_EOVERFLOW (-4)  /* total vertex weight >= 2^31, or a vertex's incident net weight
                               sum >= 2^31, or more than 2^31-1 pins */
#define JET_EUNSUPPORTED (-5) /* an input shape this library cannot process (message in
                                 jet_last_error()); no partial result is written */

typedef struct jet_ctx jet_ctx;

/* Parameters of one jet_refine / jet_rebalance call. */
typedef struct {
  int32_t limit;                /* Algorithm 1: iterations without strict improvement before a
                                   temperature round ends (paper's final setting: 8) */
  int32_t max_iters;            /* hard cap on iterations per temperature round */
  int32_t num_tau;              /* number of temperature rounds, 1..8, run one after another */
  float tau[8];                 /* temperatures in [0,1] (Section 4.1); quantised on the host to
                                   tau_q = floor(tau * 65536 + 0.5) */
  int32_t deadzone_ppm;         /* Section 4.3 deadzone factor d, times 1e6 (paper: d = 0.1) */
  int32_t max_rebalance_rounds; /* cap on rebalancing rounds per rebalancing call */
  int32_t rb_unweighted;        /* rebalancing order.  0: priority gain / c(v) for a negative gain,
                                   gain * c(v) otherwise (Section 4.3); 1: the gain alone, the
                                   priority of the original Jet rebalancer that Section 4.3
                                   contrasts (an ablation); 2: the original Jet's bucket order of
                                   the loss -- bucket 0 for gain >= 0, else 1 + floor(log2(-gain)),
                                   lower buckets first, vertex-ID order inside a bucket (an
                                   ablation).  Other values: JET_EINVAL */
} jet_params;

/* [host] results of a call */
typedef struct {
  int64_t km1_in;               /* metric of the input partition */
  int64_t km1_out;              /* metric of the output partition */
  int64_t lmax;                 /* balance limit floor((1+eps) ceil(W/k)) */
  int64_t max_block_weight;     /* of the output partition */
  int32_t iterations;           /* Jet iterations executed, summed over temperature rounds */
  int32_t rebalance_rounds;     /* rebalancing rounds executed */
  int32_t balanced;             /* output satisfies max block weight <= lmax */
  int32_t moves_executed;       /* moves kept by the afterburner, summed over iterations */
  int32_t tau_q_used[8];        /* quantised temperatures, one per temperature round */
} jet_stats;

/* [host] one record per Jet iteration (jet_refine_ex) */
typedef struct {
  int64_t km1;                  /* metric after the iteration (after rebalancing) */
  int64_t overload;             /* max(0, max block weight - lmax) after the iteration */
  int32_t n_cand;               /* |M|: move candidates (Section 4.1) */
  int32_t n_moved;              /* |X|: candidates with recomputed gain > 0 (Algorithm 2) */
  int32_t rb_rounds;            /* rebalancing rounds run in the iteration */
  int32_t rb_moved;             /* vertices moved by those rounds */
} jet_trace;

/* Fills the paper's settings: limit 8, max_iters 1000, three temperatures 0.75 / 0.375 / 0
 * (Section 7, temperature tuning), d = 0.1, 64 rebalancing rounds, the weighted priority. */
void jet_params_default(jet_params *p);

/* Creates a context for one hypergraph H = (V, E, c, omega) (Section 2).
 *  n, m              number of vertices and nets, >= 1
 *  num_pins          total number of pins p, < 2^31
 *  net_offsets[m+1]  int64, net_offsets[0] = 0, strictly increasing (every net has >= 1 pin),
 *                    net_offsets[m] = num_pins; pins of net e are pins[net_offsets[e] ..
 *                    net_offsets[e+1])
 *  pins[num_pins]    vertex IDs in [0, n), no vertex twice in one net
 *  net_weights[m]    omega(e) >= 1, or NULL for unit weights
 *  vertex_weights[n] c(v) >= 1, or NULL for unit weights; total weight W < 2^31
 *  k                 number of blocks, 2..128
 *  eps               imbalance, 0 < eps < 1; Lmax = floor((1+eps) ceil(W/k)) (Section 2)
 *  stream            hipStream_t (as void*) every later call is ordered on
 * The context copies what it needs; the caller may free its arrays afterwards.  Synchronises the
 * stream.  On success *out owns device memory until jet_free. */
int jet_init(jet_ctx **out, int32_t n, int32_t m, int64_t num_pins, const int64_t *net_offsets, const int32_t *pins,
             const int32_t *net_weights, const int32_t *vertex_weights, int32_t k, double eps, void *stream);

/* Jet refinement (Algorithm 1) of part[n] in place, one loop per temperature.  Each iteration:
 * candidates with their best target (Section 4.1), afterburner filter (Algorithm 2), move
 * application with locking, and, if a block is overloaded, deterministic rebalancing rounds
 * (Section 4.3).  Every temperature round returns its best partition by the key (overload, metric).
 * stats may be NULL.  Returns JET_OK, JET_IMBALANCED, or an error.  Synchronises the stream. */
int jet_refine(jet_ctx *ctx, int32_t *part, const jet_params *params, jet_stats *stats);
/* As jet_refine, also writing up to trace_cap [host] iteration records to trace (may be NULL);
 * *trace_len ([host], may be NULL) receives the number of iterations executed. */
int jet_refine_ex(jet_ctx *ctx, int32_t *part, const jet_params *params, jet_stats *stats, jet_trace *trace,
                  int32_t trace_cap, int32_t *trace_len);

/* Deterministic rebalancing rounds (Section 4.3) on part[n] in place until no block is overloaded,
 * a round selects nothing, or params->max_rebalance_rounds rounds ran.  Only deadzone_ppm and
 * max_rebalance_rounds are read from params.  Synchronises the stream. */
int jet_rebalance(jet_ctx *ctx, int32_t *part, const jet_params *params, jet_stats *stats);

/* Connectivity metric sum_e omega(e) (lambda(e) - 1) of part[n] (Section 2); *km1 is [host].
 * Synchronises the stream. */
int jet_km1(jet_ctx *ctx, const int32_t *part, int64_t *km1);

/* ---- learned temperature (the paper runs a fixed schedule of temperatures, Section 4.1 and the
 * temperature study of Section 7; here a small network may choose tau per level and round) ---- */

/* Exact statistics of part on this context's hypergraph into [host] out[16]:
 *  0 n, 1 m, 2 pins, 3 largest net size, 4 k, 5 total vertex weight W, 6 Lmax, 7 largest block
 *  weight, 8 cut nets (lambda(e) >= 2), 9 connectivity metric, 10 sum of net weights, 11 boundary
 *  vertices (with an incident cut net), 12 weight of the cut nets, 13 ceil(W/k), 14-15 zero.
 * Synchronises the stream. */
int jet_level_stats(jet_ctx *ctx, const int32_t *part, int64_t out[16]);

/* [host] The 16 features of one temperature round from level statistics (no device work):
 *  log2 n, log2 m, log2 pins, pins/m, log2 largest net, pins/n, log2 k, eps,
 *  level/(levels-1) (0 if levels == 1), log2(n_finest/n), largest block weight/Lmax - 1,
 *  cut nets/m, metric/(sum of net weights), boundary vertices/n, round/(rounds-1) (0 if
 *  rounds == 1), prev_gain (relative metric decrease of the previous round, 0 for the first).
 * Level 0 is the finest level. */
int jet_tau_features(const int64_t stats[16], double eps, int32_t level, int32_t levels, int64_t n_finest,
                     int32_t round, int32_t rounds, double prev_gain, float out[16]);

/* The temperature network: 16 -> 64 -> 64 -> 1, ReLU, ReLU, sigmoid, FP32, 5,313 parameters in
 * the flat order W1[64][16], b1[64], W2[64][64], b2[64], w3[64], b3; inputs are standardised with
 * a stored per-feature mean and standard deviation.  All sums run in a fixed order (no floating-point
 * atomics), so results are reproducible. */
#define JET_MLP_NPARAM 5313
typedef struct jet_mlp jet_mlp;
/* Seeded He-uniform weights (SplitMix64), zero biases, mean 0 / std 1.  *out owns device memory. */
int jet_mlp_create(jet_mlp **out, uint64_t seed, void *stream);
/* [host] arrays, any may be NULL: params[5313], mean[16], std[16] (std > 0).  Setting params
 * resets the optimiser state.  Synchronous. */
int jet_mlp_set(jet_mlp *net, const float *params, const float *mean, const float *std);
int jet_mlp_get(jet_mlp *net, float *params, float *mean, float *std);
/* tau[B] (device) for raw features X[B][16] (device). */
int jet_mlp_forward(jet_mlp *net, const float *X, int32_t B, float *tau);
/* Gradient (device grad[5313]) of L = mean_s (tau_s - t_s)^2 over the batch X[B][16], t[B]
 * (device); *loss ([host], may be NULL) receives L. */
int jet_mlp_grad(jet_mlp *net, const float *X, const float *t, int32_t B, float *grad, float *loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with learning rate lr on that gradient. */
int jet_mlp_train_step(jet_mlp *net, const float *X, const float *t, int32_t B, float lr, float *loss);
/* Parameters and standardisation to / from a file ([host] path). */
int jet_mlp_save(jet_mlp *net, const char *path);
int jet_mlp_load(jet_mlp *net, const char *path);
int jet_mlp_free(jet_mlp *net);
const char *jet_mlp_last_error(const jet_mlp *net);

/* jet_refine with one temperature per round chosen by the network: before round r the level
 * statistics of the current partition give the features (jet_tau_features with this level,
 * levels, n_finest and the previous round's relative gain), the network gives tau.  The fixed
 * temperature params->tau[r] is used instead when net is NULL or any standardised feature has
 * magnitude above 6.  Rounds run as in jet_refine (each from the previous round's best, locks
 * cleared).  tau_used ([host] [num_tau], may be NULL) receives the temperatures used and from_net
 * ([host] [num_tau], may be NULL) 1 where the network chose it, 0 where the fixed temperature was
 * used; stats as in jet_refine, summed over rounds. */
int jet_refine_learned(jet_ctx *ctx, int32_t *part, const jet_params *params, jet_mlp *net, int32_t level,
                       int32_t levels, int64_t n_finest, jet_stats *stats, float *tau_used, int32_t *from_net);

/* ---- inspection entry points: one step of the method on a given state (all device arrays) ---- */

/* Pin counts phi[e*k + b] = |e intersect V_b| (Section 4.2) into phi[m*k]. */
int jet_phi(jet_ctx *ctx, const int32_t *part, int32_t *phi);
/* Move candidates (Section 4.1) for part: t[v] best adjacent foreign block (-1 if none or locked),
 * g[v] its gain, in_m[v] 1 iff v is a candidate for temperature tau_q / 65536.  lock[n] (uint8,
 * nonzero = locked) may be NULL. */
int jet_candidates(jet_ctx *ctx, const int32_t *part, const uint8_t *lock, int32_t tau_q, int32_t *t, int32_t *g,
                   uint8_t *in_m);
/* Afterburner (Algorithm 2): recomputed gains rg[v] (0 for non-candidates) for the candidates
 * in_m with targets t (t[v] != part[v], 0 <= t[v] < k for every candidate) and gains g. */
int jet_afterburner(jet_ctx *ctx, const int32_t *part, const int32_t *t, const int32_t *g, const uint8_t *in_m,
                    int32_t *rg);
/* One rebalancing round (Section 4.3) on part in place; sel_target[v] = new block of v, -1 if v
 * did not move.  *moved ([host], may be NULL) receives the number of moved vertices. */
int jet_rebalance_round(jet_ctx *ctx, int32_t *part, int32_t deadzone_ppm, int32_t *sel_target, int32_t *moved);

/* Diagnostics of the context's last refinement or rebalancing call ([host], either may be NULL):
 * the times the host read the device loop record (one stream synchronisation each) and the
 * iteration pieces it launched (graph replays, or eager launches with JET_OPT_GRAPH 0). */
int jet_loop_counts(jet_ctx *ctx, int64_t *host_polls, int64_t *pieces);

/* ---- synchronous clustering of the coarsening phase (Section 6, Algorithm 4) ----
 *
 * Clusters the context's hypergraph as the first step of one coarsening level (contraction of the
 * clusters is the caller's).  Every vertex starts as a singleton cluster labelled by its ID.  The
 * vertices are visited in sub-rounds B_1, B_2, ... cut from order[n] (device, a permutation of
 * 0..n-1): initial_single sub-rounds of one vertex, then sizes 2, 4, 8, ... up to
 * max(1, floor(n / cap_div)) (the paper: 100 and 100, i.e. a limit of 1% of n).  In a sub-round:
 *  - every vertex u of B_i still in a singleton cluster proposes the neighbouring cluster C of
 *    highest heavy-edge rating sum over e in I(u) of w(e) [|e cap C| > 0] / (|e| - 1) (each net
 *    counted once per cluster), among clusters whose weight plus c(u) is at most
 *    max_cluster_weight; ratings are compared in 32.32 fixed point (a net adds
 *    floor(w(e) 2^32 / (|e| - 1))), ties go to the smaller label;
 *  - two vertices proposing each other are merged toward the heavier side (its own weight plus
 *    the weights of the other vertices of B_i proposing it; the smaller ID on a tie);
 *  - the proposals to each cluster are sorted by (weight, ID); the longest prefix whose weight
 *    fits max_cluster_weight minus the cluster's weight at the start of the sub-round moves.
 * label[n] (device) receives each vertex's cluster label (a vertex ID); *num_clusters ([host], may
 * be NULL) the number of clusters.  JET_EINVAL if order is not a permutation of 0..n-1 (nothing
 * written to label), max_cluster_weight < 1, initial_single < 0 or cap_div < 1;
 * JET_EUNSUPPORTED on a batch context.  Synchronises the context's stream. */
int jet_coarsen(jet_ctx *ctx, const int32_t *order, int64_t max_cluster_weight, int32_t initial_single,
                int32_t cap_div, int32_t *label, int32_t *num_clusters);
/* One sub-round of jet_coarsen on a given clustering (inspection): the vertices verts[count]
 * (device, distinct) on label[n] / cw[n] (device; cw[j] = weight of the cluster labelled j),
 * updated in place with the approved moves; targets[n] (device) receives the targets after swap
 * prevention (-1 outside verts or without a target; targets[x] = x where x keeps its place for a
 * partner proposing it). */
int jet_coarsen_subround(jet_ctx *ctx, int32_t *label, int64_t *cw, const int32_t *verts, int32_t count,
                         int64_t max_cluster_weight, int32_t *targets);

/* ---- flow-based refinement (Section 5) ----
 *
 * Two-way refinement of a block pair by incremental bipartitioning (Section 5.1, Algorithm 3) on
 * the Lawler network of the pair's induced subhypergraph, and k-way refinement by the matching
 * schedule of block pairs (Section 5.2).  Where the paper refers to earlier work the library reads
 * it as follows:
 *  - region: breadth-first levels from the pair's boundary inside each block (through any net);
 *    whole levels while their weight fits, then the next level's vertices in increasing ID while
 *    they fit.  Block a's side may hold min(floor((1 + alpha eps) ceil(c(V)/k)) - c(V_b),
 *    c(V_a) - 1) (at least 0); the vertices of a outside it are the source terminals, those of b
 *    outside b's side the sink terminals;
 *  - piercing: the side with the lighter reachable set (c(S_r) <= c(T_r): the source side) takes
 *    its whole reachable set as terminals, plus one free vertex outside it that is a pin of a net
 *    cut by it, preferring vertices the other side does not reach, then the smallest ID;
 *  - the loop ends with the first balanced bipartition of S_r or T_r (both: the one whose heavier
 *    block is lighter, then S_r's), which replaces the pair if its cut is smaller, or equal with a
 *    lighter heavier block; before piercing, it ends once the flow reaches the pair's old cut;
 *  - schedule: rounds over the quotient-graph edges with an active endpoint (all blocks in the
 *    first round); per round, maximal matchings until every edge is scheduled, blocks by
 *    decreasing remaining degree (then ID) each matched to the unmatched neighbour of highest
 *    remaining degree (then lowest ID); a block is active in the next round if a pair with it
 *    lowered its cut; at most max_rounds rounds.
 * The maximum flow is computed by push-relabel, whose flow assignment depends on the schedule of
 * the waves; the minimum-cut sides S_r (reachable from the sources in the residual network) and
 * T_r (reaching the sinks) do not, so results are deterministic.  Every call synchronises the
 * context's stream; JET_EUNSUPPORTED on a batch context.  part (device, n) must hold blocks in
 * [0, k) (JET_EINVAL otherwise). */
typedef struct {
  int64_t old_cut, new_cut;   /* the pair's cut (nets with pins in both) before, and after */
  int32_t iterations;         /* maximum flows computed */
  int32_t region_a, region_b; /* vertices in each block's side of the region */
  int32_t moved;              /* vertices that changed block */
  int32_t replaced;           /* 1 if the pair's bipartition was replaced */
  int64_t arcs;               /* sum over the iterations of the network's arcs */
} jet_flow_pair_stats;

typedef struct {
  int64_t km1_in, km1_out;
  int32_t rounds, matchings, pairs, accepted, flow_calls, moved;
  int64_t arcs;               /* sum over all iterations of all pairs of the network's arcs */
} jet_flow_stats;

/* The region of the pair (a, b) for alpha >= 0: region[n] (device) receives 1 for block a's side,
 * 2 for b's side, 0 elsewhere.  JET_EINVAL for a == b, blocks outside [0, k) or alpha < 0. */
int jet_flow_region(jet_ctx *ctx, const int32_t *part, int32_t a, int32_t b, int32_t alpha, int8_t *region);
/* Maximum flow of the pair's network with the terminals term[n] (device: for the vertices of a
 * and b, 0 free, 1 source, 2 sink; ignored elsewhere): *flow (host) its value, in_sr[n] / in_tr[n]
 * (device) 1 for the vertices the sources reach / that reach the sinks in the residual network. */
int jet_flow_mincut(jet_ctx *ctx, const int32_t *part, int32_t a, int32_t b, const int8_t *term, int64_t *flow,
                    uint8_t *in_sr, uint8_t *in_tr);
/* Two-way refinement of (a, b); part updated in place; st (host) may be NULL. */
int jet_flow_pair(jet_ctx *ctx, int32_t *part, int32_t a, int32_t b, int32_t alpha, jet_flow_pair_stats *st);
/* k-way flow refinement; part updated in place; st (host) may be NULL.  max_rounds >= 0. */
int jet_flow_refine(jet_ctx *ctx, int32_t *part, int32_t alpha, int32_t max_rounds, jet_flow_stats *st);

/* ---- options (performance knobs; results never depend on them) ---- */

/* Move application (Algorithm 1) switches from per-move atomics to per-net recounting when the
 * listed moves' incident nets times this divisor reach the number of pins; 0 = always per move.
 * Default 16. */
#define JET_OPT_APPLY_DIVISOR 1
/* 1: launch the per-net application kernels with one wave per chunk / block per net when the
 * previous application of the same kind took that path; 0 (default): small grids always. */
#define JET_OPT_APPLY_WIDE 2
/* Bit mask of the kernel families that jet_prof_enable brackets with events (bit i = family i in
 * the order candidates, candidates_hub, afterburner, select_moves, apply, rebalance_gain,
 * rebalance_select); default all.  Fewer families, less host work per launch. */
#define JET_OPT_PROF_FAMILIES 3
/* Candidate selection with unit net weights and k <= 64 uses one lane per vertex (bit-sliced
 * block counts) when the mean degree of the non-hub vertices is below this value, a group of
 * lanes per vertex otherwise; default 24, 0 = always groups.  Results do not depend on it. */
#define JET_OPT_CAND_LANE_DEGREE 4
/* The rebalancing selection's first radix pass runs over all compute units (a histogram kernel
 * and a split kernel, several workgroups per overloaded block) on levels with at least this many
 * vertices, inside the one workgroup per block otherwise; default 2^18, 0 = always.  Results do
 * not depend on it. */
#define JET_OPT_SEL_SPLIT_MIN 5
/* 1 (default): the Jet loop (Algorithm 1) runs on the device from a captured HIP graph of one
 * iteration, replayed several times between two host looks at the loop's state; 0: the same
 * kernels are launched one by one (same results). */
#define JET_OPT_GRAPH 6
/* Rebalancing rounds (Section 4.3) a replayed iteration holds room for, 1..64, default 1; an
 * iteration that needs more continues in the next replay.  Results do not depend on it. */
#define JET_OPT_RB_SLOTS 7
/* Most replays of the iteration between two host looks at the loop's state, 1..1024, default 8.
 * Replays after the loop finished return at once.  Results do not depend on it. */
#define JET_OPT_REPLAYS 8
/* Workgroups of the persistent (grid-stride) kernels: candidates, afterburner chunks, move
 * selection, rebalancing gains; 64..65536, default 2048.  Results do not depend on it. */
#define JET_OPT_GRID 9
/* Rating-table slots (16 bytes each) of one clustering launch (jet_coarsen): a sub-round whose
 * vertices need more is rated in several launches; at least one vertex's table always fits.  The
 * table is allocated at the size a pass needs, up to this.  Default 2^28 (4 GiB). */
#define JET_OPT_CO_TABLE_SLOTS 10
/* 1: the candidate kernels and the afterburner's chunk kernel give each of the eight XCDs one
 * contiguous range of vertices or nets (so the data of neighbouring vertices and nets is fetched
 * into one L2), 0: workgroups stride over the whole range.  Default 1. */
#define JET_OPT_CAND_XCD 11
/* 1: the rebalancing gain pass gives each XCD one contiguous range of its list of movable
 * vertices, 0: workgroups stride over the whole list.  Default 1. */
#define JET_OPT_RB_XCD 12
/* 1: on a graph (every net has two pins) the afterburner takes its vertex-centric form, in which a
 * candidate sums over its neighbours (a neighbour counts in its target block when it is a
 * candidate ordered before it, else in its block); 0: the general per-net replay.  Default 1. */
#define JET_OPT_GRAPH_KERNELS 13
/* 1: move application gives each XCD one contiguous range of the move list (moves with few nets)
 * and of the net chunks (per-net recount), 0: workgroups stride over the whole range.
 * Default 0. */
#define JET_OPT_APPLY_XCD 14
/* Block pairs of one matching that jet_flow_refine refines at once, each on its own stream and
 * host thread, 1..8 (1: one after the other on the context's stream).  Default 4.  Results do not
 * depend on it: the pairs of a matching are disjoint. */
#define JET_OPT_FLOW_WORKERS 15
int jet_set_option(jet_ctx *ctx, int32_t option, int64_t value);

/* ---- batches: many independent hypergraphs refined in one call ---- */

typedef struct {
  int32_t n, m;
  int64_t num_pins;
  const int64_t *net_offsets;    /* device arrays, as for jet_init */
  const int32_t *pins;
  const int32_t *net_weights;    /* or NULL */
  const int32_t *vertex_weights; /* or NULL */
  int32_t k;
  double eps;
} jet_hg_desc;
typedef struct jet_batch jet_batch;

/* The hypergraphs (descs is [host][count]; every desc is validated as by jet_init) are packed into
 * union contexts, one per value of k (split when one would exceed 4,096 hypergraphs, 16,384
 * (hypergraph, block) pairs or 2^31 pins): vertices and nets concatenated, every per-block quantity
 * kept per (hypergraph, block), one loop record per hypergraph.  Synchronises stream.  On failure
 * no batch is returned and jet_last_error(NULL) has the message (naming the hypergraph). */
int jet_batch_init(jet_batch **out, int32_t count, const jet_hg_desc *descs, void *stream);
/* Applies jet_set_option to every union context of the batch (JET_OPT_GRAPH: the batch graph). */
int jet_batch_set_option(jet_batch *b, int32_t option, int64_t value);
/* Refines every hypergraph i in place in parts[i] ([host] array of device pointers) exactly as
 * jet_refine would (Algorithm 1 per hypergraph, its own balance limit, key, limit and rollback):
 * the result of each hypergraph does not depend on the batch or on the options.  Every kernel
 * launch covers all hypergraphs of a union context, each hypergraph's vertices and nets taking part
 * only while its own loop is in the launch's phase; one captured HIP graph holds a whole iteration
 * of every union context and is replayed `replays` (1..1024) times between two host looks at the
 * loop records, until every hypergraph's loop is done.  Runs on the stream given to jet_batch_init.
 * stats and rcs ([host][count], may be NULL) receive each hypergraph's statistics and return code.
 * Returns a negative code on failure, else JET_IMBALANCED if any hypergraph is, else JET_OK. */
int jet_batch_refine(jet_batch *b, int32_t *const *parts, const jet_params *params, int32_t replays,
                     jet_stats *stats, int32_t *rcs);
int jet_batch_free(jet_batch *b);
const char *jet_batch_last_error(const jet_batch *b);

/* ---- instrumentation ---- */

/* [host] accumulated HIP-event timing of one kernel family on the context's stream */
typedef struct {
  char name[24];       /* kernel family */
  int64_t launches;    /* timed launches */
  double total_ms;     /* summed event-to-event duration */
  double alg_bytes;    /* summed algorithmic bytes (0 when data dependent) */
} jet_prof_entry;

/* on != 0: bracket every kernel launch of the context (of the families JET_OPT_PROF_FAMILIES
 * selects) with HIP events from now on (counters are reset); on == 0: stop.  Adds a few
 * microseconds of host work per bracketed launch; the durations are read at jet_prof_read. */
int jet_prof_enable(jet_ctx *ctx, int32_t on);
/* Writes up to cap [host] entries (one per kernel family that ran) and the count to *count.
 * Synchronises the stream. */
int jet_prof_read(jet_ctx *ctx, jet_prof_entry *out, int32_t cap, int32_t *count);
/* Instrumentation of every union context (as jet_prof_enable / jet_prof_read; entries summed). */
int jet_batch_prof_enable(jet_batch *b, int32_t on);
int jet_batch_prof_read(jet_batch *b, jet_prof_entry *out, int32_t cap, int32_t *count);

/* ---- allocation-free entry point ---- */

/* For callers that cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc): the connectivity metric of part, the value jet_km1 returns, from
 * the caller's CSR without a context.  Arguments as for jet_init (device net_offsets[m+1], pins,
 * net_weights or NULL, part[n]) and k in [2,128]; *km1 is a DEVICE int64 that receives the metric,
 * or -1 if an offset, pin or part value is out of range (reads never leave the stated sizes).
 * Only enqueues two kernels on stream: no allocation, no synchronisation, no host read of device
 * data.  Per-workgroup partial sums live in a static device array of 65,536 int64 (512 KiB) per GPU,
 * held until the process ends; each call overwrites the slots it uses, so calls that overlap on one
 * GPU race (order them on one stream).  m above 4,194,304 nets (64 per slot) is rejected with
 * JET_EUNSUPPORTED before any work is enqueued; bad sizes or NULL pointers give JET_EINVAL. */
int jet_km1_static(int32_t n, int32_t m, int64_t num_pins, const int64_t *net_offsets, const int32_t *pins,
                   const int32_t *net_weights, const int32_t *part, int32_t k, int64_t *km1, void *stream);
/* Message of the last jet_km1_static failure on this thread. */
const char *jet_km1_static_last_error(void);

/* Releases the context (NULL is allowed). */
int jet_free(jet_ctx *ctx);

/* Static description of an error code. */
const char *jet_strerror(int code);
/* Message of the last failure on ctx (empty string if none; ctx may be NULL for jet_init
 * failures, which are recorded per thread). */
const char *jet_last_error(const jet_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif
