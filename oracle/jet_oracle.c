/*
 * jet_oracle.c -- plain, slow, single-threaded CPU oracle for deterministic Jet refinement of a
 * partitioned hypergraph under the connectivity (lambda - 1) metric.
 *
 * TEST INFRASTRUCTURE ONLY: it is the yardstick the GPU library is checked against.  Only the
 * tests, the smoke check and the benchmark's CPU-baseline leg may load it.  It shares no code with
 * the GPU library.
 *
 * Everything here follows the paper "Deterministic Parallel High-Quality Hypergraph Partitioning"
 * (arXiv 2504.12013):
 *   - Section 2 (Preliminaries): hypergraph, blocks, balance constraint Lmax, connectivity set,
 *     connectivity lambda(e) and the (lambda - 1) metric;
 *   - Section 4.1 (Overview, Algorithm 1 "Jet Overview"): the Jet loop, move candidates with the
 *     temperature filter, locking and rollback;
 *   - Section 4.2 (Algorithm 2 "Hypergraph-Afterburner"): recomputed gains by per-net replay of
 *     the candidates in descending gain order;
 *   - Section 4.3 (Deterministic Rebalancing): priorities, deadzone, heavy-vertex rule, sort +
 *     prefix sum + binary search selection.
 * Where the paper leaves a choice open, the reading taken is written next to the code.
 *
 * Arithmetic is exact integer throughout (weights are natural numbers, Section 2).  Loops run in
 * vertex-ID or net-ID order so the code can be audited line by line against the text.
 */
#include "jet_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static inline int64_t w_net(const jo_hg *h, int64_t e) { return h->nw ? (int64_t)h->nw[e] : 1; }
static inline int64_t w_vtx(const jo_hg *h, int64_t v) { return h->vw ? (int64_t)h->vw[v] : 1; }

static void *xmalloc(size_t sz) {
  void *p = malloc(sz ? sz : 1);
  if (!p) abort();
  return p;
}
static void *xcalloc(size_t cnt, size_t sz) {
  void *p = calloc(cnt ? cnt : 1, sz ? sz : 1);
  if (!p) abort();
  return p;
}

/* ------------------------------------------------------------------ incidence lists I(v) */

typedef struct { int64_t *voff; int32_t *inc; } incidence;

static incidence build_incidence(const jo_hg *h) {
  incidence I;
  I.voff = (int64_t *)xcalloc((size_t)h->n + 1, sizeof(int64_t));
  I.inc = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)h->p);
  for (int64_t q = 0; q < h->p; ++q) I.voff[h->pins[q] + 1] += 1;
  for (int32_t v = 0; v < h->n; ++v) I.voff[v + 1] += I.voff[v];
  int64_t *cur = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)h->n);
  memcpy(cur, I.voff, sizeof(int64_t) * (size_t)h->n);
  for (int32_t e = 0; e < h->m; ++e)
    for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) I.inc[cur[h->pins[q]]++] = e;
  free(cur);
  return I;
}

static void free_incidence(incidence *I) {
  free(I->voff);
  free(I->inc);
}

/* ------------------------------------------------------------------ Section 2 definitions */

/* (lambda - 1)(Pi) = sum_e (lambda(e) - 1) w(e), lambda(e) = number of blocks that e touches */
int64_t jo_km1(const jo_hg *h, const int32_t *part) {
  int32_t *seen = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)h->k);
  for (int32_t b = 0; b < h->k; ++b) seen[b] = -1;
  int64_t total = 0;
  for (int32_t e = 0; e < h->m; ++e) {
    int64_t lambda = 0;
    for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) {
      int32_t b = part[h->pins[q]];
      if (seen[b] != e) {
        seen[b] = e;
        lambda += 1;
      }
    }
    if (lambda > 0) total += (lambda - 1) * w_net(h, e);
  }
  free(seen);
  return total;
}

/* phi_e[b] = |e intersect V_b|  (Section 4.2, the pin counts tracked per net) */
void jo_phi(const jo_hg *h, const int32_t *part, int32_t *phi) {
  memset(phi, 0, sizeof(int32_t) * (size_t)h->m * (size_t)h->k);
  for (int32_t e = 0; e < h->m; ++e)
    for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) phi[(int64_t)e * h->k + part[h->pins[q]]] += 1;
}

void jo_block_weights(const jo_hg *h, const int32_t *part, int64_t *bw) {
  for (int32_t b = 0; b < h->k; ++b) bw[b] = 0;
  for (int32_t v = 0; v < h->n; ++v) bw[part[v]] += w_vtx(h, v);
}

/* Balance constraint (Section 2): c(V_i) <= Lmax = (1 + eps) ceil(c(V)/k).  Block weights are
 * integers, so the test is bw <= floor((1 + eps) A).  Deadzone (Section 4.3): a block with
 * c(V_i) >= Lmax - d eps A is not a valid rebalancing target; as an integer threshold that is
 * bw >= ceil((1 + eps) A - d eps A).  Both are evaluated once in IEEE double. */
void jo_limits(int64_t W, int32_t k, double eps, int32_t deadzone_ppm, int64_t *A, int64_t *lmax, int64_t *dz) {
  int64_t a = (W + k - 1) / k;
  double ad = (double)a;
  double lmax_real = (1.0 + eps) * ad;
  double dz_real = lmax_real - ((double)deadzone_ppm / 1e6) * eps * ad;
  *A = a;
  *lmax = (int64_t)floor(lmax_real);
  *dz = (int64_t)ceil(dz_real);
}

/* The temperature enters the candidate filter as a 16-bit fixed-point number so that the filter
 * is an exact integer test. */
int32_t jo_quantize_tau(float tau) { return (int32_t)floor((double)tau * 65536.0 + 0.5); }

int64_t jo_gain_bruteforce(const jo_hg *h, const int32_t *part, int32_t v, int32_t b) {
  int32_t *tmp = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)h->n);
  memcpy(tmp, part, sizeof(int32_t) * (size_t)h->n);
  int64_t before = jo_km1(h, tmp);
  tmp[v] = b;
  int64_t after = jo_km1(h, tmp);
  free(tmp);
  return before - after;
}

static int64_t total_weight(const jo_hg *h) {
  int64_t W = 0;
  for (int32_t v = 0; v < h->n; ++v) W += w_vtx(h, v);
  return W;
}

static int64_t overload_of(const int64_t *bw, int32_t k, int64_t lmax) {
  int64_t worst = 0;
  for (int32_t b = 0; b < k; ++b)
    if (bw[b] - lmax > worst) worst = bw[b] - lmax;
  return worst;
}

/* ------------------------------------------------------------------ gains from pin counts */

/* For v in block s and every block b:
 *   gain(v, b) = sum_{e in I(v)} w(e) ([phi_e[s] = 1] - [phi_e[b] = 0])
 * i.e. the metric decrease of moving v alone: nets that v leaves as their last pin in s lose s
 * from their connectivity set, nets that do not yet touch b gain b.  Also returns
 *   adj[b] = 1 iff some e in I(v) has phi_e[b] > 0,
 *   aff    = sum_{e in I(v) : |e intersect V_s| > 1} w(e)    (the temperature filter's affinity).
 * gains[s] is the gain of staying (only the first sum). */
static void vertex_gains(const jo_hg *h, const incidence *I, const int32_t *phi, const int32_t *part, int32_t v,
                         int64_t *gains, uint8_t *adj, int64_t *aff_out) {
  const int32_t k = h->k, s = part[v];
  int64_t benefit = 0, aff = 0;
  for (int32_t b = 0; b < k; ++b) {
    gains[b] = 0;
    adj[b] = 0;
  }
  for (int64_t q = I->voff[v]; q < I->voff[v + 1]; ++q) {
    const int32_t e = I->inc[q];
    const int32_t *row = phi + (int64_t)e * k;
    const int64_t w = w_net(h, e);
    if (row[s] == 1) benefit += w;
    if (row[s] > 1) aff += w;
    for (int32_t b = 0; b < k; ++b) {
      if (row[b] == 0) gains[b] -= w;
      else adj[b] = 1;
    }
  }
  for (int32_t b = 0; b < k; ++b) gains[b] += benefit;
  *aff_out = aff;
}

/* ------------------------------------------------------------------ Section 4.1: candidates */

/* Section 4.1: each vertex v in V_s picks the target t(v) of highest gain, ignoring balance and
 * assuming no other vertex moves.  It becomes a candidate iff
 *     gain(v, t(v)) >= -tau * sum_{e in I(v) : |e intersect V_s| > 1} w(e).
 * Readings: targets are the blocks b != s adjacent to v (some incident net has a pin in b); ties
 * go to the lowest block ID; a vertex without such a block is never a candidate; locked vertices
 * are never candidates; tau enters as tau_q / 65536, so the test is
 *     65536 gain + tau_q aff >= 0  in exact integer arithmetic. */
static void candidates_with(const jo_hg *h, const incidence *I, const int32_t *phi, const int32_t *part,
                            const uint8_t *lock, int32_t tau_q, int32_t *t, int32_t *g, uint8_t *inM,
                            const int32_t *verts, int64_t nverts) {
  const int32_t k = h->k;
  int64_t *gains = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)k);
  uint8_t *adj = (uint8_t *)xmalloc((size_t)k);
  const int64_t count = verts ? nverts : (int64_t)h->n;
  for (int64_t i = 0; i < count; ++i) {
    const int32_t v = verts ? verts[i] : (int32_t)i;
    t[v] = -1;
    g[v] = 0;
    inM[v] = 0;
    if (lock && lock[v]) continue;
    int64_t aff;
    vertex_gains(h, I, phi, part, v, gains, adj, &aff);
    const int32_t s = part[v];
    int32_t best = -1;
    for (int32_t b = 0; b < k; ++b) {
      if (b == s || !adj[b]) continue;
      if (best < 0 || gains[b] > gains[best]) best = b;
    }
    if (best < 0) continue;
    t[v] = best;
    g[v] = (int32_t)gains[best];
    if (65536 * gains[best] + (int64_t)tau_q * aff >= 0) inM[v] = 1;
  }
  free(gains);
  free(adj);
}

void jo_candidates(const jo_hg *h, const int32_t *part, const uint8_t *lock, int32_t tau_q, int32_t *t, int32_t *g,
                   uint8_t *inM) {
  incidence I = build_incidence(h);
  int32_t *phi = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)h->m * (size_t)h->k);
  jo_phi(h, part, phi);
  candidates_with(h, &I, phi, part, lock, tau_q, t, g, inM, NULL, 0);
  free(phi);
  free_incidence(&I);
}

/* The same candidate test for the listed vertices only (t, g, inM are indexed by vertex; entries of
 * vertices not listed are left untouched).  For spot checks on inputs too large for a full pass. */
void jo_candidates_sample(const jo_hg *h, const int32_t *part, const uint8_t *lock, int32_t tau_q,
                          const int32_t *verts, int64_t nverts, int32_t *t, int32_t *g, uint8_t *inM) {
  incidence I = build_incidence(h);
  int32_t *phi = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)h->m * (size_t)h->k);
  jo_phi(h, part, phi);
  candidates_with(h, &I, phi, part, lock, tau_q, t, g, inM, verts, nverts);
  free(phi);
  free_incidence(&I);
}

/* ------------------------------------------------------------------ Section 4.2: afterburner */

/* Execution order of the candidates: highest gain first (Section 4.1/4.2).  Reading: equal gains
 * are ordered by ascending vertex ID, which makes the order total. */
typedef struct { int32_t v, g; } ord_item;

static int cmp_order(const void *a, const void *b) {
  const ord_item *x = (const ord_item *)a, *y = (const ord_item *)b;
  if (x->g != y->g) return x->g > y->g ? -1 : 1;
  return x->v < y->v ? -1 : (x->v > y->v);
}

/* Algorithm 2: for every net e, take L = e intersect M in execution order and replay the moves on
 * a private copy of the net's pin counts.  A move that empties its source block in e earns w(e);
 * a move that makes its target block appear in e costs w(e).  The sums per vertex are its
 * recomputed gains. */
static void afterburner_with(const jo_hg *h, const int32_t *phi, const int32_t *part, const int32_t *t,
                             const int32_t *g, const uint8_t *inM, int32_t *rg) {
  const int32_t k = h->k;
  int64_t *acc = (int64_t *)xcalloc((size_t)h->n, sizeof(int64_t));
  int32_t *cur = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)k);
  int64_t maxsz = 0;
  for (int32_t e = 0; e < h->m; ++e)
    if (h->off[e + 1] - h->off[e] > maxsz) maxsz = h->off[e + 1] - h->off[e];
  ord_item *L = (ord_item *)xmalloc(sizeof(ord_item) * (size_t)(maxsz > 0 ? maxsz : 1));
  for (int32_t e = 0; e < h->m; ++e) {
    int64_t cnt = 0;
    for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) {
      int32_t v = h->pins[q];
      if (inM[v]) {
        L[cnt].v = v;
        L[cnt].g = g[v];
        ++cnt;
      }
    }
    if (cnt == 0) continue; /* nets without candidates contribute nothing */
    qsort(L, (size_t)cnt, sizeof(ord_item), cmp_order);
    memcpy(cur, phi + (int64_t)e * k, sizeof(int32_t) * (size_t)k);
    const int64_t w = w_net(h, e);
    for (int64_t i = 0; i < cnt; ++i) {
      const int32_t v = L[i].v, from = part[v], to = t[v];
      cur[from] -= 1;
      if (cur[from] == 0) acc[v] += w;
      cur[to] += 1;
      if (cur[to] == 1) acc[v] -= w;
    }
  }
  for (int32_t v = 0; v < h->n; ++v) rg[v] = (int32_t)acc[v];
  free(L);
  free(cur);
  free(acc);
}

void jo_afterburner(const jo_hg *h, const int32_t *part, const int32_t *t, const int32_t *g, const uint8_t *inM,
                    int32_t *rg) {
  int32_t *phi = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)h->m * (size_t)h->k);
  jo_phi(h, part, phi);
  afterburner_with(h, phi, part, t, g, inM, rg);
  free(phi);
}

/* Section 4.1: the recomputed gain of v is the gain of moving v to t(v) assuming that every
 * candidate before v in the execution order has already moved to its target. */
void jo_afterburner_replay(const jo_hg *h, const int32_t *part, const int32_t *t, const int32_t *g,
                           const uint8_t *inM, int64_t *rg) {
  ord_item *L = (ord_item *)xmalloc(sizeof(ord_item) * (size_t)h->n);
  int64_t cnt = 0;
  for (int32_t v = 0; v < h->n; ++v) {
    rg[v] = 0;
    if (inM[v]) {
      L[cnt].v = v;
      L[cnt].g = g[v];
      ++cnt;
    }
  }
  qsort(L, (size_t)cnt, sizeof(ord_item), cmp_order);
  int32_t *cur = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)h->n);
  memcpy(cur, part, sizeof(int32_t) * (size_t)h->n);
  for (int64_t i = 0; i < cnt; ++i) {
    const int32_t v = L[i].v;
    int64_t before = jo_km1(h, cur);
    cur[v] = t[v];
    int64_t after = jo_km1(h, cur);
    rg[v] = before - after;
  }
  free(cur);
  free(L);
}

/* ------------------------------------------------------------------ Section 4.3: rebalancing */

/* pc: the weight the priority uses -- c(v), or 1 for the unweighted priority of the original Jet
 * rebalancer (an ablation; Section 4.3 contrasts the two); bucket: the loss bucket of the original
 * Jet's bucket order (the other ablation) */
typedef struct { int32_t v, target, bucket; int64_t g, c, pc; } rb_item;

/* The original Jet selects rebalancing moves by a bucket-based partial order of their loss, not by
 * a sort (Section 4.3 contrasts the two).  Reading: a move that does not lose (gain >= 0) goes to
 * bucket 0, a loss L >= 1 to bucket 1 + floor(log2 L), so each bucket spans one binary order of
 * magnitude; lower buckets are taken first. */
static int32_t loss_bucket(int64_t g) {
  if (g >= 0) return 0;
  int32_t b = 1;
  for (int64_t loss = -g; loss >= 2; loss /= 2) ++b;
  return b;
}

/* Bucket order: lower bucket first.  Within the last bucket the original takes an arbitrary subset
 * (whatever arrives first), which Section 4.3 names as its source of non-determinism; reading: the
 * vertices of a bucket are taken in vertex-ID order, so the ablation is reproducible. */
static int cmp_bucket(const void *a, const void *b) {
  const rb_item *x = (const rb_item *)a, *y = (const rb_item *)b;
  if (x->bucket != y->bucket) return x->bucket < y->bucket ? -1 : 1;
  return x->v < y->v ? -1 : (x->v > y->v);
}

/* Priority (Section 4.3): gain/c(v) if gain < 0, gain * c(v) if gain >= 0, higher first.
 * Readings: compared exactly as rationals (every non-negative gain ranks above every negative
 * one; two negatives compare g1 c2 against g2 c1); equal priorities go to the lower vertex ID.
 * With pc = 1 the priority is the gain itself. */
static int cmp_priority(const void *a, const void *b) {
  const rb_item *x = (const rb_item *)a, *y = (const rb_item *)b;
  const int xnn = x->g >= 0, ynn = y->g >= 0;
  if (xnn != ynn) return xnn ? -1 : 1;
  int64_t lhs, rhs; /* compare priority(x) against priority(y) */
  if (xnn) {
    lhs = x->g * x->pc;
    rhs = y->g * y->pc;
  } else {
    lhs = x->g * y->pc;
    rhs = y->g * x->pc;
  }
  if (lhs != rhs) return lhs > rhs ? -1 : 1;
  return x->v < y->v ? -1 : (x->v > y->v);
}

/* One round (Section 4.3).  Against the block weights at the start of the round:
 *  - only vertices of overloaded blocks (bw > Lmax) move; locks do not apply;
 *  - a vertex v with c(v) > 3/2 (c(Pi(v)) - ceil(c(V)/k)) never moves (tested as
 *    2 c(v) > 3 (bw[Pi(v)] - A));
 *  - valid targets t != Pi(v) stay balanced when v is added (bw[t] + c(v) <= Lmax) and are not in
 *    the deadzone (bw[t] < DZ); adjacency is not required;
 *  - v's gain is the best gain over valid targets (lowest block on ties); v is skipped if it has
 *    no valid target;
 *  - per overloaded block: sort by priority, prefix-sum the weights, binary-search the smallest
 *    prefix whose weight reaches bw - Lmax (all of them if the total falls short);
 *  - all selected vertices of all blocks move at once.
 * order: 0 the priority above, 1 the gain alone (pc = 1), 2 the original Jet's bucket order of
 * the loss (cmp_bucket); the prefix selection is the same for all three. */
int32_t jo_rebalance_round_w(const jo_hg *h, int32_t *part, int32_t deadzone_ppm, int32_t order,
                             int32_t *sel_target) {
  const int32_t k = h->k, n = h->n;
  int64_t A, lmax, dz;
  jo_limits(total_weight(h), k, h->eps, deadzone_ppm, &A, &lmax, &dz);
  int64_t *bw = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)k);
  jo_block_weights(h, part, bw);
  for (int32_t v = 0; v < n; ++v) sel_target[v] = -1;
  if (overload_of(bw, k, lmax) == 0) {
    free(bw);
    return 0;
  }
  incidence I = build_incidence(h);
  int32_t *phi = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)h->m * (size_t)k);
  jo_phi(h, part, phi);
  int64_t *gains = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)k);
  uint8_t *adj = (uint8_t *)xmalloc((size_t)k);
  int64_t *cnt = (int64_t *)xcalloc((size_t)k, sizeof(int64_t));
  rb_item *items = (rb_item *)xmalloc(sizeof(rb_item) * (size_t)n);
  int64_t nitems = 0;
  for (int32_t v = 0; v < n; ++v) {
    const int32_t s = part[v];
    if (bw[s] <= lmax) continue;
    const int64_t c = w_vtx(h, v);
    if (2 * c > 3 * (bw[s] - A)) continue;
    int64_t aff;
    vertex_gains(h, &I, phi, part, v, gains, adj, &aff);
    int32_t best = -1;
    for (int32_t b = 0; b < k; ++b) {
      if (b == s || bw[b] + c > lmax || bw[b] >= dz) continue;
      if (best < 0 || gains[b] > gains[best]) best = b;
    }
    if (best < 0) continue;
    items[nitems].v = v;
    items[nitems].target = best;
    items[nitems].g = gains[best];
    items[nitems].c = c;
    items[nitems].pc = order ? 1 : c;
    items[nitems].bucket = loss_bucket(gains[best]);
    ++nitems;
    cnt[s] += 1;
  }
  /* group by source block (stable counting sort keeps vertex-ID order inside a block) */
  int64_t *start = (int64_t *)xcalloc((size_t)k + 1, sizeof(int64_t));
  for (int32_t b = 0; b < k; ++b) start[b + 1] = start[b] + cnt[b];
  rb_item *grouped = (rb_item *)xmalloc(sizeof(rb_item) * (size_t)(nitems > 0 ? nitems : 1));
  int64_t *fill = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)k);
  memcpy(fill, start, sizeof(int64_t) * (size_t)k);
  for (int64_t i = 0; i < nitems; ++i) grouped[fill[part[items[i].v]]++] = items[i];
  int32_t moved = 0;
  for (int32_t b = 0; b < k; ++b) {
    if (bw[b] <= lmax || cnt[b] == 0) continue;
    rb_item *blk = grouped + start[b];
    const int64_t len = cnt[b];
    qsort(blk, (size_t)len, sizeof(rb_item), order == 2 ? cmp_bucket : cmp_priority);
    int64_t *prefix = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)len);
    int64_t run = 0;
    for (int64_t i = 0; i < len; ++i) {
      run += blk[i].c;
      prefix[i] = run;
    }
    const int64_t need = bw[b] - lmax;
    int64_t take;
    if (prefix[len - 1] < need) {
      take = len;
    } else { /* smallest i with prefix[i] >= need */
      int64_t lo = 0, hi = len - 1;
      while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (prefix[mid] >= need) hi = mid; else lo = mid + 1;
      }
      take = lo + 1;
    }
    for (int64_t i = 0; i < take; ++i) sel_target[blk[i].v] = blk[i].target;
    moved += (int32_t)take;
    free(prefix);
  }
  for (int32_t v = 0; v < n; ++v)
    if (sel_target[v] >= 0) part[v] = sel_target[v];
  free(fill);
  free(grouped);
  free(start);
  free(items);
  free(cnt);
  free(adj);
  free(gains);
  free(phi);
  free_incidence(&I);
  free(bw);
  return moved;
}

int32_t jo_rebalance_round(const jo_hg *h, int32_t *part, int32_t deadzone_ppm, int32_t *sel_target) {
  return jo_rebalance_round_w(h, part, deadzone_ppm, 0, sel_target);
}

/* Rounds until no block is overloaded, a round selects nothing, or the round cap is reached. */
static int rebalance_rounds(const jo_hg *h, int32_t *part, int32_t deadzone_ppm, int32_t unweighted,
                            int32_t max_rounds, int32_t *rounds_out, int32_t *moved_out) {
  int64_t A, lmax, dz;
  jo_limits(total_weight(h), h->k, h->eps, deadzone_ppm, &A, &lmax, &dz);
  int64_t *bw = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)h->k);
  int32_t *sel = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)h->n);
  int32_t rounds = 0, moved = 0;
  for (;;) {
    jo_block_weights(h, part, bw);
    if (overload_of(bw, h->k, lmax) == 0 || rounds >= max_rounds) break;
    int32_t mv = jo_rebalance_round_w(h, part, deadzone_ppm, unweighted, sel);
    rounds += 1;
    moved += mv;
    if (mv == 0) break;
  }
  jo_block_weights(h, part, bw);
  int balanced = overload_of(bw, h->k, lmax) == 0;
  free(sel);
  free(bw);
  *rounds_out = rounds;
  *moved_out = moved;
  return balanced ? 0 : 1;
}

static void fill_final_stats(const jo_hg *h, const int32_t *part, int32_t deadzone_ppm, jo_stats *st) {
  int64_t A, lmax, dz;
  jo_limits(total_weight(h), h->k, h->eps, deadzone_ppm, &A, &lmax, &dz);
  int64_t *bw = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)h->k);
  jo_block_weights(h, part, bw);
  int64_t mx = 0;
  for (int32_t b = 0; b < h->k; ++b)
    if (bw[b] > mx) mx = bw[b];
  st->km1_out = jo_km1(h, part);
  st->lmax = lmax;
  st->max_block_weight = mx;
  st->balanced = mx <= lmax;
  free(bw);
}

int jo_rebalance(const jo_hg *h, int32_t *part, const jo_params *prm, jo_stats *st) {
  jo_stats local;
  memset(&local, 0, sizeof local);
  local.km1_in = jo_km1(h, part);
  int32_t rounds, moved;
  int rc = rebalance_rounds(h, part, prm->deadzone_ppm, prm->rb_unweighted, prm->max_rebalance_rounds, &rounds,
                            &moved);
  local.rebalance_rounds = rounds;
  fill_final_stats(h, part, prm->deadzone_ppm, &local);
  if (st) *st = local;
  return rc;
}

/* ------------------------------------------------------------------ Algorithm 1: the Jet loop */

/* Readings of Algorithm 1 and Section 4.1:
 *  - quality of a partition is the pair (overload, metric), overload = max(0, max_b bw[b] - Lmax),
 *    compared lexicographically; "improved" means strictly better than the best seen so far;
 *  - rollback: the best partition seen is kept and returned at the end of a temperature round;
 *  - locking: a vertex moved by the afterburner-filtered moves of one iteration is not a candidate
 *    in the next iteration only; rebalancing moves do not lock; locks are cleared at the start of
 *    every temperature round;
 *  - several temperatures run as consecutive rounds, each starting from the previous round's best;
 *  - an iteration that moves nothing, rebalances nothing and started with no locked vertex leaves
 *    the state exactly as it found it, so all further iterations of the round would repeat it: the
 *    round ends there (the result is the same as running out the remaining iterations). */
int jo_refine(const jo_hg *h, int32_t *part, const jo_params *prm, jo_stats *st, jo_trace *trace,
              int32_t trace_cap, int32_t *trace_len) {
  const int32_t n = h->n, k = h->k;
  int64_t A, lmax, dz;
  jo_limits(total_weight(h), k, h->eps, prm->deadzone_ppm, &A, &lmax, &dz);
  jo_stats S;
  memset(&S, 0, sizeof S);
  S.km1_in = jo_km1(h, part);
  incidence I = build_incidence(h);
  int32_t *phi = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)h->m * (size_t)k);
  int32_t *t = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
  int32_t *g = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
  int32_t *rg = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
  uint8_t *inM = (uint8_t *)xmalloc((size_t)n);
  uint8_t *lock = (uint8_t *)xmalloc((size_t)n);
  int32_t *best = (int32_t *)xmalloc(sizeof(int32_t) * (size_t)n);
  int64_t *bw = (int64_t *)xmalloc(sizeof(int64_t) * (size_t)k);
  int32_t ntrace = 0;
  for (int32_t r = 0; r < prm->num_tau; ++r) {
    const int32_t tau_q = jo_quantize_tau(prm->tau[r]);
    S.tau_q_used[r] = tau_q;
    memset(lock, 0, (size_t)n);
    int lock_any = 0;
    memcpy(best, part, sizeof(int32_t) * (size_t)n);
    jo_block_weights(h, part, bw);
    int64_t best_ovl = overload_of(bw, k, lmax), best_km1 = jo_km1(h, part);
    int32_t round = 0, it = 0;
    while (round < prm->limit && it < prm->max_iters) {
      jo_phi(h, part, phi);
      candidates_with(h, &I, phi, part, lock, tau_q, t, g, inM, NULL, 0);
      afterburner_with(h, phi, part, t, g, inM, rg);
      int32_t ncand = 0, nmoved = 0;
      const int lock_was_any = lock_any;
      for (int32_t v = 0; v < n; ++v) { /* the kept moves X = {v in M : rg[v] > 0} */
        ncand += inM[v];
        lock[v] = 0;
        if (inM[v] && rg[v] > 0) {
          part[v] = t[v];
          lock[v] = 1;
          ++nmoved;
        }
      }
      lock_any = nmoved > 0;
      int32_t rb_rounds = 0, rb_moved = 0;
      jo_block_weights(h, part, bw);
      if (overload_of(bw, k, lmax) > 0)
        (void)rebalance_rounds(h, part, prm->deadzone_ppm, prm->rb_unweighted, prm->max_rebalance_rounds,
                               &rb_rounds, &rb_moved);
      it += 1;
      round += 1;
      jo_block_weights(h, part, bw);
      const int64_t ovl = overload_of(bw, k, lmax), km1 = jo_km1(h, part);
      if (ovl < best_ovl || (ovl == best_ovl && km1 < best_km1)) {
        best_ovl = ovl;
        best_km1 = km1;
        memcpy(best, part, sizeof(int32_t) * (size_t)n);
        round = 0;
      }
      S.iterations += 1;
      S.moves_executed += nmoved;
      S.rebalance_rounds += rb_rounds;
      if (trace && ntrace < trace_cap) {
        trace[ntrace].km1 = km1;
        trace[ntrace].overload = ovl;
        trace[ntrace].n_cand = ncand;
        trace[ntrace].n_moved = nmoved;
        trace[ntrace].rb_rounds = rb_rounds;
        trace[ntrace].rb_moved = rb_moved;
      }
      ++ntrace;
      if (nmoved == 0 && rb_moved == 0 && !lock_was_any) break;
    }
    memcpy(part, best, sizeof(int32_t) * (size_t)n);
  }
  fill_final_stats(h, part, prm->deadzone_ppm, &S);
  if (st) *st = S;
  if (trace_len) *trace_len = ntrace;
  free(bw);
  free(best);
  free(lock);
  free(inM);
  free(rg);
  free(g);
  free(t);
  free(phi);
  free_incidence(&I);
  return S.balanced ? 0 : 1;
}

/* ------------------------------------------------------------------ exhaustive 2-way optimum */

int64_t jo_bruteforce_2way(const jo_hg *h) {
  if (h->n > 24 || h->n < 1) return -1;
  const int32_t n = h->n;
  int64_t A, lmax, dz;
  jo_limits(total_weight(h), 2, h->eps, 0, &A, &lmax, &dz);
  uint32_t *netmask = (uint32_t *)xcalloc((size_t)h->m, sizeof(uint32_t));
  for (int32_t e = 0; e < h->m; ++e)
    for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) netmask[e] |= 1u << h->pins[q];
  int64_t best = -1;
  const uint32_t full = (n == 32) ? 0xFFFFFFFFu : ((1u << n) - 1u);
  for (uint32_t x = 0; x <= full; ++x) { /* bit v set: v in block 1 */
    int64_t w1 = 0, w0 = 0;
    for (int32_t v = 0; v < n; ++v) {
      if (x >> v & 1u) w1 += w_vtx(h, v); else w0 += w_vtx(h, v);
    }
    if (w0 <= lmax && w1 <= lmax) {
      int64_t cost = 0;
      for (int32_t e = 0; e < h->m; ++e) {
        const int in1 = (netmask[e] & x) != 0, in0 = (netmask[e] & ~x & full) != 0;
        if (in0 && in1) cost += w_net(h, e);
      }
      if (best < 0 || cost < best) best = cost;
    }
    if (x == full) break;
  }
  free(netmask);
  return best;
}
