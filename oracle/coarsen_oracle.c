/*
 * coarsen_oracle.c -- plain, slow, single-threaded CPU oracle for the deterministic synchronous
 * clustering of the coarsening phase (Section 6, Algorithm 4 "Synchronous Coarsening").
 *
 * TEST INFRASTRUCTURE ONLY, like jet_oracle.c: it checks the GPU library and shares no code with it.
 *
 * What is computed, in the paper's order:
 *   - the vertices are split into sub-rounds B_1, B_2, ... taken from a caller-given vertex order
 *     with the prefix-doubling schedule of Section 6 (one vertex per sub-round for the first
 *     sub-rounds, then sizes doubling up to a limit of a fraction of n);
 *   - in a sub-round every vertex u of B_i that is still a singleton cluster proposes the target
 *     cluster of highest heavy-edge rating  sum over e in I(u) of w(e) [|e cap C| > 0] / (|e| - 1),
 *     each net counted once per cluster (the corrected rating of Section 6);
 *   - pairs proposing each other are merged toward the heavier side (vertex-swap prevention);
 *   - proposals are grouped by target, each group sorted by (weight, ID), prefix-summed and cut by
 *     a binary search at the room left in the target cluster; the prefix moves.
 *
 * Readings where the text leaves a choice open (each is also stated at its use):
 *   R1  ratings are compared in fixed point: a net contributes floor(w(e) 2^32 / (|e| - 1)) and the
 *       sums are exact 64-bit integers, so the argmax does not depend on summation order;
 *   R2  the "loose weight constraint" of the proposal: a cluster C is a candidate only if its weight
 *       at the start of the sub-round plus c(u) is at most the maximum cluster weight;
 *   R3  among equal ratings the smallest cluster label wins;
 *   R4  clusters are labelled by the vertex that started them; a vertex is a singleton when it
 *       carries its own label and its cluster weighs exactly c(u); only singletons propose;
 *   R5  swap prevention: for u < v with T[u] = v and T[v] = u, each side's weight is its own plus
 *       the weights of the other vertices of B_i proposing it; the heavier side (u on a tie) keeps
 *       its place (T = itself) and the other one joins it;
 *   R6  a vertex whose target is itself does not move; approval uses each cluster's weight at the
 *       start of the sub-round; all moves of a sub-round are applied after all approvals;
 *   R7  schedule: the first `initial_single` sub-rounds hold one vertex each, then sizes 2, 4, 8, ...
 *       up to max(1, floor(n / cap_div)), after which every sub-round has that size (the last one
 *       takes what is left).
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "jet_oracle.h"

static inline int64_t c_of(const jo_hg *h, int32_t v) { return h->vw ? (int64_t)h->vw[v] : 1; }
static inline int64_t w_of(const jo_hg *h, int32_t e) { return h->nw ? (int64_t)h->nw[e] : 1; }

static void *xalloc(size_t cnt, size_t sz) {
  void *p = calloc(cnt ? cnt : 1, sz ? sz : 1);
  if (!p) abort();
  return p;
}

int64_t jo_coarsen_schedule(int32_t n, int32_t initial_single, int32_t cap_div, int32_t *sizes, int64_t max_sizes) {
  if (n < 0 || initial_single < 0 || cap_div < 1) return -1;
  const int64_t cap = n / cap_div > 1 ? n / cap_div : 1;  /* R7 */
  int64_t s = 0, i = 0;
  int64_t len = 1;
  while (s < n) {
    if (i < initial_single) {
      len = 1;
    } else if (i == initial_single) {
      len = 2 < cap ? 2 : cap;
    } else {
      len = 2 * len < cap ? 2 * len : cap;
    }
    if (len > n - s) len = n - s;
    if (sizes && i < max_sizes) sizes[i] = (int32_t)len;
    s += len;
    ++i;
  }
  return i;
}

/* incident nets of every vertex, nets ascending */
static void incidence_lists(const jo_hg *h, int64_t **voff_out, int32_t **inc_out) {
  int64_t *voff = (int64_t *)xalloc((size_t)h->n + 1, sizeof(int64_t));
  int32_t *inc = (int32_t *)xalloc((size_t)h->p, sizeof(int32_t));
  for (int64_t q = 0; q < h->p; ++q) voff[h->pins[q] + 1] += 1;
  for (int32_t v = 0; v < h->n; ++v) voff[v + 1] += voff[v];
  int64_t *cur = (int64_t *)xalloc((size_t)h->n + 1, sizeof(int64_t));
  memcpy(cur, voff, sizeof(int64_t) * ((size_t)h->n + 1));
  for (int32_t e = 0; e < h->m; ++e)
    for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) inc[cur[h->pins[q]]++] = e;
  free(cur);
  *voff_out = voff;
  *inc_out = inc;
}

typedef struct {
  int32_t target, vertex;
  int64_t weight;
} proposal;

/* group-by target, then increasing weight and ID (Algorithm 4: sort M[j]) */
static int cmp_proposal(const void *a, const void *b) {
  const proposal *x = (const proposal *)a, *y = (const proposal *)b;
  if (x->target != y->target) return x->target < y->target ? -1 : 1;
  if (x->weight != y->weight) return x->weight < y->weight ? -1 : 1;
  return (x->vertex > y->vertex) - (x->vertex < y->vertex);
}

/* One sub-round on the clustering (label, cw); voff/inc the incidence lists; scratch arrays of n
 * entries: rating (zero), seen (-1), join (zero), touched.  Returns the number of moved vertices. */
static int32_t subround(const jo_hg *h, const int64_t *voff, const int32_t *inc, int32_t *label, int64_t *cw,
                        const int32_t *B, int32_t nb, int64_t wmax, int32_t *T, uint64_t *rating, int32_t *seen,
                        int64_t *join, int32_t *touched) {
  for (int32_t x = 0; x < h->n; ++x) T[x] = -1;
  /* targets: the highest rated neighbouring cluster of every singleton u of B_i */
  for (int32_t i = 0; i < nb; ++i) {
    const int32_t u = B[i];
    if (label[u] != u || cw[u] != c_of(h, u)) continue; /* R4: not a singleton any more */
    int32_t nt = 0;
    for (int64_t j = voff[u]; j < voff[u + 1]; ++j) {
      const int32_t e = inc[j];
      const int64_t size = h->off[e + 1] - h->off[e];
      if (size < 2) continue;
      const uint64_t q = ((uint64_t)w_of(h, e) << 32) / (uint64_t)(size - 1); /* R1 */
      for (int64_t r = h->off[e]; r < h->off[e + 1]; ++r) {
        const int32_t x = h->pins[r];
        if (x == u) continue;
        const int32_t C = label[x];
        if (seen[C] == e) continue; /* the net counts once for cluster C */
        if (seen[C] == -1) touched[nt++] = C;
        seen[C] = e;
        rating[C] += q;
      }
    }
    int32_t best = -1;
    for (int32_t t = 0; t < nt; ++t) {
      const int32_t C = touched[t];
      if (cw[C] + c_of(h, u) <= wmax) { /* R2 */
        if (best < 0 || rating[C] > rating[best] || (rating[C] == rating[best] && C < best)) best = C; /* R3 */
      }
    }
    for (int32_t t = 0; t < nt; ++t) {
      rating[touched[t]] = 0;
      seen[touched[t]] = -1;
    }
    T[u] = best;
  }
  /* vertex-swap prevention (R5), decided on the proposals before any change */
  for (int32_t i = 0; i < nb; ++i) {
    const int32_t y = B[i];
    if (T[y] >= 0) join[T[y]] += c_of(h, y);
  }
  int32_t *stay = (int32_t *)xalloc((size_t)nb, sizeof(int32_t));
  int32_t ns = 0;
  for (int32_t i = 0; i < nb; ++i) {
    const int32_t u = B[i], v = T[u];
    if (v < 0 || v <= u || T[v] != u) continue;
    const int64_t wu = c_of(h, u) + join[u] - c_of(h, v);
    const int64_t wv = c_of(h, v) + join[v] - c_of(h, u);
    stay[ns++] = wu >= wv ? u : v;
  }
  for (int32_t i = 0; i < nb; ++i)
    if (T[B[i]] >= 0) join[T[B[i]]] = 0;
  for (int32_t i = 0; i < ns; ++i) T[stay[i]] = stay[i];
  free(stay);
  /* group-by target, sort, prefix sum, binary search, move (R6) */
  proposal *P = (proposal *)xalloc((size_t)nb, sizeof(proposal));
  int32_t np = 0;
  for (int32_t i = 0; i < nb; ++i) {
    const int32_t x = B[i];
    if (T[x] >= 0 && T[x] != x) {
      P[np].target = T[x];
      P[np].vertex = x;
      P[np].weight = c_of(h, x);
      ++np;
    }
  }
  qsort(P, (size_t)np, sizeof(proposal), cmp_proposal);
  int64_t *W = (int64_t *)xalloc((size_t)np + 1, sizeof(int64_t));
  proposal *moves = (proposal *)xalloc((size_t)np, sizeof(proposal));
  int32_t nm = 0;
  for (int32_t a = 0; a < np;) {
    int32_t b = a;
    while (b < np && P[b].target == P[a].target) ++b;
    const int32_t j = P[a].target;
    /* W[l] = weight of the first l members */
    W[0] = 0;
    for (int32_t l = 0; l < b - a; ++l) W[l + 1] = W[l] + P[a + l].weight;
    /* pos = largest l with W[l] <= room (W is increasing, W[0] = 0 fits when room >= 0) */
    const int64_t room = wmax - cw[j];
    int32_t lo = 0, hi = b - a;
    if (room < 0) {
      hi = 0;
    } else {
      while (lo < hi) {
        const int32_t mid = lo + (hi - lo + 1) / 2;
        if (W[mid] <= room) lo = mid;
        else hi = mid - 1;
      }
    }
    for (int32_t l = 0; l < lo; ++l) moves[nm++] = P[a + l];
    a = b;
  }
  for (int32_t i = 0; i < nm; ++i) {
    label[moves[i].vertex] = moves[i].target;
    cw[moves[i].target] += moves[i].weight;
    cw[moves[i].vertex] -= moves[i].weight;
  }
  free(P);
  free(W);
  free(moves);
  return nm;
}

static int valid_order(const int32_t *order, int32_t n) {
  uint8_t *hit = (uint8_t *)xalloc((size_t)n, 1);
  int ok = 1;
  for (int32_t i = 0; i < n && ok; ++i) {
    if (order[i] < 0 || order[i] >= n || hit[order[i]]) ok = 0;
    else hit[order[i]] = 1;
  }
  free(hit);
  return ok;
}

int32_t jo_coarsen_subround(const jo_hg *h, int32_t *label, int64_t *cw, const int32_t *B, int32_t nb, int64_t wmax,
                            int32_t *T) {
  int64_t *voff;
  int32_t *inc;
  incidence_lists(h, &voff, &inc);
  uint64_t *rating = (uint64_t *)xalloc((size_t)h->n, sizeof(uint64_t));
  int32_t *seen = (int32_t *)xalloc((size_t)h->n, sizeof(int32_t));
  int64_t *join = (int64_t *)xalloc((size_t)h->n, sizeof(int64_t));
  int32_t *touched = (int32_t *)xalloc((size_t)h->n, sizeof(int32_t));
  for (int32_t x = 0; x < h->n; ++x) seen[x] = -1;
  const int32_t moved = subround(h, voff, inc, label, cw, B, nb, wmax, T, rating, seen, join, touched);
  free(voff);
  free(inc);
  free(rating);
  free(seen);
  free(join);
  free(touched);
  return moved;
}

int32_t jo_coarsen(const jo_hg *h, const int32_t *order, int64_t wmax, int32_t initial_single, int32_t cap_div,
                   int32_t *label) {
  if (!valid_order(order, h->n)) return -1;
  const int64_t rounds = jo_coarsen_schedule(h->n, initial_single, cap_div, NULL, 0);
  if (rounds < 0) return -1;
  int32_t *sizes = (int32_t *)xalloc((size_t)rounds, sizeof(int32_t));
  jo_coarsen_schedule(h->n, initial_single, cap_div, sizes, rounds);
  int64_t *voff;
  int32_t *inc;
  incidence_lists(h, &voff, &inc);
  int64_t *cw = (int64_t *)xalloc((size_t)h->n, sizeof(int64_t));
  uint64_t *rating = (uint64_t *)xalloc((size_t)h->n, sizeof(uint64_t));
  int32_t *seen = (int32_t *)xalloc((size_t)h->n, sizeof(int32_t));
  int64_t *join = (int64_t *)xalloc((size_t)h->n, sizeof(int64_t));
  int32_t *touched = (int32_t *)xalloc((size_t)h->n, sizeof(int32_t));
  int32_t *T = (int32_t *)xalloc((size_t)h->n, sizeof(int32_t));
  for (int32_t v = 0; v < h->n; ++v) {
    label[v] = v; /* every vertex starts as a singleton cluster */
    cw[v] = c_of(h, v);
    seen[v] = -1;
  }
  int64_t s = 0;
  for (int64_t i = 0; i < rounds; ++i) {
    subround(h, voff, inc, label, cw, order + s, sizes[i], wmax, T, rating, seen, join, touched);
    s += sizes[i];
  }
  uint8_t *used = (uint8_t *)xalloc((size_t)h->n, 1);
  int32_t clusters = 0;
  for (int32_t v = 0; v < h->n; ++v) {
    if (!used[label[v]]) ++clusters;
    used[label[v]] = 1;
  }
  free(used);
  free(sizes);
  free(voff);
  free(inc);
  free(cw);
  free(rating);
  free(seen);
  free(join);
  free(touched);
  free(T);
  return clusters;
}
