/*
 * flow_oracle.c -- plain single-threaded CPU oracle for deterministic flow-based refinement
 * (Section 5): two-way refinement of a block pair by incremental bipartitioning (Algorithm 3) and
 * the k-way matching schedule of block pairs (Section 5.2).
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists to check the GPU library.  It shares no source,
 * header, table or helper with it.
 *
 * The flows run on the Lawler network of the pair's induced subhypergraph, built once per pair with
 * the initial terminal sets contracted into one source s and one sink t:
 *   nodes  s, t, one node per free vertex, and per net e two nodes e_in, e_out;
 *   arcs   x -> e_in and e_out -> x of capacity INF for every endpoint x of e (a free vertex, s if
 *          a pin of e is a source terminal, t if one is a sink terminal), e_in -> e_out of
 *          capacity w(e).
 * A net with fewer than two distinct endpoints can never be cut and is left out.  INF is one more
 * than the sum of the net weights in the network, so no minimum cut uses an INF arc, and minimum
 * s-t cuts are exactly the hypergraph cuts of least weight.  Terminals added by piercing are flags
 * on the network's nodes (a side takes every node it reaches, net nodes included), and after every
 * change the flow is augmented along shortest paths from any source node to any sink node until
 * none is left (Ford and Fulkerson), which gives a maximum flow for the new terminal sets.
 *
 * From a maximum flow the two bipartitions of Algorithm 3 are the vertices reachable from s in
 * the residual network (S_r, the inclusion-minimal source side) and the vertices that reach t
 * (T_r, the inclusion-minimal sink side).  Both are the same for every maximum flow (Section 5.1),
 * which is what lets any correct flow algorithm stand in for the paper's.
 *
 * Readings where the paper defers to earlier work (each is stated again in the design notes):
 *   F1 region: breadth-first levels from the pair's boundary, inside one block, through any net;
 *      whole levels while their weight fits, then the next level's vertices in increasing ID
 *      while they fit, then stop.  The weight bound of block a's side is
 *      min(floor((1 + alpha eps) A) - c(V_b), c(V_a) - 1), A = ceil(c(V)/k), at least 0 (a side
 *      never takes its whole block, so both terminal sets start non-empty); b's side symmetric.
 *   F2 piercing: the smaller side (c(S_r) <= c(T_r) picks the source side) absorbs its reachable
 *      set; the piercing vertex is a free vertex outside it that is a pin of a net cut by it,
 *      preferring vertices outside the other side's reachable set, then the smallest ID.
 *   F3 result: when one of the two bipartitions is balanced (both blocks within Lmax) the loop
 *      ends with it (if both are, the one whose heavier block is lighter, then the source side's);
 *      it replaces the pair if its cut is smaller, or equal with a lighter heavier block.  The
 *      loop also ends, before piercing, once the flow reaches the pair's old cut (Section 5.1,
 *      "Termination Checks"), or when no piercing vertex is left.
 *   F4 schedule: rounds over the quotient graph's edges with an active endpoint (all blocks active
 *      in the first round); in each round maximal matchings are refined one after the other until
 *      every edge of the round is scheduled: blocks are visited by decreasing remaining degree
 *      (then ID) and matched to the unmatched neighbour of highest remaining degree (then lowest
 *      ID).  A block is active in the next round if a pair with it lowered its cut.  The pairs of
 *      one matching are disjoint, so their order does not change the result.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "jet_oracle.h"

static void *xcalloc(size_t cnt, size_t sz) {
  void *p = calloc(cnt ? cnt : 1, sz ? sz : 1);
  if (!p) abort();
  return p;
}

static inline int64_t c_of(const jo_hg *h, int32_t v) { return h->vw ? (int64_t)h->vw[v] : 1; }
static inline int64_t w_of(const jo_hg *h, int32_t e) { return h->nw ? (int64_t)h->nw[e] : 1; }

/* ---- the flow network ---- */

typedef struct {
  int32_t nodes, arcs, cap_arcs;
  int32_t *head;   /* [arcs] */
  int64_t *res;    /* [arcs] residual capacity */
  int32_t *nxt;    /* [arcs] next arc out of the same tail (adjacency lists) */
  int32_t *first;  /* [nodes] first arc out of the node, -1 if none */
} net_t;

static void add_arc(net_t *g, int32_t u, int32_t v, int64_t cap) {
  if (g->arcs + 2 > g->cap_arcs) {
    g->cap_arcs = g->cap_arcs ? 2 * g->cap_arcs : 64;
    g->head = (int32_t *)realloc(g->head, sizeof(int32_t) * (size_t)g->cap_arcs);
    g->res = (int64_t *)realloc(g->res, sizeof(int64_t) * (size_t)g->cap_arcs);
    g->nxt = (int32_t *)realloc(g->nxt, sizeof(int32_t) * (size_t)g->cap_arcs);
    if (!g->head || !g->res || !g->nxt) abort();
  }
  /* arc 2i is u -> v, arc 2i + 1 its reverse */
  int32_t a = g->arcs++;
  g->head[a] = v;
  g->res[a] = cap;
  g->nxt[a] = g->first[u];
  g->first[u] = a;
  a = g->arcs++;
  g->head[a] = u;
  g->res[a] = 0;
  g->nxt[a] = g->first[v];
  g->first[v] = a;
}

static void free_net(net_t *g) {
  free(g->head);
  free(g->res);
  free(g->nxt);
  free(g->first);
}

/* term[v] for the vertices of blocks a and b: 0 free, 1 source terminal, 2 sink terminal.
 * node_of[v]: network node of a free vertex (2..), 0 for a source terminal, 1 for a sink one, -1
 * outside the pair.  Returns the network. */
static net_t build_network(const jo_hg *h, const int32_t *part, int32_t a, int32_t b, const int8_t *term,
                           int32_t *node_of) {
  int32_t nfree = 0;
  for (int32_t v = 0; v < h->n; ++v) {
    if (part[v] != a && part[v] != b) {
      node_of[v] = -1;
      continue;
    }
    node_of[v] = term[v] == 1 ? 0 : term[v] == 2 ? 1 : 2 + nfree++;
  }
  /* nets with two or more distinct endpoints, and the sum of their weights */
  int32_t relevant = 0;
  int64_t wsum = 0;
  uint8_t *keep = (uint8_t *)xcalloc((size_t)h->m, 1);
  for (int32_t e = 0; e < h->m; ++e) {
    int32_t ends = 0, has_s = 0, has_t = 0;
    for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) {
      const int32_t x = node_of[h->pins[q]];
      if (x < 0) continue;
      if (x == 0) has_s = 1;
      else if (x == 1) has_t = 1;
      else ++ends;
    }
    ends += has_s + has_t;
    if (ends >= 2) {
      keep[e] = 1;
      ++relevant;
      wsum += w_of(h, e);
    }
  }
  net_t g;
  memset(&g, 0, sizeof g);
  g.nodes = 2 + nfree + 2 * relevant;
  g.first = (int32_t *)xcalloc((size_t)g.nodes, sizeof(int32_t));
  for (int32_t i = 0; i < g.nodes; ++i) g.first[i] = -1;
  const int64_t INF = wsum + 1;
  int32_t next_node = 2 + nfree;
  for (int32_t e = 0; e < h->m; ++e) {
    if (!keep[e]) continue;
    const int32_t ein = next_node++, eout = next_node++;
    add_arc(&g, ein, eout, w_of(h, e));
    int32_t did_s = 0, did_t = 0;
    for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) {
      const int32_t x = node_of[h->pins[q]];
      if (x < 0) continue;
      if (x == 0) {
        if (did_s) continue;
        did_s = 1;
      } else if (x == 1) {
        if (did_t) continue;
        did_t = 1;
      }
      add_arc(&g, x, ein, INF);
      add_arc(&g, eout, x, INF);
    }
  }
  free(keep);
  return g;
}

/* Augments the flow along shortest paths from any source node (nterm 1) to any sink node
 * (nterm 2) until none is left; returns the flow added.  Started from any feasible flow this
 * ends with a maximum flow for these terminal sets (Ford and Fulkerson). */
static int64_t augment(net_t *g, const uint8_t *nterm) {
  int32_t *prev_arc = (int32_t *)xcalloc((size_t)g->nodes, sizeof(int32_t));
  int32_t *queue = (int32_t *)xcalloc((size_t)g->nodes, sizeof(int32_t));
  int64_t flow = 0;
  for (;;) {
    int32_t qh = 0, qt = 0, hit = -1;
    for (int32_t i = 0; i < g->nodes; ++i) {
      prev_arc[i] = -2;
      if (nterm[i] == 1) {
        prev_arc[i] = -1;
        queue[qt++] = i;
      }
    }
    while (qh < qt && hit < 0) {
      const int32_t u = queue[qh++];
      for (int32_t a = g->first[u]; a >= 0; a = g->nxt[a]) {
        const int32_t v = g->head[a];
        if (g->res[a] > 0 && prev_arc[v] == -2) {
          prev_arc[v] = a;
          if (nterm[v] == 2) {
            hit = v;
            break;
          }
          queue[qt++] = v;
        }
      }
    }
    if (hit < 0) break;
    int64_t bott = INT64_MAX;
    for (int32_t v = hit; prev_arc[v] >= 0; v = g->head[prev_arc[v] ^ 1])
      if (g->res[prev_arc[v]] < bott) bott = g->res[prev_arc[v]];
    for (int32_t v = hit; prev_arc[v] >= 0; v = g->head[prev_arc[v] ^ 1]) {
      g->res[prev_arc[v]] -= bott;
      g->res[prev_arc[v] ^ 1] += bott;
    }
    flow += bott;
  }
  free(prev_arc);
  free(queue);
  return flow;
}

/* nodes reachable from a source node (forward) or reaching a sink node (backward) in the
 * residual network */
static void reach_from_sources(const net_t *g, const uint8_t *nterm, uint8_t *reach) {
  int32_t *queue = (int32_t *)xcalloc((size_t)g->nodes, sizeof(int32_t));
  int32_t qh = 0, qt = 0;
  for (int32_t i = 0; i < g->nodes; ++i) {
    reach[i] = nterm[i] == 1;
    if (reach[i]) queue[qt++] = i;
  }
  while (qh < qt) {
    const int32_t u = queue[qh++];
    for (int32_t a = g->first[u]; a >= 0; a = g->nxt[a])
      if (g->res[a] > 0 && !reach[g->head[a]]) {
        reach[g->head[a]] = 1;
        queue[qt++] = g->head[a];
      }
  }
  free(queue);
}

static void reach_to_sinks(const net_t *g, const uint8_t *nterm, uint8_t *reach) {
  int32_t *queue = (int32_t *)xcalloc((size_t)g->nodes, sizeof(int32_t));
  int32_t qh = 0, qt = 0;
  for (int32_t i = 0; i < g->nodes; ++i) {
    reach[i] = nterm[i] == 2;
    if (reach[i]) queue[qt++] = i;
  }
  while (qh < qt) {
    const int32_t v = queue[qh++];
    /* arc a = v -> u; its reverse a ^ 1 = u -> v has residual res[a ^ 1] */
    for (int32_t a = g->first[v]; a >= 0; a = g->nxt[a]) {
      const int32_t u = g->head[a];
      if (g->res[a ^ 1] > 0 && !reach[u]) {
        reach[u] = 1;
        queue[qt++] = u;
      }
    }
  }
  free(queue);
}

static uint8_t *contracted_terminals(const net_t *g) {
  uint8_t *nterm = (uint8_t *)xcalloc((size_t)g->nodes, 1);
  nterm[0] = 1;
  nterm[1] = 2;
  return nterm;
}

/* Maximum flow and both reachable sets for the given terminals (term as in build_network).
 * in_sr[v] / in_tr[v] for the vertices of the pair (terminals included).  Returns the flow. */
int64_t jo_flow_mincut(const jo_hg *h, const int32_t *part, int32_t a, int32_t b, const int8_t *term,
                       uint8_t *in_sr, uint8_t *in_tr) {
  int32_t *node_of = (int32_t *)xcalloc((size_t)h->n, sizeof(int32_t));
  net_t g = build_network(h, part, a, b, term, node_of);
  uint8_t *nterm = contracted_terminals(&g);
  const int64_t F = augment(&g, nterm);
  uint8_t *rs = (uint8_t *)xcalloc((size_t)g.nodes, 1);
  uint8_t *rt = (uint8_t *)xcalloc((size_t)g.nodes, 1);
  reach_from_sources(&g, nterm, rs);
  reach_to_sinks(&g, nterm, rt);
  for (int32_t v = 0; v < h->n; ++v) {
    const int32_t x = node_of[v];
    in_sr[v] = x >= 0 && rs[x];
    in_tr[v] = x >= 0 && rt[x];
  }
  free(rs);
  free(rt);
  free(nterm);
  free(node_of);
  free_net(&g);
  return F;
}

/* ---- region (reading F1) ---- */

static int64_t total_weight(const jo_hg *h) {
  int64_t W = 0;
  for (int32_t v = 0; v < h->n; ++v) W += c_of(h, v);
  return W;
}

/* incidence lists of the vertices, nets in increasing order */
static void incidence(const jo_hg *h, int64_t **voff_out, int32_t **inc_out) {
  int64_t *voff = (int64_t *)xcalloc((size_t)h->n + 1, sizeof(int64_t));
  int32_t *inc = (int32_t *)xcalloc((size_t)h->p, sizeof(int32_t));
  for (int64_t q = 0; q < h->p; ++q) voff[h->pins[q] + 1] += 1;
  for (int32_t v = 0; v < h->n; ++v) voff[v + 1] += voff[v];
  int64_t *fill = (int64_t *)xcalloc((size_t)h->n, sizeof(int64_t));
  for (int32_t e = 0; e < h->m; ++e)
    for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) {
      const int32_t v = h->pins[q];
      inc[voff[v] + fill[v]++] = e;
    }
  free(fill);
  *voff_out = voff;
  *inc_out = inc;
}

/* The region of block `side` toward block `other`: in_region[v] = 1 for its vertices.  Returns
 * the number of vertices taken. */
static int32_t grow_region(const jo_hg *h, const int32_t *part, const int64_t *voff, const int32_t *inc,
                           int32_t side, int32_t other, int64_t bound, uint8_t *in_region) {
  const int32_t n = h->n;
  uint8_t *seen = (uint8_t *)xcalloc((size_t)n, 1);
  uint8_t *cur = (uint8_t *)xcalloc((size_t)n, 1);  /* the current level, as flags over the IDs */
  /* level 0: vertices of `side` with a net that has a pin in `other` */
  int32_t in_level = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (part[v] != side) continue;
    for (int64_t q = voff[v]; q < voff[v + 1] && !cur[v]; ++q) {
      const int32_t e = inc[q];
      for (int64_t r = h->off[e]; r < h->off[e + 1]; ++r)
        if (part[h->pins[r]] == other) {
          cur[v] = 1;
          break;
        }
    }
    if (cur[v]) {
      seen[v] = 1;
      ++in_level;
    }
  }
  int64_t used = 0;
  int32_t taken = 0;
  int stop = 0;
  while (in_level > 0 && !stop) {
    int64_t lw = 0;
    for (int32_t v = 0; v < n; ++v)
      if (cur[v]) lw += c_of(h, v);
    if (used + lw <= bound) {
      for (int32_t v = 0; v < n; ++v)
        if (cur[v]) {
          in_region[v] = 1;
          ++taken;
        }
      used += lw;
    } else {  /* the level in increasing ID while it fits, then stop */
      for (int32_t v = 0; v < n; ++v) {
        if (!cur[v]) continue;
        if (used + c_of(h, v) > bound) break;
        used += c_of(h, v);
        in_region[v] = 1;
        ++taken;
      }
      stop = 1;
      break;
    }
    /* next level: unseen vertices of `side` sharing a net with the current level */
    uint8_t *nxt = (uint8_t *)xcalloc((size_t)n, 1);
    in_level = 0;
    for (int32_t u = 0; u < n; ++u) {
      if (!cur[u]) continue;
      for (int64_t q = voff[u]; q < voff[u + 1]; ++q) {
        const int32_t e = inc[q];
        for (int64_t r = h->off[e]; r < h->off[e + 1]; ++r) {
          const int32_t x = h->pins[r];
          if (part[x] == side && !seen[x]) {
            seen[x] = 1;
            nxt[x] = 1;
            ++in_level;
          }
        }
      }
    }
    free(cur);
    cur = nxt;
  }
  free(seen);
  free(cur);
  return taken;
}

static void pair_limits(const jo_hg *h, int32_t alpha, int64_t *A, int64_t *lmax, int64_t *big) {
  int64_t dz;
  jo_limits(total_weight(h), h->k, h->eps, 0, A, lmax, &dz);
  *big = (int64_t)floor((1.0 + (double)alpha * h->eps) * (double)*A);
}

int32_t jo_flow_region(const jo_hg *h, const int32_t *part, int32_t a, int32_t b, int32_t alpha,
                       int8_t *region) {
  if (a < 0 || b < 0 || a >= h->k || b >= h->k || a == b || alpha < 0) return -1;
  int64_t *voff;
  int32_t *inc;
  incidence(h, &voff, &inc);
  int64_t *bw = (int64_t *)xcalloc((size_t)h->k, sizeof(int64_t));
  jo_block_weights(h, part, bw);
  int64_t A, lmax, big;
  pair_limits(h, alpha, &A, &lmax, &big);
  uint8_t *ra = (uint8_t *)xcalloc((size_t)h->n, 1);
  uint8_t *rb = (uint8_t *)xcalloc((size_t)h->n, 1);
  int64_t bound_a = big - bw[b], bound_b = big - bw[a];
  /* a side never takes its whole block, so both terminal sets start non-empty */
  if (bound_a > bw[a] - 1) bound_a = bw[a] - 1;
  if (bound_b > bw[b] - 1) bound_b = bw[b] - 1;
  if (bound_a < 0) bound_a = 0;
  if (bound_b < 0) bound_b = 0;
  int32_t cnt = grow_region(h, part, voff, inc, a, b, bound_a, ra);
  cnt += grow_region(h, part, voff, inc, b, a, bound_b, rb);
  for (int32_t v = 0; v < h->n; ++v) region[v] = ra[v] ? 1 : rb[v] ? 2 : 0;
  free(ra);
  free(rb);
  free(bw);
  free(voff);
  free(inc);
  return cnt;
}

/* ---- two-way refinement (Algorithm 3) ---- */

/* Refines blocks a and b of part in place.  Returns 1 if the pair was replaced, 0 if not, -1 on a
 * bad argument. */
int32_t jo_flow_pair(const jo_hg *h, int32_t *part, int32_t a, int32_t b, int32_t alpha, jo_flow_pair_stats *st) {
  if (a < 0 || b < 0 || a >= h->k || b >= h->k || a == b || alpha < 0) return -1;
  const int32_t n = h->n;
  jo_flow_pair_stats s;
  memset(&s, 0, sizeof s);
  int64_t *bw = (int64_t *)xcalloc((size_t)h->k, sizeof(int64_t));
  jo_block_weights(h, part, bw);
  int64_t A, lmax, big;
  pair_limits(h, alpha, &A, &lmax, &big);
  /* the pair's induced cut */
  for (int32_t e = 0; e < h->m; ++e) {
    int ina = 0, inb = 0;
    for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) {
      ina |= part[h->pins[q]] == a;
      inb |= part[h->pins[q]] == b;
    }
    if (ina && inb) s.old_cut += w_of(h, e);
  }
  s.new_cut = s.old_cut;
  int32_t result = 0;
  if (s.old_cut > 0) {
    int8_t *region = (int8_t *)xcalloc((size_t)n, 1);
    jo_flow_region(h, part, a, b, alpha, region);
    /* the network once, with a \ R_a contracted into the source node and b \ R_b into the sink
     * node; later terminals are node flags, and the flow is augmented from the previous one */
    int8_t *term = (int8_t *)xcalloc((size_t)n, 1);
    for (int32_t v = 0; v < n; ++v) {
      if (part[v] == a) {
        term[v] = region[v] ? 0 : 1;
        s.region_a += region[v] != 0;
      } else if (part[v] == b) {
        term[v] = region[v] ? 0 : 2;
        s.region_b += region[v] != 0;
      }
    }
    int32_t *node_of = (int32_t *)xcalloc((size_t)n, sizeof(int32_t));
    net_t g = build_network(h, part, a, b, term, node_of);
    uint8_t *nterm = contracted_terminals(&g);
    uint8_t *rs = (uint8_t *)xcalloc((size_t)g.nodes, 1);
    uint8_t *rt = (uint8_t *)xcalloc((size_t)g.nodes, 1);
    uint8_t *sr = (uint8_t *)xcalloc((size_t)n, 1);
    uint8_t *tr = (uint8_t *)xcalloc((size_t)n, 1);
    const int64_t wab = bw[a] + bw[b];
    const int64_t heavier_old = bw[a] > bw[b] ? bw[a] : bw[b];
    int64_t F = 0;
    for (;;) {
      F += augment(&g, nterm);
      reach_from_sources(&g, nterm, rs);
      reach_to_sinks(&g, nterm, rt);
      ++s.iterations;
      if (F > s.old_cut) break;
      int64_t w1 = 0, w2 = 0;
      for (int32_t v = 0; v < n; ++v) {
        const int32_t x = node_of[v];
        sr[v] = x >= 0 && rs[x];
        tr[v] = x >= 0 && rt[x];
        if (sr[v]) w1 += c_of(h, v);
        if (tr[v]) w2 += c_of(h, v);
      }
      /* bipartition 1: (S_r, rest) with weights (w1, wab - w1); 2: (rest, T_r) with (wab - w2, w2) */
      const int64_t h1 = w1 > wab - w1 ? w1 : wab - w1;
      const int64_t h2 = w2 > wab - w2 ? w2 : wab - w2;
      const int bal1 = w1 <= lmax && wab - w1 <= lmax;
      const int bal2 = w2 <= lmax && wab - w2 <= lmax;
      if (bal1 || bal2) {
        const int use1 = bal1 && (!bal2 || h1 <= h2);
        const int64_t hv = use1 ? h1 : h2;
        if (F < s.old_cut || hv < heavier_old) {
          for (int32_t v = 0; v < n; ++v) {
            if (part[v] != a && part[v] != b) continue;
            const int src = use1 ? sr[v] : !tr[v];
            const int32_t nb = src ? a : b;
            if (nb != part[v]) {
              part[v] = nb;
              ++s.moved;
            }
          }
          s.new_cut = F;
          result = 1;
        }
        break;
      }
      if (F >= s.old_cut) break;  /* the termination check comes before piercing */
      /* piercing (reading F2): the smaller side's reachable nodes become its terminals */
      const int source_side = w1 <= w2;
      const uint8_t side = source_side ? 1 : 2;
      const uint8_t *mine_node = source_side ? rs : rt;
      const uint8_t *mine = source_side ? sr : tr;
      const uint8_t *theirs = source_side ? tr : sr;
      for (int32_t u = 0; u < g.nodes; ++u)
        if (mine_node[u] && nterm[u] == 0) nterm[u] = side;
      int32_t best = -1, best_key = 0;
      for (int32_t e = 0; e < h->m; ++e) {
        int in_mine = 0, out_mine = 0;
        for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) {
          const int32_t x = h->pins[q];
          if (part[x] != a && part[x] != b) continue;
          if (mine[x]) in_mine = 1;
          else out_mine = 1;
        }
        if (!in_mine || !out_mine) continue;
        for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) {
          const int32_t x = h->pins[q];
          if ((part[x] != a && part[x] != b) || mine[x] || node_of[x] < 2 || nterm[node_of[x]] != 0) continue;
          const int32_t key = theirs[x] ? 1 : 0;
          if (best < 0 || key < best_key || (key == best_key && x < best)) {
            best = x;
            best_key = key;
          }
        }
      }
      if (best < 0) break;
      nterm[node_of[best]] = side;
    }
    free(sr);
    free(tr);
    free(rs);
    free(rt);
    free(nterm);
    free(node_of);
    free_net(&g);
    free(term);
    free(region);
  }
  free(bw);
  if (st) *st = s;
  return result;
}

/* ---- k-way schedule (reading F4) ---- */

int32_t jo_flow_refine(const jo_hg *h, int32_t *part, int32_t alpha, int32_t max_rounds, jo_flow_stats *st) {
  if (alpha < 0 || max_rounds < 0) return -1;
  const int32_t k = h->k;
  jo_flow_stats s;
  memset(&s, 0, sizeof s);
  s.km1_in = jo_km1(h, part);
  uint8_t *active = (uint8_t *)xcalloc((size_t)k, 1);
  uint8_t *next_active = (uint8_t *)xcalloc((size_t)k, 1);
  uint8_t *edge = (uint8_t *)xcalloc((size_t)k * (size_t)k, 1);
  uint8_t *seen_blk = (uint8_t *)xcalloc((size_t)k, 1);
  int32_t *deg = (int32_t *)xcalloc((size_t)k, sizeof(int32_t));
  int32_t *order = (int32_t *)xcalloc((size_t)k, sizeof(int32_t));
  int32_t *mate = (int32_t *)xcalloc((size_t)k, sizeof(int32_t));
  for (int32_t b = 0; b < k; ++b) active[b] = 1;
  for (int32_t round = 0; round < max_rounds; ++round) {
    /* quotient graph edges with an active endpoint, from the partition at the round's start */
    memset(edge, 0, (size_t)k * (size_t)k);
    int32_t remaining = 0;
    for (int32_t e = 0; e < h->m; ++e) {
      memset(seen_blk, 0, (size_t)k);
      for (int64_t q = h->off[e]; q < h->off[e + 1]; ++q) seen_blk[part[h->pins[q]]] = 1;
      for (int32_t i = 0; i < k; ++i) {
        if (!seen_blk[i]) continue;
        for (int32_t j = i + 1; j < k; ++j)
          if (seen_blk[j] && (active[i] || active[j]) && !edge[i * k + j]) {
            edge[i * k + j] = edge[j * k + i] = 1;
            ++remaining;
          }
      }
    }
    if (remaining == 0) break;
    ++s.rounds;
    memset(next_active, 0, (size_t)k);
    while (remaining > 0) {
      for (int32_t i = 0; i < k; ++i) {
        deg[i] = 0;
        for (int32_t j = 0; j < k; ++j) deg[i] += edge[i * k + j];
        order[i] = i;
        mate[i] = -1;
      }
      /* blocks by decreasing remaining degree, then increasing ID (insertion sort) */
      for (int32_t i = 1; i < k; ++i) {
        const int32_t x = order[i];
        int32_t j = i - 1;
        while (j >= 0 && (deg[order[j]] < deg[x] || (deg[order[j]] == deg[x] && order[j] > x))) {
          order[j + 1] = order[j];
          --j;
        }
        order[j + 1] = x;
      }
      for (int32_t oi = 0; oi < k; ++oi) {
        const int32_t i = order[oi];
        if (mate[i] >= 0 || deg[i] == 0) continue;
        int32_t best = -1;
        for (int32_t j = 0; j < k; ++j) {
          if (!edge[i * k + j] || mate[j] >= 0) continue;
          if (best < 0 || deg[j] > deg[best] || (deg[j] == deg[best] && j < best)) best = j;
        }
        if (best >= 0) {
          mate[i] = best;
          mate[best] = i;
        }
      }
      ++s.matchings;
      for (int32_t i = 0; i < k; ++i) {
        const int32_t j = mate[i];
        if (j < 0 || j < i) continue;
        edge[i * k + j] = edge[j * k + i] = 0;
        --remaining;
        jo_flow_pair_stats ps;
        const int32_t r = jo_flow_pair(h, part, i, j, alpha, &ps);
        ++s.pairs;
        s.flow_calls += ps.iterations;
        if (r == 1) {
          ++s.accepted;
          s.moved += ps.moved;
          if (ps.new_cut < ps.old_cut) next_active[i] = next_active[j] = 1;
        }
      }
    }
    int32_t any = 0;
    for (int32_t b = 0; b < k; ++b) {
      active[b] = next_active[b];
      any |= active[b];
    }
    if (!any) break;
  }
  s.km1_out = jo_km1(h, part);
  free(active);
  free(next_active);
  free(edge);
  free(seen_blk);
  free(deg);
  free(order);
  free(mate);
  if (st) *st = s;
  return 0;
}
