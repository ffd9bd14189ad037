/*
 * Multilevel starting points for the refinement benchmarks: a seeded random-matching hierarchy
 * (each level pairs vertices along nets, halving the vertex count), contraction of the nets, and a
 * seeded greedy balanced partition of the coarsest level.
 *
 * This is input construction only (the paper's own coarsening is not reproduced): it gives every
 * level a realistic projected partition to refine.  None of the refinement arithmetic is here.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct { uint64_t s; } hm64;

static inline uint64_t hm_next(hm64 *r) {
  uint64_t z = (r->s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static hm64 hm_stream(uint64_t seed, uint64_t id) {
  hm64 r;
  r.s = seed ^ (0x9E3779B97F4A7C15ULL * (id + 1));
  (void)hm_next(&r);
  return r;
}

static inline uint64_t hm_below(hm64 *r, uint64_t range) {
  uint64_t x = hm_next(r);
  __uint128_t mm = (__uint128_t)x * range;
  uint64_t lo = (uint64_t)mm;
  if (lo < range) {
    uint64_t thr = (0 - range) % range;
    while (lo < thr) {
      x = hm_next(r);
      mm = (__uint128_t)x * range;
      lo = (uint64_t)mm;
    }
  }
  return (uint64_t)(mm >> 64);
}

typedef struct {
  int32_t n, m;
  int64_t p;
  int64_t *off;
  int32_t *pins;
  int32_t *nw;  /* NULL if the fine level had unit net weights */
  int32_t *vw;
} coarse_hg;

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

static inline int64_t nx_find(int32_t *nx, int64_t q) {
  while (nx[q] != q) {
    nx[q] = nx[nx[q]];
    q = nx[q];
  }
  return q;
}

/* Contraction of a clustering: parent[v] in [0, nc) is v's coarse vertex.  Coarse weights are
 * sums; nets are mapped, deduplicated, single-pin nets dropped, parallel nets kept.  Every net is
 * mapped, sorted and deduplicated in place of its fine pins in a scratch copy (nets are
 * independent, so threads may take them in any order), then the kept nets are packed in net
 * order: the result is the same for any number of threads. */
static coarse_hg *contract(int32_t m, int64_t p, const int64_t *off, const int32_t *pins, const int32_t *nw,
                           const int32_t *vw, int32_t n, const int32_t *parent, int32_t nc) {
  coarse_hg *h = (coarse_hg *)calloc(1, sizeof(coarse_hg));
  h->n = nc;
  h->vw = (int32_t *)calloc((size_t)nc, sizeof(int32_t));
  for (int32_t v = 0; v < n; ++v) h->vw[parent[v]] += vw ? vw[v] : 1;
  int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * (size_t)(p ? p : 1));
  int64_t *len = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m ? m : 1));
#pragma omp parallel for schedule(dynamic, 1024)
  for (int32_t e = 0; e < m; ++e) {
    const int64_t a = off[e], b = off[e + 1];
    for (int64_t q = a; q < b; ++q) tmp[q] = parent[pins[q]];
    qsort(tmp + a, (size_t)(b - a), sizeof(int32_t), cmp_i32);
    int64_t w = a;
    for (int64_t q = a; q < b; ++q)
      if (q == a || tmp[q] != tmp[q - 1]) tmp[w++] = tmp[q];
    len[e] = w - a >= 2 ? w - a : 0;
  }
  h->off = (int64_t *)malloc(sizeof(int64_t) * ((size_t)m + 1));
  h->nw = nw ? (int32_t *)malloc(sizeof(int32_t) * (size_t)(m ? m : 1)) : NULL;
  int64_t pc = 0;
  int32_t mc = 0;
  h->off[0] = 0;
  for (int32_t e = 0; e < m; ++e) {
    if (len[e] == 0) continue;
    if (h->nw) h->nw[mc] = nw[e];
    pc += len[e];
    h->off[++mc] = pc;
  }
  h->pins = (int32_t *)malloc(sizeof(int32_t) * (size_t)(pc ? pc : 1));
  {
    int32_t *src_net = (int32_t *)malloc(sizeof(int32_t) * (size_t)(mc ? mc : 1));
    int32_t j = 0;
    for (int32_t e = 0; e < m; ++e)
      if (len[e]) src_net[j++] = e;
#pragma omp parallel for schedule(dynamic, 1024)
    for (int32_t x = 0; x < mc; ++x)
      memcpy(h->pins + h->off[x], tmp + off[src_net[x]], sizeof(int32_t) * (size_t)(h->off[x + 1] - h->off[x]));
    free(src_net);
  }
  free(tmp);
  free(len);
  h->m = mc;
  h->p = pc;
  return h;
}

/* Contraction of a given clustering (parent[v] in [0, nc), every coarse vertex used or not):
 * returns a handle with the coarse hypergraph (free with wl_coarse_free), NULL for a bad parent. */
void *wl_contract(int32_t n, int32_t m, int64_t p, const int64_t *off, const int32_t *pins, const int32_t *nw,
                  const int32_t *vw, const int32_t *parent, int32_t nc, int32_t *mc_out, int64_t *pc_out) {
  for (int32_t v = 0; v < n; ++v)
    if (parent[v] < 0 || parent[v] >= nc) return NULL;
  coarse_hg *h = contract(m, p, off, pins, nw, vw, n, parent, nc);
  *mc_out = h->m;
  *pc_out = h->p;
  return h;
}

/* One contraction level.  parent[v] receives v's coarse vertex; returns a handle with the coarse
 * hypergraph (free with wl_coarse_free) and its sizes. */
void *wl_coarsen(int32_t n, int32_t m, int64_t p, const int64_t *off, const int32_t *pins, const int32_t *nw,
                 const int32_t *vw, uint64_t seed, int32_t *parent, int32_t *nc_out, int32_t *mc_out,
                 int64_t *pc_out) {
  /* incidence lists: net and pin position of every incidence of a vertex, nets ascending */
  int64_t *voff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  int32_t *inc = (int32_t *)malloc(sizeof(int32_t) * (size_t)(p ? p : 1));
  int32_t *incpos = (int32_t *)malloc(sizeof(int32_t) * (size_t)(p ? p : 1));
  for (int64_t q = 0; q < p; ++q) voff[pins[q] + 1]++;
  for (int32_t v = 0; v < n; ++v) voff[v + 1] += voff[v];
  int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
  memcpy(cur, voff, sizeof(int64_t) * (size_t)n);
  for (int32_t e = 0; e < m; ++e)
    for (int64_t q = off[e]; q < off[e + 1]; ++q) {
      inc[cur[pins[q]]] = e;
      incpos[cur[pins[q]]++] = (int32_t)q;
    }
  free(cur);
  /* nx: next pin position >= q whose vertex is still unmatched (union-find with path halving over
   * the pin array, position p a sentinel), so a scan of a mostly matched large net is cheap */
  int32_t *nx = (int32_t *)malloc(sizeof(int32_t) * ((size_t)p + 1));
  for (int64_t q = 0; q <= p; ++q) nx[q] = (int32_t)q;
  /* matching along a random incident net, in a random vertex order */
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  int32_t *match = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  hm64 r = hm_stream(seed, 11);
  for (int32_t i = 0; i < n; ++i) {
    perm[i] = i;
    match[i] = -1;
  }
  for (int32_t i = n - 1; i > 0; --i) {
    int32_t j = (int32_t)hm_below(&r, (uint64_t)i + 1);
    int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
  for (int32_t i = 0; i < n; ++i) {
    const int32_t u = perm[i];
    if (match[u] >= 0) continue;
    const int64_t d = voff[u + 1] - voff[u];
    if (d == 0) continue;
    const int32_t e = inc[voff[u] + (int64_t)hm_below(&r, (uint64_t)d)];
    const int64_t a = off[e], b = off[e + 1];
    const int64_t start = (int64_t)hm_below(&r, (uint64_t)(b - a));
    /* the first pin other than u, cyclically from a + start, whose vertex is unmatched */
    int64_t q = nx_find(nx, a + start);
    while (q < b && pins[q] == u) q = nx_find(nx, q + 1);
    if (q >= b) {
      q = nx_find(nx, a);
      while (q < a + start && pins[q] == u) q = nx_find(nx, q + 1);
      if (q >= a + start) q = -1;
    }
    if (q >= 0) {
      const int32_t w = pins[q];
      match[u] = w;
      match[w] = u;
      for (int64_t j = voff[u]; j < voff[u + 1]; ++j) nx[incpos[j]] = incpos[j] + 1;
      for (int64_t j = voff[w]; j < voff[w + 1]; ++j) nx[incpos[j]] = incpos[j] + 1;
    }
  }
  free(nx);
  free(incpos);
  int32_t pending = -1; /* leftover singletons pair up in permutation order */
  for (int32_t i = 0; i < n; ++i) {
    const int32_t u = perm[i];
    if (match[u] >= 0) continue;
    if (pending < 0) {
      pending = u;
    } else {
      match[u] = pending;
      match[pending] = u;
      pending = -1;
    }
  }
  free(perm);
  free(voff);
  free(inc);
  /* coarse IDs in order of the smaller fine ID of each pair */
  for (int32_t v = 0; v < n; ++v) parent[v] = -1;
  int32_t nc = 0;
  for (int32_t v = 0; v < n; ++v) {
    if (parent[v] >= 0) continue;
    parent[v] = nc;
    if (match[v] >= 0) parent[match[v]] = nc;
    ++nc;
  }
  free(match);
  coarse_hg *h = contract(m, p, off, pins, nw, vw, n, parent, nc);
  *nc_out = nc;
  *mc_out = h->m;
  *pc_out = h->p;
  return h;
}

void wl_coarse_fill(void *handle, int64_t *off, int32_t *pins, int32_t *nw, int32_t *vw) {
  coarse_hg *h = (coarse_hg *)handle;
  memcpy(off, h->off, sizeof(int64_t) * ((size_t)h->m + 1));
  memcpy(pins, h->pins, sizeof(int32_t) * (size_t)h->p);
  if (nw && h->nw) memcpy(nw, h->nw, sizeof(int32_t) * (size_t)h->m);
  memcpy(vw, h->vw, sizeof(int32_t) * (size_t)h->n);
}

void wl_coarse_free(void *handle) {
  coarse_hg *h = (coarse_hg *)handle;
  if (!h) return;
  free(h->off);
  free(h->pins);
  free(h->nw);
  free(h->vw);
  free(h);
}

/* Greedy balanced start: seeded shuffle, then each vertex joins the currently lightest block
 * (lowest block ID on ties). */
void wl_greedy_initial(int32_t n, int32_t k, const int32_t *vw, uint64_t seed, int32_t *part) {
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  hm64 r = hm_stream(seed, 12);
  for (int32_t i = 0; i < n; ++i) perm[i] = i;
  for (int32_t i = n - 1; i > 0; --i) {
    int32_t j = (int32_t)hm_below(&r, (uint64_t)i + 1);
    int32_t t = perm[i];
    perm[i] = perm[j];
    perm[j] = t;
  }
  int64_t *bw = (int64_t *)calloc((size_t)k, sizeof(int64_t));
  for (int32_t i = 0; i < n; ++i) {
    const int32_t v = perm[i];
    int32_t best = 0;
    for (int32_t b = 1; b < k; ++b)
      if (bw[b] < bw[best]) best = b;
    part[v] = best;
    bw[best] += vw ? vw[v] : 1;
  }
  free(bw);
  free(perm);
}
