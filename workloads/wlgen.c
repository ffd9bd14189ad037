/*
 * Seeded synthetic hypergraph workloads.
 *
 * This file only builds inputs: hypergraph structure (CSR of pins per net), vertex weights and
 * starting partitions.  It contains none of the refinement arithmetic, so both the CPU oracle and
 * the GPU library can consume its output without sharing any method code.
 *
 * Random numbers: SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014).  One independent stream per purpose, seeded from the user seed and a
 * stream id.  Bounded integers use Lemire's multiply-shift with rejection ("Fast random integer
 * generation in an interval", TOMACS 2019).  Distinct pins are drawn with Floyd's sampling
 * (Bentley and Floyd, "Programming pearls: a sample of brilliance", CACM 1987) and stored sorted.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ random numbers */

typedef struct { uint64_t s; } sm64;

static inline uint64_t sm_next(sm64 *r) {
  uint64_t z = (r->s += 0x9E3779B97F4A7C15ULL);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

static sm64 sm_stream(uint64_t seed, uint64_t stream_id) {
  sm64 r;
  r.s = seed ^ (0x9E3779B97F4A7C15ULL * (stream_id + 1));
  (void)sm_next(&r);
  return r;
}

/* uniform integer in [0, range), range >= 1 */
static inline uint64_t sm_below(sm64 *r, uint64_t range) {
  uint64_t x = sm_next(r);
  __uint128_t mm = (__uint128_t)x * range;
  uint64_t lo = (uint64_t)mm;
  if (lo < range) {
    uint64_t thr = (0 - range) % range;
    while (lo < thr) {
      x = sm_next(r);
      mm = (__uint128_t)x * range;
      lo = (uint64_t)mm;
    }
  }
  return (uint64_t)(mm >> 64);
}

/* uniform double in [0, 1) with 53 random bits */
static inline double sm_unit(sm64 *r) { return (double)(sm_next(r) >> 11) * 0x1.0p-53; }

/* ------------------------------------------------------------------ specification */

enum { SIZE_UNIFORM = 0, SIZE_GEOMETRIC = 1, SIZE_ZIPF = 2 };
enum { PLACE_UNIFORM = 0, PLACE_RANDOM_ANCHOR = 1, PLACE_ROW_ANCHOR = 2 };

typedef struct {
  int32_t n;          /* vertices */
  int32_t m;          /* nets (ignored when p_target > 0) */
  int64_t p_target;   /* > 0: draw net sizes until their sum reaches p_target */
  int32_t size_kind;  /* SIZE_* */
  int32_t size_a;     /* uniform: low; geometric: base; zipf: low end of the support */
  int32_t size_b;     /* uniform: high; geometric and zipf: cap */
  double size_q;      /* geometric: success probability; zipf: exponent */
  int32_t place_kind; /* PLACE_* */
  int32_t win_fixed;  /* half-width of the anchor window (minimum half-width for row anchors) */
  int32_t win_mult;   /* row anchors: half-width = max(win_mult*|e|, win_fixed) */
  int32_t sort_by_anchor; /* random anchors: number nets in ascending anchor order */
  int32_t pad_;
  uint64_t seed;
} wl_spec;

/* stream ids */
#define ST_SIZE 1
#define ST_ANCHOR 2
#define ST_PINS 3
#define ST_VW 4
#define ST_PART 5
#define ST_NOISE 6

/* Zipf(s) on [lo, hi] by inverse CDF over a table of cumulative weights */
typedef struct { int32_t lo, hi; double *cdf; } zipf_table;

static int zipf_init(zipf_table *z, int32_t lo, int32_t hi, double s) {
  int64_t cnt = (int64_t)hi - lo + 1;
  z->lo = lo;
  z->hi = hi;
  z->cdf = (double *)malloc(sizeof(double) * (size_t)cnt);
  if (!z->cdf) return -1;
  double acc = 0.0;
  for (int64_t i = 0; i < cnt; ++i) {
    acc += pow((double)(lo + i), -s);
    z->cdf[i] = acc;
  }
  for (int64_t i = 0; i < cnt; ++i) z->cdf[i] /= acc;
  z->cdf[cnt - 1] = 1.0;
  return 0;
}

static int32_t zipf_draw(const zipf_table *z, sm64 *r) {
  double u = sm_unit(r);
  int64_t a = 0, b = (int64_t)z->hi - z->lo; /* smallest index with cdf > u */
  while (a < b) {
    int64_t mid = (a + b) >> 1;
    if (z->cdf[mid] > u) b = mid; else a = mid + 1;
  }
  return (int32_t)(z->lo + a);
}

static int32_t draw_size(const wl_spec *sp, const zipf_table *z, sm64 *r) {
  switch (sp->size_kind) {
  case SIZE_UNIFORM:
    return sp->size_a + (int32_t)sm_below(r, (uint64_t)(sp->size_b - sp->size_a + 1));
  case SIZE_GEOMETRIC: {
    /* number of failures before the first success, by inversion */
    double u = 1.0 - sm_unit(r); /* (0, 1] */
    double g = floor(log(u) / log(1.0 - sp->size_q));
    double s = (double)sp->size_a + g;
    if (s > (double)sp->size_b) s = (double)sp->size_b;
    return (int32_t)s;
  }
  default:
    return zipf_draw(z, r);
  }
}

typedef struct { int64_t anchor; int64_t idx; int32_t size; int32_t pad_; } net_desc;

static int cmp_desc(const void *a, const void *b) {
  const net_desc *x = (const net_desc *)a, *y = (const net_desc *)b;
  if (x->anchor != y->anchor) return x->anchor < y->anchor ? -1 : 1;
  return x->idx < y->idx ? -1 : (x->idx > y->idx);
}

/* Draws the size and anchor of every net, in final net order.  Caller frees *out. */
static int describe_nets(const wl_spec *sp, net_desc **out, int32_t *m_out, int64_t *p_out) {
  zipf_table z = {0, 0, NULL};
  if (sp->size_kind == SIZE_ZIPF && zipf_init(&z, sp->size_a, sp->size_b, sp->size_q)) return -1;
  sm64 rs = sm_stream(sp->seed, ST_SIZE), ra = sm_stream(sp->seed, ST_ANCHOR);
  int64_t cap = sp->p_target > 0 ? 1024 : sp->m;
  net_desc *d = (net_desc *)malloc(sizeof(net_desc) * (size_t)(cap > 0 ? cap : 1));
  if (!d) { free(z.cdf); return -1; }
  int64_t m = 0, p = 0;
  for (;;) {
    if (sp->p_target > 0) {
      if (p >= sp->p_target) break;
    } else if (m >= sp->m) {
      break;
    }
    if (m == cap) {
      cap *= 2;
      net_desc *nd = (net_desc *)realloc(d, sizeof(net_desc) * (size_t)cap);
      if (!nd) { free(d); free(z.cdf); return -1; }
      d = nd;
    }
    int32_t s = draw_size(sp, &z, &rs);
    if (s > sp->n) s = sp->n;
    if (sp->p_target > 0 && p + s > sp->p_target) { /* truncate the last net */
      s = (int32_t)(sp->p_target - p);
      if (s < 2) s = 2;
    }
    d[m].size = s;
    d[m].idx = m;
    d[m].anchor = 0;
    if (sp->place_kind == PLACE_RANDOM_ANCHOR) d[m].anchor = (int64_t)sm_below(&ra, (uint64_t)sp->n);
    ++m;
    p += s;
  }
  free(z.cdf);
  if (sp->place_kind == PLACE_RANDOM_ANCHOR && sp->sort_by_anchor) qsort(d, (size_t)m, sizeof(net_desc), cmp_desc);
  if (m > INT32_MAX) { free(d); return -1; }
  *out = d;
  *m_out = (int32_t)m;
  *p_out = p;
  return 0;
}

/* ------------------------------------------------------------------ distinct sampling */

typedef struct { int64_t cap; int64_t *slot; } hset; /* open addressing, -1 = empty */

static int hset_init(hset *h, int64_t want) {
  int64_t c = 16;
  while (c < 2 * want) c <<= 1;
  h->cap = c;
  h->slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)c);
  if (!h->slot) return -1;
  memset(h->slot, 0xff, sizeof(int64_t) * (size_t)c);
  return 0;
}

/* returns 1 if inserted, 0 if already present */
static int hset_insert(hset *h, int64_t x) {
  uint64_t hh = (uint64_t)x * 0x9E3779B97F4A7C15ULL;
  int64_t i = (int64_t)(hh >> 17) & (h->cap - 1);
  for (;;) {
    if (h->slot[i] == -1) { h->slot[i] = x; return 1; }
    if (h->slot[i] == x) return 0;
    i = (i + 1) & (h->cap - 1);
  }
}

static int cmp_i32(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

/* s distinct values from [lo, lo + range), sorted ascending, written to out */
static int floyd_sample(sm64 *r, int64_t lo, int64_t range, int32_t s, int32_t *out) {
  if (s <= 64) {
    int32_t cnt = 0;
    for (int64_t j = range - s; j < range; ++j) {
      int64_t t = (int64_t)sm_below(r, (uint64_t)(j + 1));
      int found = 0;
      for (int32_t q = 0; q < cnt; ++q)
        if (out[q] == (int32_t)(lo + t)) { found = 1; break; }
      out[cnt++] = (int32_t)(lo + (found ? j : t));
    }
  } else {
    hset h;
    if (hset_init(&h, s)) return -1;
    int32_t cnt = 0;
    for (int64_t j = range - s; j < range; ++j) {
      int64_t t = (int64_t)sm_below(r, (uint64_t)(j + 1));
      int64_t pick = hset_insert(&h, t) ? t : j;
      if (pick == j) hset_insert(&h, j);
      out[cnt++] = (int32_t)(lo + pick);
    }
    free(h.slot);
  }
  qsort(out, (size_t)s, sizeof(int32_t), cmp_i32);
  return 0;
}

/* ------------------------------------------------------------------ public API */

/* Pass 1: number of nets and pins the spec produces. */
int wl_sizes(const wl_spec *sp, int32_t *m_out, int64_t *p_out) {
  net_desc *d = NULL;
  if (describe_nets(sp, &d, m_out, p_out)) return -1;
  free(d);
  return 0;
}

/* Pass 2: fill net_offsets[m+1] and pins[p] (caller-allocated, sizes from wl_sizes). */
int wl_fill(const wl_spec *sp, int32_t m, int64_t p, int64_t *off, int32_t *pins) {
  net_desc *d = NULL;
  int32_t mm;
  int64_t pp;
  if (describe_nets(sp, &d, &mm, &pp)) return -1;
  if (mm != m || pp != p) { free(d); return -2; }
  off[0] = 0;
  for (int32_t e = 0; e < m; ++e) off[e + 1] = off[e] + d[e].size;
  for (int32_t e = 0; e < m; ++e) {
    int32_t s = d[e].size;
    sm64 r = sm_stream(sp->seed ^ 0xD1B54A32D192ED03ULL, ((uint64_t)ST_PINS << 40) + (uint64_t)d[e].idx);
    int64_t lo = 0, range = sp->n;
    if (sp->place_kind != PLACE_UNIFORM) {
      int64_t a = d[e].anchor, h = sp->win_fixed;
      if (sp->place_kind == PLACE_ROW_ANCHOR) {
        a = (int64_t)((double)d[e].idx * (double)sp->n / (double)m);
        int64_t hm = (int64_t)sp->win_mult * s;
        if (hm > h) h = hm;
      }
      lo = a - h < 0 ? 0 : a - h;
      int64_t hi = a + h > sp->n - 1 ? sp->n - 1 : a + h;
      range = hi - lo + 1;
      if (range < s) { /* widen symmetric window until it holds the net */
        lo = 0;
        range = sp->n;
      }
    }
    if (floyd_sample(&r, lo, range, s, pins + off[e])) { free(d); return -1; }
  }
  free(d);
  return 0;
}

/* weights uniform in {1..wmax}; stream 0 for vertex weights, 1 for net weights */
void wl_weights(int64_t count, int32_t wmax, uint64_t seed, int32_t stream, int32_t *w) {
  sm64 r = sm_stream(seed, ST_VW + 16 * (uint64_t)stream);
  for (int64_t i = 0; i < count; ++i) w[i] = 1 + (int32_t)sm_below(&r, (uint64_t)wmax);
}

/* seeded permutation pi, then part[pi_i] = i mod k (equal block sizes up to one vertex) */
void wl_part_roundrobin(int32_t n, int32_t k, uint64_t seed, int32_t *part) {
  int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  sm64 r = sm_stream(seed, ST_PART);
  for (int32_t i = 0; i < n; ++i) perm[i] = i;
  for (int32_t i = n - 1; i > 0; --i) { /* Fisher-Yates */
    int32_t j = (int32_t)sm_below(&r, (uint64_t)i + 1);
    int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
  }
  for (int32_t i = 0; i < n; ++i) part[perm[i]] = i % k;
  free(perm);
}

/* part[v] = floor(v*k/n), then n_noise distinct vertices (Floyd) reassigned uniformly in [0,k) */
int wl_part_ranges_noise(int32_t n, int32_t k, int32_t n_noise, uint64_t seed, int32_t *part) {
  for (int32_t v = 0; v < n; ++v) part[v] = (int32_t)(((int64_t)v * k) / n);
  if (n_noise <= 0) return 0;
  int32_t *pick = (int32_t *)malloc(sizeof(int32_t) * (size_t)n_noise);
  if (!pick) return -1;
  sm64 r = sm_stream(seed, ST_NOISE);
  if (floyd_sample(&r, 0, n, n_noise, pick)) { free(pick); return -1; }
  for (int32_t i = 0; i < n_noise; ++i) part[pick[i]] = (int32_t)sm_below(&r, (uint64_t)k);
  free(pick);
  return 0;
}

/* uniform random partition, each vertex independently in [0,k) */
void wl_part_uniform(int32_t n, int32_t k, uint64_t seed, int32_t *part) {
  sm64 r = sm_stream(seed, ST_PART + 100);
  for (int32_t v = 0; v < n; ++v) part[v] = (int32_t)sm_below(&r, (uint64_t)k);
}

/* raw stream access for tests that need seeded integers */
void wl_randint(uint64_t seed, uint64_t stream, int64_t count, uint64_t range, int64_t *out) {
  sm64 r = sm_stream(seed, stream);
  for (int64_t i = 0; i < count; ++i) out[i] = (int64_t)sm_below(&r, range);
}
