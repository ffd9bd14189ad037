// Deterministic flow-based refinement of one block pair (Section 5.1, Algorithm 3) on gfx950.
//
// The pair (a, b) is refined on the Lawler network of its induced subhypergraph (layout in
// FlowState).  Algorithm 3 runs on the host, every step of it in kernels:
//   region      breadth-first levels from the pair's boundary inside each block, a level taken
//               whole while its weight fits the side's bound, then the next level's vertices in
//               increasing ID while they fit (a scan of their weights); every net is expanded once;
//   network     node numbers of the region vertices (a scan), endpoints per net, arc blocks (a
//               scan), arcs and the vertex nodes' adjacency;
//   max flow    lock-free push-relabel: one thread per node pushes to its lowest residual
//               neighbour or relabels, with atomics on residuals and excesses only, and global
//               relabels (breadth-first distances to the sinks, then to the sources above N, by
//               the same frontier searches) at the start and whenever the sweeps since the last
//               one took twice its time; after a piercing step that may open augmenting paths
//               the flow is augmented from the previous one;
//   cuts        the nodes the sources reach in the residual network (S_r) and those that reach the
//               sinks (T_r), by breadth-first search (first level arc-parallel, then a wave per
//               frontier node); after a piercing vertex the other side does not reach, the flow
//               stays maximum and the pierced side's set only grows by a search from that vertex;
//   piercing    per cut net of the smaller side, its free endpoints outside that side, the least
//               key (in the other side's set, vertex ID) by one atomic minimum.
// Push-relabel leaves a maximum flow whose assignment depends on the schedule of the waves.  S_r
// and T_r do not: they are the inclusion-minimal source and sink sides of the minimum cuts, the
// same for every maximum flow (Section 5.1), so every decision the host takes is deterministic.
// The k-way schedule of Section 5.2 (flow_refine) refines the disjoint pairs of each matching at
// once on worker contexts, each with its own stream, host thread and flow state.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <string>
#include <thread>
#include <vector>

#include "dev_util.h"
#include "jet_internal.h"

namespace jet {
namespace {

constexpr int kFB = 256;
constexpr int64_t kFGridCap = 1 << 14;
constexpr int kPushCycles = 64;        // push or relabel steps of one node per sweep
constexpr int kSweepsPerCheck = 8;     // sweeps between two counts of the active nodes
constexpr int kLevelBatch = 4;         // breadth-first levels launched between two looks, doubling
constexpr int kLevelBatchMax = 64;     // up to this while the search goes on
constexpr int64_t kLevelGrid = 512;    // workgroups of a frontier level launch
constexpr int64_t kMaxChecks = 1 << 16;  // a flow that needs more is reported, not waited for

inline unsigned fgrid(int64_t work) {
  int64_t g = (work + kFB - 1) / kFB;
  if (g < 1) g = 1;
  if (g > kFGridCap) g = kFGridCap;
  return (unsigned)g;
}

// scalar slots of FlowState::sc
enum : int {
  kScCut = 0, kScBwA, kScBwB, kScLw, kScCnt, kScWsum, kScFlow, kScW1, kScW2, kScActive, kScChanged,
  kScBest, kScMoved, kScErr, kScN
};

__device__ __forceinline__ int64_t cv(const int32_t *vw, int32_t v) { return vw ? (int64_t)vw[v] : 1; }
__device__ __forceinline__ int64_t wn(const int32_t *nw, int32_t e) { return nw ? (int64_t)nw[e] : 1; }

template <typename T>
__device__ __forceinline__ T ld(const T *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void add_sc(int64_t *sc, int slot, int64_t x) {
  x = wave_sum(x);
  if (lane_id() == 0 && x != 0) atomicAdd((unsigned long long *)&sc[slot], (unsigned long long)x);
}

// ---- pair scalars ----

__global__ void k_fl_nets(const int64_t *__restrict__ off, const int32_t *__restrict__ pins,
                          const int32_t *__restrict__ nw, const int32_t *__restrict__ part, int32_t m, int32_t a,
                          int32_t b, int32_t *__restrict__ cnt_a, int32_t *__restrict__ cnt_b, int64_t *sc) {
  int64_t cut = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t ca = 0, cb = 0;
    for (int64_t q = off[e]; q < off[e + 1]; ++q) {
      const int32_t x = part[pins[q]];
      ca += x == a;
      cb += x == b;
    }
    cnt_a[e] = ca;
    cnt_b[e] = cb;
    if (ca > 0 && cb > 0) cut += wn(nw, (int32_t)e);
  }
  add_sc(sc, kScCut, cut);
}

__global__ void k_fl_bw(const int32_t *__restrict__ part, const int32_t *__restrict__ vw, int32_t n, int32_t a,
                        int32_t b, int64_t *sc) {
  int64_t wa = 0, wb = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = part[v];
    if (x == a) wa += cv(vw, (int32_t)v);
    else if (x == b) wb += cv(vw, (int32_t)v);
  }
  add_sc(sc, kScBwA, wa);
  add_sc(sc, kScBwB, wb);
}

__global__ void k_fl_fill(int32_t *__restrict__ p, int64_t count, int32_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void k_fl_fill8(int8_t *__restrict__ p, int64_t count, int8_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// ---- region (reading F1 of the design notes) ----

// level 0: vertices of `side` with a net that has a pin in the other block; sc[kScLw] += weights
__global__ void k_fl_level0(const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
                            const int32_t *__restrict__ part, const int32_t *__restrict__ cnt_other,
                            const int32_t *__restrict__ vw, int32_t n, int32_t side, int32_t *__restrict__ lvl,
                            int64_t *sc) {
  int64_t lw = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (part[v] != side) continue;
    bool bnd = false;
    for (int64_t q = voff[v]; q < voff[v + 1] && !bnd; ++q) bnd = cnt_other[inc[q]] > 0;
    if (bnd) {
      lvl[v] = 0;
      lw += cv(vw, (int32_t)v);
    }
  }
  add_sc(sc, kScLw, lw);
}

__global__ void k_fl_take(const int32_t *__restrict__ lvl, int32_t n, int32_t L, int8_t *__restrict__ rmark,
                          int8_t mark, int64_t *sc) {
  int64_t cnt = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (lvl[v] == L) {
      rmark[v] = mark;
      ++cnt;
    }
  add_sc(sc, kScCnt, cnt);
}

// level L + 1: the unseen vertices of `side` on the nets of level L (each net expanded once);
// sc[kScLw] += their weights
__global__ void k_fl_expand(const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
                            const int64_t *__restrict__ off, const int32_t *__restrict__ pins,
                            const int32_t *__restrict__ part, const int32_t *__restrict__ vw, int32_t n, int32_t side,
                            int32_t L, int32_t *__restrict__ lvl, int32_t *__restrict__ nexp, int64_t *sc) {
  int64_t lw = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    if (ld(&lvl[v]) != L) continue;
    for (int64_t q = voff[v]; q < voff[v + 1]; ++q) {
      const int32_t e = inc[q];
      if (atomicExch(&nexp[e], 1) != 0) continue;
      for (int64_t r = off[e]; r < off[e + 1]; ++r) {
        const int32_t x = pins[r];
        if (part[x] == side && ld(&lvl[x]) == -1 && atomicCAS(&lvl[x], -1, L + 1) == -1) lw += cv(vw, x);
      }
    }
  }
  add_sc(sc, kScLw, lw);
}

__global__ void k_fl_level_w(const int32_t *__restrict__ lvl, const int32_t *__restrict__ vw, int32_t n, int32_t L,
                             int32_t *__restrict__ wtmp) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    wtmp[v] = lvl[v] == L ? (int32_t)cv(vw, (int32_t)v) : 0;
}

// the level's vertices in increasing ID while the running weight stays within rem; sc[kScCnt] +=
// their number, sc[kScLw] += their weight
__global__ void k_fl_take_partial(const int32_t *__restrict__ lvl, const int64_t *__restrict__ wscan,
                                  const int32_t *__restrict__ vw, int32_t n, int32_t L, int64_t rem,
                                  int8_t *__restrict__ rmark, int8_t mark, int64_t *sc) {
  int64_t cnt = 0, w = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (lvl[v] == L && wscan[v] + cv(vw, (int32_t)v) <= rem) {
      rmark[v] = mark;
      ++cnt;
      w += cv(vw, (int32_t)v);
    }
  add_sc(sc, kScCnt, cnt);
  add_sc(sc, kScLw, w);
}

// ---- network ----

// free vertices (term == nullptr: the region; else the pair's vertices with term 0) for the scan
__global__ void k_fl_free(const int32_t *__restrict__ part, const int8_t *__restrict__ rmark,
                          const int8_t *__restrict__ term, int32_t n, int32_t a, int32_t b, int32_t *__restrict__ wtmp) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = part[v];
    const bool pair = x == a || x == b;
    wtmp[v] = term ? (pair && term[v] == 0) : rmark[v] != 0;
  }
}

// node of every vertex of the pair: free vertices 2 + their rank; terminals 0 (source) or 1 (sink):
// by block without term, by term with it
__global__ void k_fl_vnode(const int32_t *__restrict__ part, const int8_t *__restrict__ term,
                           const int32_t *__restrict__ wtmp, const int64_t *__restrict__ wscan, int32_t n, int32_t a,
                           int32_t b, int32_t *__restrict__ vnode, int32_t *__restrict__ nvert) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = part[v];
    int32_t node = -1;
    if (wtmp[v]) {
      node = 2 + (int32_t)wscan[v];
      nvert[wscan[v]] = (int32_t)v;
    } else if (x == a || x == b) {
      node = term ? (term[v] == 1 ? 0 : 1) : (x == a ? 0 : 1);
    }
    vnode[v] = node;
  }
}

// distinct endpoints per net; arc block size and relevance; sc[kScWsum] += weights of relevant nets
__global__ void k_fl_ends(const int64_t *__restrict__ off, const int32_t *__restrict__ pins,
                          const int32_t *__restrict__ nw, const int32_t *__restrict__ vnode, int32_t m,
                          int32_t *__restrict__ ends, int32_t *__restrict__ asize, int32_t *__restrict__ rel,
                          int64_t *sc) {
  int64_t ws = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    int32_t fr = 0, hs = 0, ht = 0;
    for (int64_t q = off[e]; q < off[e + 1]; ++q) {
      const int32_t x = vnode[pins[q]];
      if (x == 0) hs = 1;
      else if (x == 1) ht = 1;
      else if (x >= 2) ++fr;
    }
    const int32_t en = fr + hs + ht;
    const bool r = en >= 2;
    ends[e] = en;
    asize[e] = r ? 2 + 4 * en : 0;
    rel[e] = r;
    if (r) ws += wn(nw, (int32_t)e);
  }
  add_sc(sc, kScWsum, ws);
}

__global__ void k_fl_nmeta(const int32_t *__restrict__ rel, const int64_t *__restrict__ nrid,
                           const int64_t *__restrict__ nbase, const int32_t *__restrict__ ends, int32_t m,
                           int32_t *__restrict__ rnet, int64_t *__restrict__ rbase, int32_t *__restrict__ rends) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    if (!rel[e]) continue;
    const int64_t r = nrid[e];
    rnet[r] = (int32_t)e;
    rbase[r] = nbase[e];
    rends[r] = ends[e];
  }
}

// the endpoints of relevant net r in their order: the source node, the sink node, then the free
// vertices in pin order; f(j, node)
template <typename F>
__device__ __forceinline__ void for_endpoints(const int64_t *off, const int32_t *pins, const int32_t *vnode,
                                              int32_t e, F f) {
  bool hs = false, ht = false;
  for (int64_t q = off[e]; q < off[e + 1]; ++q) {
    const int32_t x = vnode[pins[q]];
    hs |= x == 0;
    ht |= x == 1;
  }
  int32_t j = 0;
  if (hs) f(j++, 0);
  if (ht) f(j++, 1);
  for (int64_t q = off[e]; q < off[e + 1]; ++q) {
    const int32_t x = vnode[pins[q]];
    if (x >= 2) f(j++, x);
  }
}

__global__ void k_fl_adj_count(const int64_t *__restrict__ off, const int32_t *__restrict__ pins,
                               const int32_t *__restrict__ vnode, int64_t mrel, const int32_t *__restrict__ rnet,
                               int32_t *__restrict__ vcnt) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < mrel; r += (int64_t)gridDim.x * blockDim.x)
    for_endpoints(off, pins, vnode, rnet[r], [&](int32_t, int32_t x) { atomicAdd(&vcnt[x], 1); });
}

__global__ void k_fl_build(const int64_t *__restrict__ off, const int32_t *__restrict__ pins,
                           const int32_t *__restrict__ nw, const int32_t *__restrict__ vnode, int64_t mrel,
                           const int32_t *__restrict__ rnet, const int64_t *__restrict__ rbase, int32_t nv,
                           int64_t inf, const int64_t *__restrict__ voffn, int32_t *__restrict__ vcur,
                           int32_t *__restrict__ head, int32_t *__restrict__ tail, int64_t *__restrict__ res,
                           int64_t *__restrict__ vadj) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < mrel; r += (int64_t)gridDim.x * blockDim.x) {
    const int32_t e = rnet[r];
    const int64_t B = rbase[r];
    const int32_t ein = nv + 2 * (int32_t)r, eout = ein + 1;
    tail[B] = ein;
    head[B] = eout;
    res[B] = wn(nw, e);
    tail[B + 1] = eout;
    head[B + 1] = ein;
    res[B + 1] = 0;
    for_endpoints(off, pins, vnode, e, [&](int32_t j, int32_t x) {
      const int64_t a0 = B + 2 + 4 * (int64_t)j;
      tail[a0] = x;        head[a0] = ein;      res[a0] = inf;
      tail[a0 + 1] = ein;  head[a0 + 1] = x;    res[a0 + 1] = 0;
      tail[a0 + 2] = eout; head[a0 + 2] = x;    res[a0 + 2] = inf;
      tail[a0 + 3] = x;    head[a0 + 3] = eout; res[a0 + 3] = 0;
      vadj[voffn[x] + atomicAdd(&vcur[x], 1)] = a0;
    });
  }
}

__global__ void k_fl_init_nodes(int64_t N, uint8_t *__restrict__ term, int32_t *__restrict__ h,
                                int64_t *__restrict__ ex) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < N; u += (int64_t)gridDim.x * blockDim.x) {
    term[u] = u == 0 ? 1 : u == 1 ? 2 : 0;
    h[u] = 0;
    ex[u] = 0;
  }
}

// ---- maximum flow ----

// the arcs out of node u: f(arc)
template <typename F>
__device__ __forceinline__ void for_out(int64_t u, int32_t nv, const int64_t *voffn, const int64_t *vadj,
                                        const int64_t *rbase, const int32_t *rends, F f) {
  if (u < nv) {
    for (int64_t i = voffn[u]; i < voffn[u + 1]; ++i) {
      const int64_t a0 = vadj[i];
      f(a0);      // x -> e_in
      f(a0 + 3);  // x -> e_out (reverse of e_out -> x)
    }
  } else {
    const int64_t r = (u - nv) >> 1;
    const bool out = ((u - nv) & 1) != 0;
    const int64_t B = rbase[r];
    const int32_t E = rends[r];
    f(out ? B + 1 : B);
    for (int32_t j = 0; j < E; ++j) f(B + 2 + 4 * (int64_t)j + (out ? 2 : 1));
  }
}

__device__ __forceinline__ void push(int64_t a, int32_t u, int32_t v, int64_t d, int64_t *res, int64_t *ex) {
  atomicAdd((unsigned long long *)&res[a], (unsigned long long)(-d));
  atomicAdd((unsigned long long *)&res[a ^ 1], (unsigned long long)d);
  atomicAdd((unsigned long long *)&ex[u], (unsigned long long)(-d));
  atomicAdd((unsigned long long *)&ex[v], (unsigned long long)d);
}

// every residual arc from a source to a non-source node is saturated
__global__ void k_fl_saturate(int64_t A, const int32_t *__restrict__ tail, const int32_t *__restrict__ head,
                              const uint8_t *__restrict__ term, int64_t *__restrict__ res, int64_t *__restrict__ ex) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < A; a += (int64_t)gridDim.x * blockDim.x) {
    const int32_t u = tail[a], v = head[a];
    if (term[u] != 1 || term[v] == 1) continue;
    const int64_t d = ld(&res[a]);
    if (d > 0) push(a, u, v, d, res, ex);
  }
}

// global relabel, phase 1 start: sinks 0, sources N, the rest unlabelled (-1)
__global__ void k_fl_gr_init(int64_t N, const uint8_t *__restrict__ term, int32_t *__restrict__ h) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < N; u += (int64_t)gridDim.x * blockDim.x)
    h[u] = term[u] == 2 ? 0 : term[u] == 1 ? (int32_t)N : -1;
}

// free nodes that reach neither side: height 2N (they hold no excess)
__global__ void k_fl_gr_rest(int64_t N, const uint8_t *__restrict__ term, int32_t *__restrict__ h) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < N; u += (int64_t)gridDim.x * blockDim.x)
    if (term[u] == 0 && h[u] == -1) h[u] = (int32_t)(2 * N);
}

// residual reachability: the flags of the terminal side start the search (dir bit 1: the nodes
// the sources reach, rs; bit 2: the nodes that reach the sinks, rt)
__global__ void k_fl_reach_init(int64_t N, const uint8_t *__restrict__ term, int32_t dir, uint8_t *__restrict__ rs,
                                uint8_t *__restrict__ rt) {
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < N; u += (int64_t)gridDim.x * blockDim.x) {
    if (dir & 1) rs[u] = term[u] == 1;
    if (dir & 2) rt[u] = term[u] == 2;
  }
}

// ---- breadth-first searches over frontiers ----
//
// A search claims nodes level by level.  REACH: a node reached over a residual arc gets its flag set
// (S_r forward from the sources, T_r backward to the sinks); else (a global relabel) a free
// unlabelled node gets the level's label.  The first level from the terminal sets runs arc-parallel
// (terminal nodes can have a great many arcs); later levels take a wave per frontier node.  The
// frontier sizes live on the device in three rotating counters: a level reads one, appends to the
// next and clears the one after, so levels are launched back to back without the host looking.

// arcs out of node u by index: vertex-type nodes (u < nv) have two per adjacency entry (x -> e_in,
// x -> e_out), net nodes one to their partner node and one per endpoint
__device__ __forceinline__ int64_t out_degree(int64_t u, int32_t nv, const int64_t *voffn, const int32_t *rends) {
  return u < nv ? 2 * (voffn[u + 1] - voffn[u]) : 1 + (int64_t)rends[(u - nv) >> 1];
}

__device__ __forceinline__ int64_t out_arc(int64_t u, int64_t i, int32_t nv, const int64_t *voffn,
                                           const int64_t *vadj, const int64_t *rbase) {
  if (u < nv) {
    const int64_t a0 = vadj[voffn[u] + (i >> 1)];
    return (i & 1) ? a0 + 3 : a0;
  }
  const bool out = ((u - nv) & 1) != 0;
  const int64_t B = rbase[(u - nv) >> 1];
  if (i == 0) return out ? B + 1 : B;
  return B + 2 + 4 * (i - 1) + (out ? 2 : 1);
}

// claims node v for the search; true for the one thread that claims it
template <bool REACH>
__device__ __forceinline__ bool claim(int32_t v, const uint8_t *term, uint8_t *flag, int32_t *h, int32_t L) {
  if (REACH) {
    if (ld(&flag[v])) return false;
    // flags are bytes: claimed through the aligned word that holds the byte
    unsigned int *w = (unsigned int *)((uintptr_t)&flag[v] & ~(uintptr_t)3);
    const unsigned int bit = 1u << (8 * ((uintptr_t)&flag[v] & 3));
    return (atomicOr(w, bit) & bit) == 0;
  }
  return term[v] == 0 && ld(&h[v]) == -1 && atomicCAS(&h[v], -1, L + 1) == -1;
}

// the first level, arc-parallel: from the nodes of the terminal side over residual arcs (BACK: into
// them); claimed nodes (REACH: flagged; relabel: label L + 1) appended to front / cnt
template <bool BACK, bool REACH>
__global__ void k_fl_first(int64_t A, const int32_t *__restrict__ tail, const int32_t *__restrict__ head,
                           const int64_t *__restrict__ res, const uint8_t *__restrict__ term, uint8_t side,
                           uint8_t *__restrict__ flag, int32_t *__restrict__ h, int32_t L, int32_t *__restrict__ front,
                           int32_t *__restrict__ cnt) {
  for (int64_t a = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; a < A; a += (int64_t)gridDim.x * blockDim.x) {
    if (res[a] <= 0) continue;
    // BACK: a = u -> v residual with v a terminal, u claimed; else u a terminal, v claimed
    const int32_t from = BACK ? head[a] : tail[a], to = BACK ? tail[a] : head[a];
    if (term[from] != side) continue;
    if (claim<REACH>(to, term, flag, h, L)) front[atomicAdd(cnt, 1)] = to;
  }
}

// one later level: a wave per frontier node in front_in (size *cnt_in), claimed nodes appended to
// front_out / cnt_out; *cnt_zero (the counter two levels ahead) is cleared
template <bool BACK, bool REACH>
__global__ __launch_bounds__(kFB) void k_fl_level(
    const int32_t *__restrict__ front_in, const int32_t *__restrict__ cnt_in, int32_t *__restrict__ front_out,
    int32_t *__restrict__ cnt_out, int32_t *__restrict__ cnt_zero, int32_t L, int32_t nv,
    const int64_t *__restrict__ voffn, const int64_t *__restrict__ vadj, const int64_t *__restrict__ rbase,
    const int32_t *__restrict__ rends, const int32_t *__restrict__ head, const int64_t *__restrict__ res,
    const uint8_t *__restrict__ term, uint8_t *__restrict__ flag, int32_t *__restrict__ h) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *cnt_zero = 0;
  const int32_t count = *cnt_in;
  const int l = lane_id();
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave; i < count;
       i += (int64_t)gridDim.x * blockDim.x / kWave) {
    const int64_t u = front_in[i];
    const int64_t deg = out_degree(u, nv, voffn, rends);
    for (int64_t j = l; j < deg; j += kWave) {
      const int64_t a = out_arc(u, j, nv, voffn, vadj, rbase);
      if ((BACK ? res[a ^ 1] : res[a]) <= 0) continue;
      const int32_t v = head[a];
      if (claim<REACH>(v, term, flag, h, L)) front_out[atomicAdd(cnt_out, 1)] = v;
    }
  }
}

// a search from one node: its flag set, the frontier {node}
__global__ void k_fl_seed_one(uint8_t *flag, int32_t node, int32_t *front, int32_t *cnt) {
  flag[node] = 1;
  front[0] = node;
  cnt[0] = 1;
  cnt[1] = 0;
}

// Push-relabel sweep: every active node (free, positive excess, height below 2N) pushes to its
// lowest residual neighbour if it is higher, else relabels to one above it.  Only u's thread lowers
// u's excess and the residuals of u's arcs, so a push never takes more than is there.
__global__ void k_fl_sweep(int64_t N, int32_t nv, const uint8_t *__restrict__ term, int32_t *__restrict__ h,
                           int64_t *__restrict__ ex, int64_t *__restrict__ res, const int32_t *__restrict__ head,
                           const int64_t *__restrict__ voffn, const int64_t *__restrict__ vadj,
                           const int64_t *__restrict__ rbase, const int32_t *__restrict__ rends, int64_t *sc) {
  const int32_t h2n = (int32_t)(2 * N);
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < N; u += (int64_t)gridDim.x * blockDim.x) {
    if (term[u] != 0) continue;
    for (int c = 0; c < kPushCycles; ++c) {
      const int64_t e = ld(&ex[u]);
      const int32_t hu = h[u];
      if (e <= 0 || hu >= h2n) break;
      int64_t best_a = -1;
      int32_t best_h = INT32_MAX;
      for_out(u, nv, voffn, vadj, rbase, rends, [&](int64_t a) {
        if (ld(&res[a]) <= 0) return;
        const int32_t hv = ld(&h[head[a]]);
        if (hv < best_h) {
          best_h = hv;
          best_a = a;
        }
      });
      if (best_a < 0) {  // cannot happen for a node with excess; reported, never left looping
        atomicAdd((unsigned long long *)&sc[kScErr], 1ull);
        __hip_atomic_store(&h[u], h2n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        break;
      }
      if (hu > best_h) {
        const int64_t r = ld(&res[best_a]);
        const int64_t d = e < r ? e : r;
        push(best_a, (int32_t)u, head[best_a], d, res, ex);
      } else {
        __hip_atomic_store(&h[u], best_h + 1 < h2n ? best_h + 1 : h2n, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
  }
}

// active nodes; a free node left with excess at height 2N would leave no valid flow: counted as an
// error
__global__ void k_fl_active(int64_t N, const uint8_t *__restrict__ term, const int32_t *__restrict__ h,
                            const int64_t *__restrict__ ex, int64_t *sc) {
  const int32_t h2n = (int32_t)(2 * N);
  int64_t cnt = 0, stuck = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < N; u += (int64_t)gridDim.x * blockDim.x) {
    if (term[u] != 0 || ex[u] <= 0) continue;
    if (h[u] < h2n) ++cnt;
    else ++stuck;
  }
  add_sc(sc, kScActive, cnt);
  add_sc(sc, kScErr, stuck);
}

__global__ void k_fl_sinkflow(int64_t N, const uint8_t *__restrict__ term, const int64_t *__restrict__ ex,
                              int64_t *sc) {
  int64_t f = 0;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < N; u += (int64_t)gridDim.x * blockDim.x)
    if (term[u] == 2) f += ex[u];
  add_sc(sc, kScFlow, f);
}

// ---- residual reachability ----

// weights of the vertices on the source side (S_r) and on the sink side (T_r): the region vertices'
// nodes, and the contracted terminals (weight cs on node 0, ct on node 1)
__global__ void k_fl_sidew(const int32_t *__restrict__ nvert, const int32_t *__restrict__ vw, int32_t nv,
                           const uint8_t *__restrict__ rs, const uint8_t *__restrict__ rt, int64_t cs, int64_t ct,
                           int64_t *sc) {
  int64_t w1 = 0, w2 = 0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // the contracted terminals: cs on node 0, ct on node 1
    w1 += (rs[0] ? cs : 0) + (rs[1] ? ct : 0);
    w2 += (rt[0] ? cs : 0) + (rt[1] ? ct : 0);
  }
  for (int64_t x = 2 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; x < nv; x += (int64_t)gridDim.x * blockDim.x) {
    const int64_t w = cv(vw, nvert[x - 2]);
    if (rs[x]) w1 += w;
    if (rt[x]) w2 += w;
  }
  add_sc(sc, kScW1, w1);
  add_sc(sc, kScW2, w2);
}

// piercing candidates: free vertex endpoints outside `mine` of nets with endpoints on both sides of
// it; the least key (in `theirs` << 31 | vertex ID) goes to sc[kScBest]
__global__ void k_fl_cand(int64_t mrel, const int64_t *__restrict__ rbase, const int32_t *__restrict__ rends,
                          const int32_t *__restrict__ tail, int32_t nv, const uint8_t *__restrict__ mine,
                          const uint8_t *__restrict__ theirs, const uint8_t *__restrict__ term,
                          const int32_t *__restrict__ nvert, int64_t *sc) {
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < mrel; r += (int64_t)gridDim.x * blockDim.x) {
    const int64_t B = rbase[r];
    const int32_t E = rends[r];
    bool in = false, out = false;
    for (int32_t j = 0; j < E; ++j) {
      if (mine[tail[B + 2 + 4 * (int64_t)j]]) in = true;
      else out = true;
    }
    if (!in || !out) continue;
    for (int32_t j = 0; j < E; ++j) {
      const int32_t x = tail[B + 2 + 4 * (int64_t)j];
      if (x < 2 || x >= nv || mine[x] || term[x] != 0) continue;
      const uint64_t key = ((uint64_t)theirs[x] << 31) | (uint64_t)nvert[x - 2];
      atomicMin((unsigned long long *)&sc[kScBest], (unsigned long long)key);
    }
  }
}

// the nodes of `mine` become terminals of that side; the piercing key is reset to `none`
__global__ void k_fl_absorb(int64_t N, const uint8_t *__restrict__ mine, uint8_t *__restrict__ term, uint8_t side,
                            int64_t *sc, int64_t none) {
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[kScBest] = none;
  for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < N; u += (int64_t)gridDim.x * blockDim.x)
    if (mine[u] && term[u] == 0) term[u] = side;
}

// the piercing vertex chosen by k_fl_cand (if any) becomes a terminal of `side`
__global__ void k_fl_pierce(const int64_t *sc, const int32_t *__restrict__ vnode, uint8_t *__restrict__ term,
                            uint8_t side, int64_t none) {
  const int64_t key = sc[kScBest];
  if (key != none) term[vnode[key & 0x7fffffff]] = side;
}


// the chosen bipartition onto the region vertices
__global__ void k_fl_apply(const int32_t *__restrict__ vnode, int32_t n, int32_t nv, int32_t a, int32_t b,
                           int32_t use_source_side, const uint8_t *__restrict__ rs, const uint8_t *__restrict__ rt,
                           int32_t *__restrict__ part, int64_t *sc) {
  int64_t moved = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = vnode[v];
    if (x < 2 || x >= nv) continue;
    const bool src = use_source_side ? rs[x] != 0 : rt[x] == 0;
    const int32_t nb = src ? a : b;
    if (part[v] != nb) {
      part[v] = nb;
      ++moved;
    }
  }
  add_sc(sc, kScMoved, moved);
}

__global__ void k_fl_export(const int32_t *__restrict__ vnode, int32_t n, const uint8_t *__restrict__ rs,
                            const uint8_t *__restrict__ rt, uint8_t *__restrict__ in_sr, uint8_t *__restrict__ in_tr) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = vnode[v];
    in_sr[v] = x >= 0 ? rs[x] : 0;
    in_tr[v] = x >= 0 ? rt[x] : 0;
  }
}

// ---- k-way schedule ----

// connectivity metric sum_e w(e) (lambda(e) - 1) into sc[kScFlow]; with quot != nullptr also
// quot[i * k + j] = 1 for every two blocks i < j that share a net
__global__ void k_fl_km1_quot(const int64_t *__restrict__ off, const int32_t *__restrict__ pins,
                              const int32_t *__restrict__ nw, const int32_t *__restrict__ part, int32_t m, int32_t k,
                              uint8_t *__restrict__ quot, int64_t *sc) {
  int64_t km1 = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    uint64_t lo = 0, hi = 0;
    for (int64_t q = off[e]; q < off[e + 1]; ++q) {
      const int32_t x = part[pins[q]];
      if (x < 64) lo |= 1ull << x;
      else hi |= 1ull << (x - 64);
    }
    const int lam = __popcll(lo) + __popcll(hi);
    km1 += (int64_t)(lam - 1) * wn(nw, (int32_t)e);
    if (!quot || lam < 2) continue;
    for (uint64_t a1 = lo, a2 = hi; a1 | a2;) {
      const int32_t i = a1 ? __builtin_ctzll(a1) : 64 + __builtin_ctzll(a2);
      if (a1) a1 &= a1 - 1;
      else a2 &= a2 - 1;
      for (uint64_t b1 = a1, b2 = a2; b1 | b2;) {
        const int32_t j = b1 ? __builtin_ctzll(b1) : 64 + __builtin_ctzll(b2);
        if (b1) b1 &= b1 - 1;
        else b2 &= b2 - 1;
        quot[(int64_t)i * k + j] = 1;
      }
    }
  }
  add_sc(sc, kScFlow, km1);
}

// ---- host side ----

int hip_fail(Ctx &c, hipError_t e, const char *what) {
  c.last_error = std::string(what) + ": " + hipGetErrorString(e);
  return JET_EHIP;
}

#define FL_OK(expr)                                  \
  do {                                               \
    hipError_t _e = (expr);                          \
    if (_e != hipSuccess) return hip_fail(c, _e, #expr); \
  } while (0)

#define FL_RC(expr)             \
  do {                          \
    int _rc = (expr);           \
    if (_rc != JET_OK) return _rc; \
  } while (0)

template <typename T>
hipError_t falloc(T **p, int64_t count) {
  *p = nullptr;  // stays null if the allocation fails
  return hipMalloc((void **)p, sizeof(T) * (size_t)(count > 0 ? count : 1));
}

int alloc_state(Ctx &c) {
  FlowState &s = *c.fl;
  const int64_t n = c.n, m = c.m;
  FL_OK(falloc(&s.cnt_a, m));
  FL_OK(falloc(&s.cnt_b, m));
  FL_OK(falloc(&s.nexp, m));
  FL_OK(falloc(&s.ends, m));
  FL_OK(falloc(&s.asize, m));
  FL_OK(falloc(&s.rel, m));
  FL_OK(falloc(&s.nbase, m + 1));
  FL_OK(falloc(&s.nrid, m + 1));
  FL_OK(falloc(&s.rnet, m));
  FL_OK(falloc(&s.rends, m));
  FL_OK(falloc(&s.rbase, m));
  FL_OK(falloc(&s.lvl, n));
  FL_OK(falloc(&s.rmark, n));
  FL_OK(falloc(&s.wtmp, n));
  FL_OK(falloc(&s.wscan, n + 1));
  FL_OK(falloc(&s.vnode, n));
  FL_OK(falloc(&s.nvert, n));
  FL_OK(falloc(&s.vcnt, n + 2));
  FL_OK(falloc(&s.voffn, n + 3));
  FL_OK(falloc(&s.sc, kScN));
  FL_OK(falloc(&s.fcnt, 3));
  FL_OK(hipHostMalloc((void **)&s.hsc, sizeof(int64_t) * kScN));
  return JET_OK;
}

// The per-context flow state, allocated at the first flow call; a partly allocated state is freed
// again, so a later call starts over instead of using missing arrays.
int ensure_state(Ctx &c) {
  if (c.fl) return JET_OK;
  c.fl = new FlowState();
  const int rc = alloc_state(c);
  if (rc != JET_OK) flow_free(c);
  return rc;
}

template <typename T>
void release(T *&p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Grows the network arrays; a capacity is raised only once all its arrays are allocated, and a
// freed array is cleared at once, so a failed allocation leaves nothing to free twice.
int grow(Ctx &c, int64_t nodes, int64_t arcs, int64_t vadj) {
  FlowState &s = *c.fl;
  if (nodes > s.node_cap) {
    s.node_cap = 0;
    release(s.h);
    release(s.ex);
    release(s.term);
    release(s.rs);
    release(s.rt);
    for (int i = 0; i < 3; ++i) release(s.front[i]);
    FL_OK(falloc(&s.h, nodes));
    FL_OK(falloc(&s.ex, nodes));
    FL_OK(falloc(&s.term, nodes));
    FL_OK(falloc(&s.rs, nodes + 8));  // byte flags are claimed through their aligned 4-byte word
    FL_OK(falloc(&s.rt, nodes + 8));
    for (int i = 0; i < 3; ++i) FL_OK(falloc(&s.front[i], nodes));
    s.node_cap = nodes;
  }
  if (arcs > s.arc_cap) {
    s.arc_cap = 0;
    release(s.head);
    release(s.tail);
    release(s.res);
    FL_OK(falloc(&s.head, arcs));
    FL_OK(falloc(&s.tail, arcs));
    FL_OK(falloc(&s.res, arcs));
    s.arc_cap = arcs;
  }
  if (vadj > s.vadj_cap) {
    s.vadj_cap = 0;
    release(s.vadj);
    FL_OK(falloc(&s.vadj, vadj));
    s.vadj_cap = vadj;
  }
  return JET_OK;
}

// the pair's scalars, read to the host: sc slots copied into s.hsc
int read_sc(Ctx &c) {
  FlowState &s = *c.fl;
  FL_OK(hipMemcpyAsync(s.hsc, s.sc, sizeof(int64_t) * kScN, hipMemcpyDeviceToHost, c.stream));
  FL_OK(hipStreamSynchronize(c.stream));
  return JET_OK;
}

// Clears the scalar slots except the error count, which lasts for the whole call.  The host
// mirror is cleared with them: it always holds the value a slot had at its last read (or clear),
// so the loops of the piercing step take differences of sums instead of clearing the device slots
// before every launch.
int zero_sc(Ctx &c) {
  FL_OK(hipMemsetAsync(c.fl->sc, 0, sizeof(int64_t) * kScErr, c.stream));
  for (int i = 0; i < kScErr; ++i) c.fl->hsc[i] = 0;
  return JET_OK;
}

int start_call(Ctx &c) {
  FL_OK(hipMemsetAsync(c.fl->sc, 0, sizeof(int64_t) * kScN, c.stream));
  for (int i = 0; i < kScN; ++i) c.fl->hsc[i] = 0;
  return JET_OK;
}

int64_t total_weight_bound(const Ctx &c, int32_t alpha) {
  return (int64_t)std::floor((1.0 + (double)alpha * c.eps) * (double)c.A);
}

// per-net pin counts of the pair, its induced cut and block weights (into hsc)
int pair_scalars(Ctx &c, const int32_t *part, int32_t a, int32_t b) {
  FlowState &s = *c.fl;
  FL_RC(zero_sc(c));
  hipLaunchKernelGGL(k_fl_nets, dim3(fgrid(c.m)), dim3(kFB), 0, c.stream, c.off, c.pins, c.nw, part, c.m, a, b,
                     s.cnt_a, s.cnt_b, s.sc);
  hipLaunchKernelGGL(k_fl_bw, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, part, c.vw, c.n, a, b, s.sc);
  FL_OK(hipGetLastError());
  return read_sc(c);
}

// one side's region: rmark = mark on the taken vertices; returns the count in *taken
int grow_side(Ctx &c, const int32_t *part, int32_t side, const int32_t *cnt_other, int64_t bound, int8_t mark,
              int32_t *taken, int64_t *weight) {
  FlowState &s = *c.fl;
  hipLaunchKernelGGL(k_fl_fill, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, s.lvl, (int64_t)c.n, -1);
  hipLaunchKernelGGL(k_fl_fill, dim3(fgrid(c.m)), dim3(kFB), 0, c.stream, s.nexp, (int64_t)c.m, 0);
  FL_RC(zero_sc(c));
  hipLaunchKernelGGL(k_fl_level0, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, c.voff, c.inc, part, cnt_other, c.vw,
                     c.n, side, s.lvl, s.sc);
  FL_OK(hipGetLastError());
  FL_RC(read_sc(c));
  int64_t used = 0, count = 0;
  for (int32_t L = 0;; ++L) {
    const int64_t lw = s.hsc[kScLw];
    if (lw == 0) break;
    if (used + lw <= bound) {
      used += lw;
      FL_RC(zero_sc(c));
      hipLaunchKernelGGL(k_fl_take, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, s.lvl, c.n, L, s.rmark, mark, s.sc);
      hipLaunchKernelGGL(k_fl_expand, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, c.voff, c.inc, c.off, c.pins, part,
                         c.vw, c.n, side, L, s.lvl, s.nexp, s.sc);
      FL_OK(hipGetLastError());
      FL_RC(read_sc(c));
      count += s.hsc[kScCnt];
    } else {
      hipLaunchKernelGGL(k_fl_level_w, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, s.lvl, c.vw, c.n, L, s.wtmp);
      FL_OK(launch_exclusive_scan_i32_to_i64(c, s.wtmp, s.wscan, c.n));
      FL_RC(zero_sc(c));
      hipLaunchKernelGGL(k_fl_take_partial, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, s.lvl, s.wscan, c.vw, c.n, L,
                         bound - used, s.rmark, mark, s.sc);
      FL_OK(hipGetLastError());
      FL_RC(read_sc(c));
      count += s.hsc[kScCnt];
      used += s.hsc[kScLw];
      break;
    }
  }
  *taken = (int32_t)count;
  *weight = used;
  return JET_OK;
}

int regions(Ctx &c, const int32_t *part, int32_t a, int32_t b, int32_t alpha, int64_t bwa, int64_t bwb,
            int32_t *ra, int32_t *rb, int64_t *wa = nullptr, int64_t *wb = nullptr) {
  FlowState &s = *c.fl;
  const int64_t big = total_weight_bound(c, alpha);
  // a side never takes its whole block, so both terminal sets start non-empty
  const int64_t bound_a = std::max<int64_t>(0, std::min(big - bwb, bwa - 1));
  const int64_t bound_b = std::max<int64_t>(0, std::min(big - bwa, bwb - 1));
  hipLaunchKernelGGL(k_fl_fill8, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, s.rmark, (int64_t)c.n, (int8_t)0);
  int64_t ua = 0, ub = 0;
  FL_RC(grow_side(c, part, a, s.cnt_b, bound_a, 1, ra, &ua));
  FL_RC(grow_side(c, part, b, s.cnt_a, bound_b, 2, rb, &ub));
  if (wa) *wa = ua;
  if (wb) *wb = ub;
  return JET_OK;
}

// network of the pair; free vertices from rmark (term == nullptr) or from term
struct Net {
  int64_t N = 0, A = 0, mrel = 0;
  int32_t nv = 0;
};

int build_net(Ctx &c, const int32_t *part, int32_t a, int32_t b, const int8_t *term, Net *net) {
  FlowState &s = *c.fl;
  hipLaunchKernelGGL(k_fl_free, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, part, s.rmark, term, c.n, a, b, s.wtmp);
  FL_OK(launch_exclusive_scan_i32_to_i64(c, s.wtmp, s.wscan, c.n));
  hipLaunchKernelGGL(k_fl_vnode, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, part, term, s.wtmp, s.wscan, c.n, a, b,
                     s.vnode, s.nvert);
  FL_RC(zero_sc(c));
  hipLaunchKernelGGL(k_fl_ends, dim3(fgrid(c.m)), dim3(kFB), 0, c.stream, c.off, c.pins, c.nw, s.vnode, c.m, s.ends,
                     s.asize, s.rel, s.sc);
  FL_OK(launch_exclusive_scan_i32_to_i64(c, s.asize, s.nbase, c.m));
  FL_OK(launch_exclusive_scan_i32_to_i64(c, s.rel, s.nrid, c.m));
  hipLaunchKernelGGL(k_fl_nmeta, dim3(fgrid(c.m)), dim3(kFB), 0, c.stream, s.rel, s.nrid, s.nbase, s.ends, c.m,
                     s.rnet, s.rbase, s.rends);
  int64_t nfree = 0, arcs = 0, mrel = 0;
  FL_OK(hipMemcpyAsync(&nfree, s.wscan + c.n, sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
  FL_OK(hipMemcpyAsync(&arcs, s.nbase + c.m, sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
  FL_OK(hipMemcpyAsync(&mrel, s.nrid + c.m, sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
  FL_RC(read_sc(c));
  const int64_t wsum = s.hsc[kScWsum];
  net->nv = (int32_t)(2 + nfree);
  net->mrel = mrel;
  net->N = 2 + nfree + 2 * mrel;
  net->A = arcs;
  if (net->N >= (int64_t)1 << 30 || net->A >= (int64_t)1 << 40) {
    c.last_error = "flow network too large";
    return JET_EUNSUPPORTED;
  }
  // vertex-node adjacency
  hipLaunchKernelGGL(k_fl_fill, dim3(fgrid(net->nv)), dim3(kFB), 0, c.stream, s.vcnt, (int64_t)net->nv, 0);
  hipLaunchKernelGGL(k_fl_adj_count, dim3(fgrid(mrel)), dim3(kFB), 0, c.stream, c.off, c.pins, s.vnode, mrel, s.rnet,
                     s.vcnt);
  FL_OK(launch_exclusive_scan_i32_to_i64(c, s.vcnt, s.voffn, net->nv));
  int64_t nadj = 0;
  FL_OK(hipMemcpyAsync(&nadj, s.voffn + net->nv, sizeof(int64_t), hipMemcpyDeviceToHost, c.stream));
  FL_OK(hipStreamSynchronize(c.stream));
  FL_RC(grow(c, net->N, net->A, nadj));
  hipLaunchKernelGGL(k_fl_fill, dim3(fgrid(net->nv)), dim3(kFB), 0, c.stream, s.vcnt, (int64_t)net->nv, 0);
  hipLaunchKernelGGL(k_fl_build, dim3(fgrid(mrel)), dim3(kFB), 0, c.stream, c.off, c.pins, c.nw, s.vnode, mrel,
                     s.rnet, s.rbase, net->nv, wsum + 1, s.voffn, s.vcnt, s.head, s.tail, s.res, s.vadj);
  hipLaunchKernelGGL(k_fl_init_nodes, dim3(fgrid(net->N)), dim3(kFB), 0, c.stream, net->N, s.term, s.h, s.ex);
  FL_OK(hipGetLastError());
  return JET_OK;
}

// Runs the later levels of a search whose frontier is in front[0] / fcnt[0] (fcnt[1] clear): level
// launches between two looks at the frontier size double while the search goes on (a level after
// the last finds an empty frontier and does nothing).  L is the label of the frontier's nodes.
template <bool BACK, bool REACH>
int levels(Ctx &c, const Net &net, uint8_t *flag, int32_t L) {
  FlowState &s = *c.fl;
  // most levels of a deep search hold few nodes: a modest grid strides over a large frontier rather
  // than dispatching idle workgroups at every level
  const unsigned grid = (unsigned)std::min<int64_t>(kLevelGrid, std::max<int64_t>(1, net.N * kWave / kFB));
  int cur = 0;
  for (int batch = kLevelBatch;; batch = std::min(2 * batch, kLevelBatchMax)) {
    for (int i = 0; i < batch; ++i) {
      const int out = (cur + 1) % 3, zero = (cur + 2) % 3;
      hipLaunchKernelGGL((k_fl_level<BACK, REACH>), dim3(grid), dim3(kFB), 0, c.stream, s.front[cur], s.fcnt + cur,
                         s.front[out], s.fcnt + out, s.fcnt + zero, L, net.nv, s.voffn, s.vadj, s.rbase, s.rends,
                         s.head, s.res, s.term, flag, s.h);
      cur = out;
      ++L;
    }
    FL_OK(hipGetLastError());
    int32_t left = 0;
    FL_OK(hipMemcpyAsync(&left, s.fcnt + cur, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
    FL_OK(hipStreamSynchronize(c.stream));
    if (left == 0) break;
  }
  return JET_OK;
}

// a whole search from the terminals of `side`
template <bool BACK, bool REACH>
int search(Ctx &c, const Net &net, uint8_t side, uint8_t *flag, int32_t L) {
  FlowState &s = *c.fl;
  FL_OK(hipMemsetAsync(s.fcnt, 0, sizeof(int32_t) * 3, c.stream));
  hipLaunchKernelGGL((k_fl_first<BACK, REACH>), dim3(fgrid(net.A)), dim3(kFB), 0, c.stream, net.A, s.tail, s.head,
                     s.res, s.term, side, flag, s.h, L, s.front[0], s.fcnt);
  FL_OK(hipGetLastError());
  return levels<BACK, REACH>(c, net, flag, L + 1);
}

// heights: breadth-first distance to the sinks, else N + distance to the sources, else 2N
int global_relabel(Ctx &c, const Net &net) {
  FlowState &s = *c.fl;
  hipLaunchKernelGGL(k_fl_gr_init, dim3(fgrid(net.N)), dim3(kFB), 0, c.stream, net.N, s.term, s.h);
  FL_RC((search<true, false>(c, net, 2, nullptr, 0)));
  FL_RC((search<true, false>(c, net, 1, nullptr, (int32_t)net.N)));
  hipLaunchKernelGGL(k_fl_gr_rest, dim3(fgrid(net.N)), dim3(kFB), 0, c.stream, net.N, s.term, s.h);
  FL_OK(hipGetLastError());
  return JET_OK;
}

// maximum flow from the current one for the current terminals; its value in *flow
int max_flow(Ctx &c, const Net &net, int64_t *flow) {
  FlowState &s = *c.fl;
  using clock = std::chrono::steady_clock;
  hipLaunchKernelGGL(k_fl_saturate, dim3(fgrid(net.A)), dim3(kFB), 0, c.stream, net.A, s.tail, s.head, s.term, s.res,
                     s.ex);
  FL_OK(hipGetLastError());
  auto t0 = clock::now();
  FL_RC(global_relabel(c, net));
  // A global relabel costs a few hundred launches on a deep network and little on a shallow one:
  // the next one comes once the sweeps since the last have taken twice as long as it did.  (Heights
  // only steer the pushes; the flow value and the cut sides do not depend on them.)
  double relabel_s = std::chrono::duration<double>(clock::now() - t0).count(), sweeps_s = 0.0;
  for (int64_t check = 0;; ++check) {
    if (check >= kMaxChecks) {
      c.last_error = "flow: push-relabel did not finish";
      return JET_EHIP;
    }
    if (sweeps_s > 2.0 * relabel_s) {
      t0 = clock::now();
      FL_RC(global_relabel(c, net));
      relabel_s = std::chrono::duration<double>(clock::now() - t0).count();
      sweeps_s = 0.0;
    }
    t0 = clock::now();
    for (int i = 0; i < kSweepsPerCheck; ++i)
      hipLaunchKernelGGL(k_fl_sweep, dim3(fgrid(net.N)), dim3(kFB), 0, c.stream, net.N, net.nv, s.term, s.h, s.ex,
                         s.res, s.head, s.voffn, s.vadj, s.rbase, s.rends, s.sc);
    const int64_t before = s.hsc[kScActive];
    hipLaunchKernelGGL(k_fl_active, dim3(fgrid(net.N)), dim3(kFB), 0, c.stream, net.N, s.term, s.h, s.ex, s.sc);
    FL_OK(hipGetLastError());
    FL_RC(read_sc(c));
    sweeps_s += std::chrono::duration<double>(clock::now() - t0).count();
    if (s.hsc[kScErr] != 0) {
      c.last_error = "flow: a node with excess cannot push";
      return JET_EHIP;
    }
    if (s.hsc[kScActive] == before) break;
  }
  const int64_t before = s.hsc[kScFlow];
  hipLaunchKernelGGL(k_fl_sinkflow, dim3(fgrid(net.N)), dim3(kFB), 0, c.stream, net.N, s.term, s.ex, s.sc);
  FL_OK(hipGetLastError());
  FL_RC(read_sc(c));
  *flow = s.hsc[kScFlow] - before;
  return JET_OK;
}

// residual reachability for the sides in dir (bit 1: rs, bit 2: rt) from scratch, or, with
// from >= 0 and one bit, the side's set grown by the nodes reachable from node `from`
int reach(Ctx &c, const Net &net, int32_t dir, int32_t from = -1) {
  FlowState &s = *c.fl;
  for (int d = 1; d <= 2; ++d) {
    if (!(dir & d)) continue;
    uint8_t *flag = d == 1 ? s.rs : s.rt;
    if (from >= 0) {
      hipLaunchKernelGGL(k_fl_seed_one, dim3(1), dim3(1), 0, c.stream, flag, from, s.front[0], s.fcnt);
      FL_OK(hipGetLastError());
      if (d == 1) FL_RC((levels<false, true>(c, net, flag, 0)));
      else FL_RC((levels<true, true>(c, net, flag, 0)));
    } else {
      hipLaunchKernelGGL(k_fl_reach_init, dim3(fgrid(net.N)), dim3(kFB), 0, c.stream, net.N, s.term, d, s.rs, s.rt);
      if (d == 1) FL_RC((search<false, true>(c, net, 1, flag, 0)));
      else FL_RC((search<true, true>(c, net, 2, flag, 0)));
    }
  }
  return JET_OK;
}

int check_err(Ctx &c) {
  FL_RC(read_sc(c));
  if (c.fl->hsc[kScErr] != 0) {
    c.last_error = "flow: a node with excess had no residual arc";
    return JET_EHIP;
  }
  return JET_OK;
}

}  // namespace

void flow_free(Ctx &c) {
  if (!c.fl) return;
  FlowState &s = *c.fl;
  for (void *p : {(void *)s.cnt_a, (void *)s.cnt_b, (void *)s.nexp, (void *)s.ends, (void *)s.asize, (void *)s.rel,
                  (void *)s.nbase, (void *)s.nrid, (void *)s.rnet, (void *)s.rends, (void *)s.rbase, (void *)s.lvl,
                  (void *)s.rmark, (void *)s.wtmp, (void *)s.wscan, (void *)s.vnode, (void *)s.nvert,
                  (void *)s.vcnt, (void *)s.voffn, (void *)s.sc, (void *)s.head, (void *)s.tail, (void *)s.res,
                  (void *)s.vadj, (void *)s.h, (void *)s.ex, (void *)s.term, (void *)s.rs, (void *)s.rt,
                  (void *)s.front[0], (void *)s.front[1], (void *)s.front[2], (void *)s.fcnt})
    if (p) (void)hipFree(p);
  if (s.hsc) (void)hipHostFree(s.hsc);
  delete c.fl;
  c.fl = nullptr;
}

int flow_region(Ctx &c, const int32_t *part, int32_t a, int32_t b, int32_t alpha, int8_t *region) {
  FL_RC(ensure_state(c));
  FL_RC(start_call(c));
  FL_RC(pair_scalars(c, part, a, b));
  FlowState &s = *c.fl;
  int32_t ra = 0, rb = 0;
  FL_RC(regions(c, part, a, b, alpha, s.hsc[kScBwA], s.hsc[kScBwB], &ra, &rb));
  FL_OK(hipMemcpyAsync(region, s.rmark, (size_t)c.n, hipMemcpyDeviceToDevice, c.stream));
  FL_OK(hipStreamSynchronize(c.stream));
  return JET_OK;
}

int flow_mincut(Ctx &c, const int32_t *part, int32_t a, int32_t b, const int8_t *term, int64_t *flow,
                uint8_t *in_sr, uint8_t *in_tr) {
  FL_RC(ensure_state(c));
  FL_RC(start_call(c));
  FlowState &s = *c.fl;
  Net net;
  FL_RC(build_net(c, part, a, b, term, &net));
  FL_RC(max_flow(c, net, flow));
  FL_RC(reach(c, net, 3));
  hipLaunchKernelGGL(k_fl_export, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, s.vnode, c.n, s.rs, s.rt, in_sr, in_tr);
  FL_OK(hipGetLastError());
  FL_RC(check_err(c));
  return JET_OK;
}

// Algorithm 3 for the pair (a, b); readings F1-F3 of the design notes
int flow_pair(Ctx &c, int32_t *part, int32_t a, int32_t b, int32_t alpha, FlowPairResult *out) {
  FL_RC(ensure_state(c));
  FL_RC(start_call(c));
  FlowState &s = *c.fl;
  FlowPairResult r;
  FL_RC(pair_scalars(c, part, a, b));
  r.old_cut = r.new_cut = s.hsc[kScCut];
  const int64_t bwa = s.hsc[kScBwA], bwb = s.hsc[kScBwB];
  if (r.old_cut == 0) {
    *out = r;
    return JET_OK;
  }
  int64_t rwa = 0, rwb = 0;  // weights of the two sides of the region
  FL_RC(regions(c, part, a, b, alpha, bwa, bwb, &r.region_a, &r.region_b, &rwa, &rwb));
  Net net;
  FL_RC(build_net(c, part, a, b, nullptr, &net));
  const int64_t wab = bwa + bwb, heavier_old = std::max(bwa, bwb), lmax = c.lmax;
  // After a piercing vertex the other side does not reach, no augmenting path can exist: the flow
  // stays maximum and only the pierced side's reachable set changes (the other side's residual
  // network and terminals are as they were).
  int64_t F = 0;
  int32_t need = 3;  // 3: maximum flow and both sets; 1 / 2: only the source / sink side's set
  int32_t pierced = -1;
  for (int64_t guard = 0; guard <= (int64_t)net.nv + 2; ++guard) {
    if (need == 3) {
      FL_RC(max_flow(c, net, &F));
      FL_RC(reach(c, net, 3));
    } else {
      FL_RC(reach(c, net, need, pierced));
    }
    ++r.iterations;
    r.arcs += net.A;
    if (F > r.old_cut) break;
    const int64_t w1_before = s.hsc[kScW1], w2_before = s.hsc[kScW2];
    hipLaunchKernelGGL(k_fl_sidew, dim3(fgrid(net.nv)), dim3(kFB), 0, c.stream, s.nvert, c.vw, net.nv, s.rs, s.rt,
                       bwa - rwa, bwb - rwb, s.sc);
    FL_OK(hipGetLastError());
    FL_RC(read_sc(c));
    const int64_t w1 = s.hsc[kScW1] - w1_before, w2 = s.hsc[kScW2] - w2_before;
    const int64_t h1 = std::max(w1, wab - w1), h2 = std::max(w2, wab - w2);
    const bool bal1 = w1 <= lmax && wab - w1 <= lmax;
    const bool bal2 = w2 <= lmax && wab - w2 <= lmax;
    if (bal1 || bal2) {
      const bool use1 = bal1 && (!bal2 || h1 <= h2);
      const int64_t hv = use1 ? h1 : h2;
      if (F < r.old_cut || hv < heavier_old) {
        FL_RC(zero_sc(c));
        hipLaunchKernelGGL(k_fl_apply, dim3(fgrid(c.n)), dim3(kFB), 0, c.stream, s.vnode, c.n, net.nv, a, b,
                           use1 ? 1 : 0, s.rs, s.rt, part, s.sc);
        FL_OK(hipGetLastError());
        FL_RC(read_sc(c));
        r.moved = (int32_t)s.hsc[kScMoved];
        r.new_cut = F;
        r.replaced = 1;
      }
      break;
    }
    if (F >= r.old_cut) break;  // the termination check comes before piercing
    const bool source_side = w1 <= w2;
    const uint8_t *mine = source_side ? s.rs : s.rt;
    const uint8_t *theirs = source_side ? s.rt : s.rs;
    const uint8_t side = source_side ? 1 : 2;
    const int64_t none = (int64_t)1 << 40;
    hipLaunchKernelGGL(k_fl_absorb, dim3(fgrid(net.N)), dim3(kFB), 0, c.stream, net.N, mine, s.term, side, s.sc,
                       none);
    hipLaunchKernelGGL(k_fl_cand, dim3(fgrid(net.mrel)), dim3(kFB), 0, c.stream, net.mrel, s.rbase, s.rends, s.tail,
                       net.nv, mine, theirs, s.term, s.nvert, s.sc);
    hipLaunchKernelGGL(k_fl_pierce, dim3(1), dim3(1), 0, c.stream, s.sc, s.vnode, s.term, side, none);
    FL_OK(hipGetLastError());
    FL_RC(read_sc(c));
    const int64_t key = s.hsc[kScBest];
    if (key == none) break;
    // a piercing vertex the other side does not reach opens no augmenting path
    need = (key >> 31) & 1 ? 3 : side;
    FL_OK(hipMemcpyAsync(&pierced, s.vnode + (key & 0x7fffffff), sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
    FL_OK(hipStreamSynchronize(c.stream));
  }
  FL_RC(check_err(c));
  *out = r;
  return JET_OK;
}

// metric and (quot != nullptr) quotient-graph edges of part
int km1_quot(Ctx &c, const int32_t *part, uint8_t *quot_dev, std::vector<uint8_t> *quot, int64_t *km1) {
  FlowState &s = *c.fl;
  const int64_t kk = (int64_t)c.k * c.k;
  if (quot_dev) FL_OK(hipMemsetAsync(quot_dev, 0, (size_t)kk, c.stream));
  FL_RC(zero_sc(c));
  hipLaunchKernelGGL(k_fl_km1_quot, dim3(fgrid(c.m)), dim3(kFB), 0, c.stream, c.off, c.pins, c.nw, part, c.m, c.k,
                     quot_dev, s.sc);
  FL_OK(hipGetLastError());
  if (quot_dev) {
    quot->resize((size_t)kk);
    FL_OK(hipMemcpyAsync(quot->data(), quot_dev, (size_t)kk, hipMemcpyDeviceToHost, c.stream));
  }
  FL_RC(read_sc(c));
  *km1 = s.hsc[kScFlow];
  return JET_OK;
}

// k-way refinement with the matching schedule of Section 5.2 (reading F4 of the design notes)
int flow_refine(Ctx &c, int32_t *part, int32_t alpha, int32_t max_rounds, FlowRefineResult *out) {
  FL_RC(ensure_state(c));
  FL_RC(start_call(c));
  const int32_t k = c.k;
  FlowRefineResult r;
  uint8_t *quot_dev = nullptr;
  FL_OK(falloc(&quot_dev, (int64_t)k * k));
  std::vector<uint8_t> quot;
  int rc = km1_quot(c, part, nullptr, nullptr, &r.km1_in);
  // worker contexts: the hypergraph of c with a stream, scan scratch and flow state of their own
  // (with one worker the pairs run on c itself, on the calling thread)
  int device = 0;
  FL_OK(hipGetDevice(&device));
  FL_OK(hipStreamSynchronize(c.stream));
  std::vector<Ctx *> workers;
  const int32_t nworkers = std::min<int32_t>(c.flow_workers, std::max<int32_t>(1, k / 2));
  if (nworkers == 1) workers.push_back(&c);
  for (int32_t w = 0; nworkers > 1 && w < nworkers && rc == JET_OK; ++w) {
    Ctx *x = new Ctx(c);
    x->fl = nullptr;
    x->co = nullptr;
    x->scan_tmp = nullptr;
    x->scan_tmp_len = 0;
    x->last_error.clear();
    workers.push_back(x);
    hipError_t e = hipStreamCreateWithFlags(&x->stream, hipStreamNonBlocking);
    if (e != hipSuccess) {
      x->stream = nullptr;
      rc = hip_fail(c, e, "hipStreamCreateWithFlags");
    }
  }
  std::vector<uint8_t> active((size_t)k, 1), next((size_t)k, 0), edge((size_t)k * k, 0);
  std::vector<int32_t> deg((size_t)k), order((size_t)k), mate((size_t)k);
  for (int32_t round = 0; rc == JET_OK && round < max_rounds; ++round) {
    int64_t unused = 0;
    if ((rc = km1_quot(c, part, quot_dev, &quot, &unused)) != JET_OK) break;
    int64_t remaining = 0;
    for (int32_t i = 0; i < k; ++i)
      for (int32_t j = 0; j < k; ++j) {
        const int32_t lo = std::min(i, j), hi = std::max(i, j);
        const bool on = i != j && quot[(size_t)lo * k + hi] && (active[(size_t)i] || active[(size_t)j]);
        edge[(size_t)i * k + j] = on;
        remaining += on && i < j;
      }
    if (remaining == 0) break;
    ++r.rounds;
    std::fill(next.begin(), next.end(), 0);
    while (remaining > 0 && rc == JET_OK) {
      for (int32_t i = 0; i < k; ++i) {
        deg[(size_t)i] = 0;
        for (int32_t j = 0; j < k; ++j) deg[(size_t)i] += edge[(size_t)i * k + j];
        order[(size_t)i] = i;
        mate[(size_t)i] = -1;
      }
      std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) {
        return deg[(size_t)x] != deg[(size_t)y] ? deg[(size_t)x] > deg[(size_t)y] : x < y;
      });
      for (int32_t i : order) {
        if (mate[(size_t)i] >= 0 || deg[(size_t)i] == 0) continue;
        int32_t best = -1;
        for (int32_t j = 0; j < k; ++j) {
          if (!edge[(size_t)i * k + j] || mate[(size_t)j] >= 0) continue;
          if (best < 0 || deg[(size_t)j] > deg[(size_t)best]) best = j;
        }
        if (best >= 0) {
          mate[(size_t)i] = best;
          mate[(size_t)best] = i;
        }
      }
      ++r.matchings;
      std::vector<std::pair<int32_t, int32_t>> pairs;
      for (int32_t i = 0; i < k; ++i) {
        const int32_t j = mate[(size_t)i];
        if (j < 0 || j < i) continue;
        edge[(size_t)i * k + j] = edge[(size_t)j * k + i] = 0;
        --remaining;
        pairs.emplace_back(i, j);
      }
      // The pairs of a matching are disjoint: each reads and writes only its two blocks' vertices,
      // so they run at once, one host thread and stream each, and the result is that of any order.
      std::vector<FlowPairResult> res(pairs.size());
      std::vector<int> rcs(pairs.size(), JET_OK);
      const size_t nw = std::min(pairs.size(), workers.size());
      auto work = [&](size_t w) {
        for (size_t q = w; q < pairs.size(); q += nw)
          if ((rcs[q] = flow_pair(*workers[w], part, pairs[q].first, pairs[q].second, alpha, &res[q])) != JET_OK)
            break;
      };
      if (nw == 1) {
        work(0);
      } else {
        std::vector<std::thread> th;
        for (size_t w = 0; w < nw; ++w)
          th.emplace_back([&, w] {
            (void)hipSetDevice(device);
            work(w);
          });
        for (auto &t : th) t.join();
      }
      for (size_t q = 0; q < pairs.size(); ++q) {
        if (rcs[q] != JET_OK) {
          rc = rcs[q];
          c.last_error = workers[q % nw]->last_error;
          break;
        }
        const FlowPairResult &pr = res[q];
        ++r.pairs;
        r.flow_calls += pr.iterations;
        r.arcs += pr.arcs;
        if (pr.replaced) {
          ++r.accepted;
          r.moved += pr.moved;
          if (pr.new_cut < pr.old_cut) next[(size_t)pairs[q].first] = next[(size_t)pairs[q].second] = 1;
        }
      }
      if (rc != JET_OK) break;
    }
    bool any = false;
    for (int32_t b = 0; b < k; ++b) {
      active[(size_t)b] = next[(size_t)b];
      any |= next[(size_t)b] != 0;
    }
    if (!any) break;
  }
  for (Ctx *x : workers) {
    if (x == &c) continue;
    flow_free(*x);
    if (x->scan_tmp) (void)hipFree(x->scan_tmp);
    if (x->stream) (void)hipStreamDestroy(x->stream);
    delete x;
  }
  if (rc == JET_OK) rc = km1_quot(c, part, nullptr, nullptr, &r.km1_out);
  (void)hipFree(quot_dev);
  if (rc == JET_OK) *out = r;
  return rc;
}

}  // namespace jet
