// Synchronous clustering of the coarsening phase (Section 6, Algorithm 4) on gfx950.
//
// One sub-round B_i (a contiguous slice of the caller's vertex order) runs as a short chain of
// kernels over the clustering (label[n] = cluster label of every vertex, cw[n] = weight of the
// cluster with that label):
//   k_co_rate     targets T[u] for the singletons of B_i: a group of eight lanes per vertex (a
//                 wave of its own for a vertex with a large table) accumulates the heavy-edge rating of
//                 every neighbouring cluster in the vertex's own open-addressing table (global
//                 scratch, sized from the vertex's incident pins); the nets of the vertex
//                 are taken one after the other and a per-slot "last net" mark makes each net count
//                 once per cluster; ratings are 32.32 fixed point, exact 64-bit integer sums, so
//                 the argmax (rating, then smallest label) does not depend on the order of atomics;
//   k_co_join     weight of the proposals per target;
//   k_co_swap     vertex-swap prevention: of a pair proposing each other the heavier side (its own
//                 weight plus the proposals it received, the smaller ID on a tie) keeps its place;
//                 every thread writes only its own vertex's target;
//   k_co_group    group-by target: counts per target and a group number per distinct target;
//   k_co_scan     group offsets (one workgroup);
//   k_co_scatter  proposals into their group's range;
//   k_co_approve  per group: sort by (weight, ID) in LDS (bitonic; rank sums for groups above the
//                 LDS capacity), prefix sums, approve the prefix that fits the room left in the
//                 target at the start of the sub-round;
//   k_co_apply    move the approved vertices, update cluster weights, clear the per-sub-round
//                 state (so it is all -1 / 0 again between sub-rounds).
// Sub-rounds of at most 1,024 vertices (the first hundred hold one) run k_co_join .. k_co_apply as
// the phases of one workgroup, k_co_settle_small, with barriers between the phases.
// All weight updates are integer atomics: the result is the same for any schedule of the waves.
#include <hip/hip_runtime.h>

#include "dev_util.h"
#include "jet_internal.h"

namespace jet {
namespace {

constexpr int kCoBlock = 256;
constexpr int kCoSortCap = 2048;  // largest group sorted in LDS

__device__ __forceinline__ int64_t cvw(const int32_t *vw, int32_t v) { return vw ? (int64_t)vw[v] : 1; }

__global__ void k_co_qnet(const int64_t *__restrict__ off, const int32_t *__restrict__ nw, int32_t m,
                          uint64_t *__restrict__ qnet) {
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t sz = off[e + 1] - off[e];
    const uint64_t w = nw ? (uint64_t)nw[e] : 1ull;
    qnet[e] = sz >= 2 ? (w << 32) / (uint64_t)(sz - 1) : 0ull;
  }
}

// D(v) = sum over incident nets with at least two pins of (|e| - 1): an upper bound on the number
// of neighbouring clusters, which sizes the vertex's rating table
__global__ void k_co_degree(const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
                            const int64_t *__restrict__ off, int32_t n, int64_t *__restrict__ deg) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int64_t d = 0;
    for (int64_t q = voff[v]; q < voff[v + 1]; ++q) {
      const int32_t e = inc[q];
      const int64_t sz = off[e + 1] - off[e];
      if (sz >= 2) d += sz - 1;
    }
    deg[v] = d;
  }
}

__global__ void k_co_init(int32_t *__restrict__ label, int64_t *__restrict__ cw, const int32_t *__restrict__ vw,
                          int32_t n) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    label[v] = (int32_t)v;
    cw[v] = cvw(vw, (int32_t)v);
  }
}

// bad[0] += entries of list[len] outside [0, n) or repeated; flag[n] must be zero and is left set
__global__ void k_co_check(const int32_t *__restrict__ list, int64_t len, int32_t n, int32_t *__restrict__ flag,
                           int32_t *__restrict__ bad) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = list[i];
    if (x < 0 || x >= n || atomicExch(&flag[x], 1) != 0) atomicAdd(bad, 1);
  }
}

// Rating of the vertex at list position t by G lanes (lane gl of G): its table is cleared, its nets
// are taken one after the other (the G lanes striding over a net's pins), and the best eligible
// cluster goes to tp[u].  G is 8 or 64; a group of G lanes is aligned to G within the wave.
constexpr int kU = 8;  // pins per lane in flight in the rating loop

template <int G>
__device__ __forceinline__ void rate_vertex(int64_t t, int gl, const int32_t *__restrict__ verts,
                                            const int64_t *__restrict__ ptab, int64_t base,
                                            const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
                                            const int64_t *__restrict__ off, const int32_t *__restrict__ pins,
                                            const uint64_t *__restrict__ qnet, const int32_t *__restrict__ vw,
                                            const int32_t *__restrict__ label, const int64_t *__restrict__ cw,
                                            int64_t wmax, CoSlot *__restrict__ tab, int32_t *__restrict__ tp) {
  const int32_t u = verts[t];
  const int64_t cap = ptab[t + 1] - ptab[t];
  const int64_t cu = cvw(vw, u);
  unsigned long long bv = 0ull;
  int32_t bk = -1;
  if (label[u] == u && cw[u] == cu && cap > 0) {  // a singleton with some neighbour
    CoSlot *T = tab + (ptab[t] - base);
    int4 *T4 = reinterpret_cast<int4 *>(T);  // slots are 16 bytes at 16-byte aligned offsets
    for (int64_t s = gl; s < cap; s += G) T4[s] = make_int4(-1, -1, 0, 0);
    __threadfence();
    const int shift = 32 - (63 - __builtin_clzll((unsigned long long)cap));
    const uint32_t mask = (uint32_t)(cap - 1);
    for (int64_t q = voff[u]; q < voff[u + 1]; ++q) {  // one net at a time (uniform in the group)
      const int32_t e = inc[q];
      const int64_t lo = off[e], hi = off[e + 1];
      if (hi - lo < 2) continue;
      const unsigned long long qe = qnet[e];
      // kU pins per lane at a time: their label loads and table atomics are independent, so they
      // are in flight together (pins of one cluster in one lane still hit one slot in order)
      for (int64_t r = lo + gl; r < hi; r += kU * G) {
        int32_t C[kU];
        uint32_t h[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) {
          const int64_t rj = r + (int64_t)j * G;
          const int32_t x = rj < hi ? pins[rj] : u;
          C[j] = x == u ? -1 : label[x];
        }
        int32_t k0[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) {
          h[j] = ((uint32_t)C[j] * 0x9E3779B1u) >> shift;
          k0[j] = C[j] >= 0 ? atomicCAS(&T[h[j]].key, -1, C[j]) : -1;
        }
#pragma unroll
        for (int j = 0; j < kU; ++j) {
          while (k0[j] != -1 && k0[j] != C[j]) {  // linear probing
            h[j] = (h[j] + 1) & mask;
            k0[j] = atomicCAS(&T[h[j]].key, -1, C[j]);
          }
        }
        int32_t m0[kU];
#pragma unroll
        for (int j = 0; j < kU; ++j) m0[j] = C[j] >= 0 ? atomicExch(&T[h[j]].mark, e) : e;
#pragma unroll
        for (int j = 0; j < kU; ++j)
          if (m0[j] != e) atomicAdd(&T[h[j]].val, qe);  // once per (net, cluster)
      }
    }
    __threadfence();
    for (int64_t s0 = gl; s0 < cap; s0 += kU * G) {
      int32_t k[kU];
      int64_t w[kU];
#pragma unroll
      for (int j = 0; j < kU; ++j) {
        const int64_t sj = s0 + (int64_t)j * G;
        k[j] = sj < cap ? __hip_atomic_load(&T[sj].key, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) : -1;
      }
#pragma unroll
      for (int j = 0; j < kU; ++j) w[j] = k[j] >= 0 ? cw[k[j]] : 0;
#pragma unroll
      for (int j = 0; j < kU; ++j) {
        if (k[j] < 0 || w[j] + cu > wmax) continue;  // the proposal-time weight filter
        const unsigned long long v =
            __hip_atomic_load(&T[s0 + (int64_t)j * G].val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        if (bk < 0 || v > bv || (v == bv && k[j] < bk)) {
          bv = v;
          bk = k[j];
        }
      }
    }
  }
#pragma unroll
  for (int o = G / 2; o >= 1; o >>= 1) {
    const unsigned long long ov = __shfl_xor(bv, o, kWave);
    const int32_t ok = __shfl_xor(bk, o, kWave);
    if (ok >= 0 && (bk < 0 || ov > bv || (ov == bv && ok < bk))) {
      bv = ov;
      bk = ok;
    }
  }
  if (gl == 0) tp[u] = bk;
}

constexpr int kCoGroup = 8;          // lanes per vertex for small tables
constexpr int64_t kCoSmallTable = 256;  // largest table rated by a group of kCoGroup lanes

// Two parts in one grid.  The first small_blocks workgroups: each wave takes kCoGroup consecutive
// list positions and rates those with small tables, a group of kCoGroup lanes per vertex.  The
// others: one wave per list position, rating it if its table is large.  A vertex with a large table
// meets many pins, so it gets a whole wave, and one wave each keeps enough of them in flight.
__global__ __launch_bounds__(kCoBlock) void k_co_rate(
    const int32_t *__restrict__ verts, int64_t a, int64_t b, uint32_t small_blocks, const int64_t *__restrict__ ptab,
    int64_t base, const int64_t *__restrict__ voff, const int32_t *__restrict__ inc, const int64_t *__restrict__ off,
    const int32_t *__restrict__ pins, const uint64_t *__restrict__ qnet, const int32_t *__restrict__ vw,
    const int32_t *__restrict__ label, const int64_t *__restrict__ cw, int64_t wmax, CoSlot *__restrict__ tab,
    int32_t *__restrict__ tp) {
  const int wave = (int)(threadIdx.x / kWave), l = lane_id();
  if (blockIdx.x >= small_blocks) {  // workgroup-uniform
    const int64_t t = a + (int64_t)(blockIdx.x - small_blocks) * (kCoBlock / kWave) + wave;
    if (t < b && ptab[t + 1] - ptab[t] > kCoSmallTable)
      rate_vertex<kWave>(t, l, verts, ptab, base, voff, inc, off, pins, qnet, vw, label, cw, wmax, tab, tp);
    return;
  }
  const int64_t t = a + ((int64_t)blockIdx.x * (kCoBlock / kWave) + wave) * (kWave / kCoGroup) + l / kCoGroup;
  if (t < b && ptab[t + 1] - ptab[t] <= kCoSmallTable)
    rate_vertex<kCoGroup>(t, l % kCoGroup, verts, ptab, base, voff, inc, off, pins, qnet, vw, label, cw, wmax, tab,
                          tp);
}

__global__ void k_co_join(const int32_t *__restrict__ verts, int64_t len, const int32_t *__restrict__ tp,
                          const int32_t *__restrict__ vw, unsigned long long *__restrict__ jw,
                          int32_t *__restrict__ ngroups) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *ngroups = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = verts[i];
    const int32_t j = tp[x];
    if (j >= 0) atomicAdd(&jw[j], (unsigned long long)cvw(vw, x));
  }
}

__global__ void k_co_swap(const int32_t *__restrict__ verts, int64_t len, const int32_t *__restrict__ tp,
                          const int32_t *__restrict__ vw, const unsigned long long *__restrict__ jw,
                          int32_t *__restrict__ tt) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = verts[i];
    const int32_t v = tp[x];
    int32_t tx = v;
    if (v >= 0 && tp[v] == x) {  // x and v propose each other (tp is -1 outside the sub-round)
      const int32_t lo = x < v ? x : v, hi = x < v ? v : x;
      const int64_t wl = cvw(vw, lo) + (int64_t)jw[lo] - cvw(vw, hi);
      const int64_t wh = cvw(vw, hi) + (int64_t)jw[hi] - cvw(vw, lo);
      const int32_t stay = wl >= wh ? lo : hi;
      tx = x == stay ? x : v;
    }
    tt[x] = tx;
  }
}

__global__ void k_co_group(const int32_t *__restrict__ verts, int64_t len, const int32_t *__restrict__ tt,
                           int32_t *__restrict__ gcnt, int32_t *__restrict__ gslot, int32_t *__restrict__ gtarget,
                           int32_t *__restrict__ gpos, int32_t *__restrict__ ngroups) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = verts[i];
    const int32_t j = tt[x];
    if (j < 0 || j == x) continue;  // no target, or keeps its place
    gpos[i] = atomicAdd(&gcnt[j], 1);
    if (atomicCAS(&gslot[j], -1, -2) == -1) {
      const int32_t g = atomicAdd(ngroups, 1);
      gtarget[g] = j;
      atomicExch(&gslot[j], g);
    }
  }
}

__global__ __launch_bounds__(1024) void k_co_scan(const int32_t *__restrict__ gcnt,
                                                  const int32_t *__restrict__ gtarget,
                                                  const int32_t *__restrict__ ngroups, int64_t *__restrict__ goff) {
  __shared__ int64_t sm[1024 / kWave + 1];
  const int32_t G = *ngroups;
  int64_t carry = 0;
  for (int32_t g0 = 0; g0 < G; g0 += 1024) {
    const int32_t g = g0 + (int32_t)threadIdx.x;
    const int64_t sz = g < G ? (int64_t)gcnt[gtarget[g]] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan<1024, int64_t>(sz, sm, &tot);
    if (g < G) goff[g] = carry + ex;
    carry += tot;
  }
  if (threadIdx.x == 0) goff[G] = carry;
}

__global__ void k_co_scatter(const int32_t *__restrict__ verts, int64_t len, const int32_t *__restrict__ tt,
                             const int32_t *__restrict__ gslot, const int64_t *__restrict__ goff,
                             const int32_t *__restrict__ gpos, int32_t *__restrict__ members) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = verts[i];
    const int32_t j = tt[x];
    if (j < 0 || j == x) continue;
    members[goff[gslot[j]] + gpos[i]] = x;
  }
}

// one workgroup per group (grid-stride): approve the (weight, ID) prefix that fits the room
__global__ __launch_bounds__(kCoBlock) void k_co_approve(const int32_t *__restrict__ gtarget,
                                                         const int64_t *__restrict__ goff,
                                                         const int32_t *__restrict__ ngroups,
                                                         const int32_t *__restrict__ members,
                                                         const int32_t *__restrict__ vw,
                                                         const int64_t *__restrict__ cw, int64_t wmax,
                                                         int32_t *__restrict__ newlab,
                                                         int64_t *__restrict__ gmoved) {
  __shared__ unsigned long long key[kCoSortCap];
  __shared__ int64_t sm[kCoBlock / kWave + 1];
  const int32_t G = *ngroups;
  for (int32_t g = blockIdx.x; g < G; g += gridDim.x) {
    const int32_t j = gtarget[g];
    const int64_t lo = goff[g], sz = goff[g + 1] - lo;
    const int64_t room = wmax - cw[j];
    int64_t moved = 0;
    if (sz <= kCoSortCap) {
      int32_t np2 = 1;
      while (np2 < sz) np2 <<= 1;
      for (int32_t i = threadIdx.x; i < np2; i += kCoBlock) {
        if (i < sz) {
          const int32_t x = members[lo + i];
          key[i] = ((unsigned long long)cvw(vw, x) << 32) | (uint32_t)x;
        } else {
          key[i] = ~0ull;
        }
      }
      __syncthreads();
      for (int32_t kk = 2; kk <= np2; kk <<= 1) {  // bitonic sort, ascending
        for (int32_t jj = kk >> 1; jj > 0; jj >>= 1) {
          for (int32_t i = threadIdx.x; i < np2; i += kCoBlock) {
            const int32_t p = i ^ jj;
            if (p > i) {
              const unsigned long long a = key[i], b = key[p];
              const bool up = (i & kk) == 0;
              if ((a > b) == up) {
                key[i] = b;
                key[p] = a;
              }
            }
          }
          __syncthreads();
        }
      }
      int64_t carry = 0;
      for (int32_t i0 = 0; i0 < sz; i0 += kCoBlock) {
        const int32_t i = i0 + (int32_t)threadIdx.x;
        const int64_t c = i < sz ? (int64_t)(key[i] >> 32) : 0;
        int64_t tot;
        const int64_t ex = block_excl_scan<kCoBlock, int64_t>(c, sm, &tot);
        if (i < sz && room >= 0 && carry + ex + c <= room) {
          newlab[(int32_t)(key[i] & 0xffffffffull)] = j;
          moved += c;
        }
        carry += tot;
      }
    } else {
      // large group: each member's inclusive prefix weight by a scan of all members
      for (int64_t i = threadIdx.x; i < sz; i += kCoBlock) {
        const int32_t x = members[lo + i];
        const int64_t cx = cvw(vw, x);
        int64_t S = 0;
        for (int64_t y = 0; y < sz; ++y) {
          const int32_t z = members[lo + y];
          const int64_t cz = cvw(vw, z);
          if (cz < cx || (cz == cx && z <= x)) S += cz;
        }
        if (room >= 0 && S <= room) {
          newlab[x] = j;
          moved += cx;
        }
      }
    }
    int64_t tot;
    block_excl_scan<kCoBlock, int64_t>(moved, sm, &tot);
    if (threadIdx.x == 0) gmoved[g] = tot;
    __syncthreads();
  }
}

__global__ void k_co_apply(const int32_t *__restrict__ verts, int64_t len, int32_t *__restrict__ tp,
                           int32_t *__restrict__ tt, const int32_t *__restrict__ vw, int32_t *__restrict__ label,
                           unsigned long long *__restrict__ cw, unsigned long long *__restrict__ jw,
                           int32_t *__restrict__ gcnt, int32_t *__restrict__ gslot, int32_t *__restrict__ newlab,
                           const int32_t *__restrict__ gtarget, const int64_t *__restrict__ gmoved,
                           const int32_t *__restrict__ ngroups) {
  const int32_t G = *ngroups;
  const int64_t span = len > G ? len : G;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < span; i += (int64_t)gridDim.x * blockDim.x) {
    if (i < len) {
      const int32_t x = verts[i];
      const int32_t nl = newlab[x];
      if (nl >= 0) {
        label[x] = nl;
        atomicAdd(&cw[x], (unsigned long long)(-cvw(vw, x)));
        newlab[x] = -1;
      }
      const int32_t j0 = tp[x], j = tt[x];
      if (j0 >= 0) jw[j0] = 0ull;
      if (j >= 0) {
        gcnt[j] = 0;
        gslot[j] = -1;
      }
      tp[x] = -1;
      tt[x] = -1;
    }
    if (i < G) atomicAdd(&cw[gtarget[i]], (unsigned long long)gmoved[i]);
  }
}

constexpr int kCoSmallRound = 1024;  // largest sub-round settled by one workgroup

__global__ __launch_bounds__(kCoSmallRound) void k_co_settle_small(
    const int32_t *__restrict__ verts, int64_t len, int32_t *__restrict__ tp, int32_t *__restrict__ tt,
    const int32_t *__restrict__ vw, int32_t *__restrict__ label, unsigned long long *__restrict__ cw,
    unsigned long long *__restrict__ jw, int32_t *__restrict__ gcnt, int32_t *__restrict__ gslot, int64_t wmax) {
  __shared__ int32_t s_gtarget[kCoSmallRound], s_members[kCoSmallRound];
  __shared__ int64_t s_goff[kCoSmallRound + 1];
  __shared__ unsigned long long s_gmoved[kCoSmallRound];
  __shared__ int64_t sm[kCoSmallRound / kWave + 1];
  __shared__ int32_t s_ng;
  const int i = threadIdx.x;
  const bool act = i < len;
  const int32_t x = act ? verts[i] : -1;
  const int64_t cx = act ? cvw(vw, x) : 0;
  const int32_t j0 = act ? tp[x] : -1;
  if (i == 0) s_ng = 0;
  // proposal weights per target
  if (j0 >= 0) atomicAdd(&jw[j0], (unsigned long long)cx);
  __syncthreads();
  // swap prevention (each thread decides its own vertex)
  int32_t tx = j0;
  if (j0 >= 0 && tp[j0] == x) {
    const int32_t lo = x < j0 ? x : j0, hi = x < j0 ? j0 : x;
    const int64_t jl = (int64_t)__hip_atomic_load(&jw[lo], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t jh = (int64_t)__hip_atomic_load(&jw[hi], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int64_t wl = cvw(vw, lo) + jl - cvw(vw, hi);
    const int64_t wh = cvw(vw, hi) + jh - cvw(vw, lo);
    const int32_t stay = wl >= wh ? lo : hi;
    tx = x == stay ? x : j0;
  }
  // group-by target
  const bool prop = tx >= 0 && tx != x;
  int32_t pos = 0;
  if (prop) {
    pos = atomicAdd(&gcnt[tx], 1);
    if (atomicCAS(&gslot[tx], -1, -2) == -1) {
      const int32_t g = atomicAdd(&s_ng, 1);
      s_gtarget[g] = tx;
      atomicExch(&gslot[tx], g);
    }
  }
  __syncthreads();
  const int32_t G = s_ng;
  {
    const int64_t sz = i < G ? (int64_t)__hip_atomic_load(&gcnt[s_gtarget[i]], __ATOMIC_RELAXED,
                                                          __HIP_MEMORY_SCOPE_AGENT) : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan<kCoSmallRound, int64_t>(sz, sm, &tot);
    if (i < G) {
      s_goff[i] = ex;
      s_gmoved[i] = 0ull;
    }
    if (i == 0) s_goff[G] = tot;
  }
  __syncthreads();
  int32_t g = -1;
  if (prop) {
    g = __hip_atomic_load(&gslot[tx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    s_members[s_goff[g] + pos] = x;
  }
  __syncthreads();
  // approval: the (weight, ID) prefix of the group that fits the room left in the target
  bool ok = false;
  if (prop) {
    int64_t S = 0;
    for (int64_t y = s_goff[g]; y < s_goff[g + 1]; ++y) {
      const int32_t z = s_members[y];
      const int64_t cz = cvw(vw, z);
      if (cz < cx || (cz == cx && z <= x)) S += cz;
    }
    const int64_t room = wmax - (int64_t)cw[tx];
    ok = room >= 0 && S <= room;
    if (ok) atomicAdd(&s_gmoved[g], (unsigned long long)cx);
  }
  __syncthreads();
  // moves, cluster weights, and the per-sub-round state back to -1 / 0
  if (ok) {
    label[x] = tx;
    atomicAdd(&cw[x], (unsigned long long)(-cx));
  }
  if (i < G) atomicAdd(&cw[s_gtarget[i]], s_gmoved[i]);
  if (act) {
    if (j0 >= 0) jw[j0] = 0ull;
    if (tx >= 0) {
      gcnt[tx] = 0;
      gslot[tx] = -1;
    }
    tp[x] = -1;
    tt[x] = -1;
  }
}

__global__ void k_co_count(const int32_t *__restrict__ label, int32_t n, int32_t *__restrict__ flag,
                           int32_t *__restrict__ count) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    if (atomicExch(&flag[label[v]], 1) == 0) atomicAdd(count, 1);
}

unsigned grid_for(int64_t items, int64_t cap) {
  const int64_t g = (items + kCoBlock - 1) / kCoBlock;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(g, cap));
}

}  // namespace

hipError_t launch_co_prepare(Ctx &c) {
  CoState &s = *c.co;
  hipLaunchKernelGGL(k_co_qnet, dim3(grid_for(c.m, 4096)), dim3(kCoBlock), 0, c.stream, c.off, c.nw, c.m, s.qnet);
  hipLaunchKernelGGL(k_co_degree, dim3(grid_for(c.n, 4096)), dim3(kCoBlock), 0, c.stream, c.voff, c.inc, c.off, c.n,
                     s.deg);
  return hipGetLastError();
}

hipError_t launch_co_init(Ctx &c, int32_t *label, int64_t *cw) {
  hipLaunchKernelGGL(k_co_init, dim3(grid_for(c.n, 4096)), dim3(kCoBlock), 0, c.stream, label, cw, c.vw, c.n);
  return hipGetLastError();
}

hipError_t launch_co_check(Ctx &c, const int32_t *list, int64_t len, int32_t *bad) {
  CoState &s = *c.co;
  hipError_t e = hipMemsetAsync(s.flag, 0, sizeof(int32_t) * (size_t)c.n, c.stream);
  if (e != hipSuccess) return e;
  if ((e = hipMemsetAsync(bad, 0, sizeof(int32_t), c.stream)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_co_check, dim3(grid_for(len, 4096)), dim3(kCoBlock), 0, c.stream, list, len, c.n, s.flag, bad);
  return hipGetLastError();
}

hipError_t launch_co_rate(Ctx &c, const int32_t *verts, int64_t a, int64_t b, int64_t base, const int32_t *label,
                          const int64_t *cw, int64_t wmax) {
  CoState &s = *c.co;
  const int64_t per = (kCoBlock / kWave) * (kWave / kCoGroup);  // list positions per small-part workgroup
  const unsigned small_blocks = (unsigned)((b - a + per - 1) / per);
  const unsigned wave_blocks = (unsigned)((b - a + kCoBlock / kWave - 1) / (kCoBlock / kWave));
  hipLaunchKernelGGL(k_co_rate, dim3(small_blocks + wave_blocks), dim3(kCoBlock), 0, c.stream, verts, a, b,
                     small_blocks, s.ptab, base, c.voff, c.inc, c.off, c.pins, s.qnet, c.vw, label, cw, wmax, s.tab,
                     s.tp);
  return hipGetLastError();
}

hipError_t launch_co_settle(Ctx &c, const int32_t *verts, int64_t len, int32_t *label, int64_t *cw, int64_t wmax,
                            int32_t *t_out) {
  CoState &s = *c.co;
  if (len <= kCoSmallRound && !t_out) {
    hipLaunchKernelGGL(k_co_settle_small, dim3(1), dim3(kCoSmallRound), 0, c.stream, verts, len, s.tp, s.tt, c.vw,
                       label, (unsigned long long *)cw, s.jw, s.gcnt, s.gslot, wmax);
    return hipGetLastError();
  }
  const unsigned g = grid_for(len, 2048);
  unsigned long long *jw = (unsigned long long *)s.jw;
  hipLaunchKernelGGL(k_co_join, dim3(g), dim3(kCoBlock), 0, c.stream, verts, len, s.tp, c.vw, jw, s.ngroups);
  hipLaunchKernelGGL(k_co_swap, dim3(g), dim3(kCoBlock), 0, c.stream, verts, len, s.tp, c.vw, jw, s.tt);
  hipLaunchKernelGGL(k_co_group, dim3(g), dim3(kCoBlock), 0, c.stream, verts, len, s.tt, s.gcnt, s.gslot,
                     s.gtarget, s.gpos, s.ngroups);
  hipLaunchKernelGGL(k_co_scan, dim3(1), dim3(1024), 0, c.stream, s.gcnt, s.gtarget, s.ngroups, s.goff);
  hipLaunchKernelGGL(k_co_scatter, dim3(g), dim3(kCoBlock), 0, c.stream, verts, len, s.tt, s.gslot, s.goff, s.gpos,
                     s.members);
  hipLaunchKernelGGL(k_co_approve, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(len, 4096))),
                     dim3(kCoBlock), 0, c.stream, s.gtarget, s.goff, s.ngroups, s.members, c.vw, cw, wmax,
                     s.newlab, s.gmoved);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (t_out && (e = hipMemcpyAsync(t_out, s.tt, sizeof(int32_t) * (size_t)c.n, hipMemcpyDeviceToDevice,
                                   c.stream)) != hipSuccess)
    return e;
  hipLaunchKernelGGL(k_co_apply, dim3(g), dim3(kCoBlock), 0, c.stream, verts, len, s.tp, s.tt, c.vw, label,
                     (unsigned long long *)cw, jw, s.gcnt, s.gslot, s.newlab, s.gtarget, s.gmoved, s.ngroups);
  return hipGetLastError();
}

hipError_t launch_co_count(Ctx &c, const int32_t *label, int32_t *count) {
  CoState &s = *c.co;
  hipError_t e = hipMemsetAsync(s.flag, 0, sizeof(int32_t) * (size_t)c.n, c.stream);
  if (e != hipSuccess) return e;
  if ((e = hipMemsetAsync(count, 0, sizeof(int32_t), c.stream)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_co_count, dim3(grid_for(c.n, 4096)), dim3(kCoBlock), 0, c.stream, label, c.n, s.flag, count);
  return hipGetLastError();
}

}  // namespace jet
