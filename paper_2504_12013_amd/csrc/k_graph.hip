// Graph-specialised kernels: every net has exactly two pins (a graph; the metric is the weighted
// edge cut).  The paper's partitioner refines graphs with an implementation specialised to them
// (data structures and algorithms for edges instead of general nets); here the specialisation is
// the afterburner.
//
// For a net e = {v, u} Algorithm 2 replays the candidates of e in (gain desc, ID asc) order: when
// candidate v moves from s to t, u sits in its target block t_u if u is a candidate ordered before
// v, else in its current block; the net's contribution to v's recomputed gain is
// w(e) ([t = eff(u)] - [s = eff(u)]).  So every candidate sums over its neighbours alone: no sort,
// no per-net state and no atomics, one gather of the neighbour's block (and record, when the
// neighbour is a candidate) per incidence.  The neighbour of every incidence is stored at init
// (adj[q] = the other pin of net inc[q]), next to the incidence lists.
#include <hip/hip_runtime.h>

#include "dev_util.h"
#include "jet_internal.h"

namespace jet {
namespace {

constexpr int kGraphBlock = 256;

__global__ void k_build_adj(const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
                            const int64_t *__restrict__ off, const int32_t *__restrict__ pins, int32_t n,
                            int32_t *__restrict__ adj) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    for (int64_t q = voff[v]; q < voff[v + 1]; ++q) {
      const int64_t a = off[inc[q]];
      adj[q] = pins[a] == (int32_t)v ? pins[a + 1] : pins[a];
    }
}

// G lanes per vertex (G = 1 on light graphs, 8 otherwise), each taking every G-th neighbour.
template <int G>
__global__ __launch_bounds__(kGraphBlock) void k_ab_graph(const int32_t *__restrict__ part,
                                                          const int64_t *__restrict__ voff,
                                                          const int32_t *__restrict__ adj,
                                                          const int32_t *__restrict__ inc,
                                                          const int32_t *__restrict__ nw,
                                                          const uint32_t *__restrict__ inm,
                                                          const uint64_t *__restrict__ rec, int32_t n,
                                                          int32_t *__restrict__ rg, DevStatus *st,
                                                          const LoopCtl *lc, int32_t want) {
  JET_GATE(lc, want);
  constexpr int VPB = kGraphBlock / G;
  __shared__ unsigned long long wsum[kGraphBlock / kWave];
  const int lg = threadIdx.x % G;
  unsigned long long scanned = 0ull;
  for (int64_t base = (int64_t)blockIdx.x * VPB; base < n; base += (int64_t)gridDim.x * VPB) {
    const int64_t v = base + threadIdx.x / G;
    bool cand = false;
    int32_t gv = 0, tv = 0, sv = 0;
    int64_t q0 = 0, q1 = 0;
    if (v < n) {
      cand = (inm[v >> 5] >> (v & 31)) & 1u;
      if (cand) {
        const uint64_t r = rec[v];
        gv = (int32_t)(uint32_t)r;
        tv = (int32_t)((r >> 32) & 0xffu);
        sv = (int32_t)((r >> 40) & 0xffu);
        q0 = voff[v];
        q1 = voff[v + 1];
      }
    }
    int32_t acc = 0;
    for (int64_t q = q0 + lg; q < q1; q += G) {
      const int32_t u = adj[q];
      int32_t eff = part[u];
      if ((inm[u >> 5] >> (u & 31)) & 1u) {  // a candidate: moved first iff it precedes v
        const uint64_t r = rec[u];
        const int32_t gu = (int32_t)(uint32_t)r;
        if (gu > gv || (gu == gv && u < (int32_t)v)) eff = (int32_t)((r >> 32) & 0xffu);
      }
      const int32_t w = nw ? nw[inc[q]] : 1;
      acc += (eff == tv ? w : 0) - (eff == sv ? w : 0);
    }
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, kWave);
    if (v < n && lg == 0) {
      rg[v] = cand ? acc : 0;
      if (cand) scanned += (unsigned long long)(q1 - q0);
    }
  }
  scanned = wave_sum(scanned);
  if (lane_id() == 0) wsum[threadIdx.x / kWave] = scanned;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0ull;
    for (int i = 0; i < kGraphBlock / kWave; ++i) t += wsum[i];
    if (t) atomicAdd((unsigned long long *)&st->ab_inc, t);
  }
}

}  // namespace

hipError_t launch_build_adj(Ctx &c) {
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(4096, ((int64_t)c.n + 255) / 256));
  hipLaunchKernelGGL(k_build_adj, dim3(grid), dim3(256), 0, c.stream, c.voff, c.inc, c.off, c.pins, c.n, c.adj);
  return hipGetLastError();
}

bool graph_afterburner(const Ctx &c) { return c.adj != nullptr && c.H == 1 && c.graph_kernels; }

hipError_t launch_ab_graph(Ctx &c, const int32_t *part, const LoopCtl *lc, int32_t want) {
  // one lane per vertex while the mean degree is below lane_degree, eight otherwise
  if (c.p < (int64_t)c.lane_degree * c.n) {
    const unsigned grid = (unsigned)std::min<int64_t>(c.grid_cap, ((int64_t)c.n + kGraphBlock - 1) / kGraphBlock);
    hipLaunchKernelGGL(k_ab_graph<1>, dim3(grid), dim3(kGraphBlock), 0, c.stream, part, c.voff, c.adj, c.inc, c.nw,
                       c.inm, c.rec, c.n, c.rg, c.st, lc, want);
  } else {
    const unsigned grid =
        (unsigned)std::min<int64_t>(c.grid_cap, ((int64_t)c.n + kGraphBlock / 8 - 1) / (kGraphBlock / 8));
    hipLaunchKernelGGL(k_ab_graph<8>, dim3(grid), dim3(kGraphBlock), 0, c.stream, part, c.voff, c.adj, c.inc, c.nw,
                       c.inm, c.rec, c.n, c.rg, c.st, lc, want);
  }
  return hipGetLastError();
}

}  // namespace jet
