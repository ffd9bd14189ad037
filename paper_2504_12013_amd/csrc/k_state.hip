// Partition state from scratch (start of every call): pin counts phi_e[b] = |e intersect V_b| and
// the connectivity set Lambda(e) (Section 2; tracked per net as in Section 4.2), block weights
// c(V_b), and the (lambda - 1) metric.  All sums are integer and commutative, so the result does
// not depend on scheduling.
#include "chunk.h"
#include "dev_util.h"
#include "jet_internal.h"
#include "phi.h"

namespace jet {

namespace {

__global__ void k_check_part(const int32_t *__restrict__ part, int32_t n, int32_t k, DevStatus *st) {
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t b = part[v];
    if (b < 0 || b >= k)
      if (atomicCAS(&st->err, 0, kErrPartRange) == 0) st->err_arg = (int32_t)v;
  }
}

// small nets: one wave per chunk, one pin per lane
template <typename T>
__global__ __launch_bounds__(256) void k_phi_chunks(const int64_t *__restrict__ off, const int32_t *__restrict__ pins,
                                                    const int4 *__restrict__ chunks, const uint8_t *__restrict__ pnet,
                                                    int32_t nchunks,
                                                    const int32_t *__restrict__ part, int32_t k,
                                                    T *__restrict__ phi) {
  const int w = threadIdx.x / kWave;
  const int32_t c = blockIdx.x * 4 + w;
  const bool has = c < nchunks;
  const int4 cd = has ? chunks[c] : make_int4(0, 0, 0, 0);
  const ChunkLane cl = chunk_lane(cd, pnet, has);
  if (cl.active) phi_atomic_add(phi, (int64_t)cl.net * k + part[pins[cl.q]], 1);
}

// larger nets: one block per net, histogram in LDS, then the block writes the row it owns
template <typename T>
__global__ __launch_bounds__(256) void k_phi_large(const int64_t *__restrict__ off, const int32_t *__restrict__ pins,
                                                   const int32_t *__restrict__ nets, const int32_t *__restrict__ part,
                                                   int32_t k, T *__restrict__ phi) {
  __shared__ int32_t hist[kMaxK];
  const int32_t e = nets[blockIdx.x];
  for (int b = threadIdx.x; b < k; b += blockDim.x) hist[b] = 0;
  __syncthreads();
  for (int64_t q = off[e] + threadIdx.x; q < off[e + 1]; q += blockDim.x) atomicAdd(&hist[part[pins[q]]], 1);
  __syncthreads();
  for (int b = threadIdx.x; b < k; b += blockDim.x) phi[(int64_t)e * k + b] = (T)hist[b];
}

// Connectivity words from pin counts: mask bit b = (phi_e[b] > 0), single bit b = (phi_e[b] == 1).
// Lane i of the flattened (net, padded block) index space reads one count; ballots form the words.
template <int KP, typename T>
__global__ __launch_bounds__(256) void k_build_ns(const T *__restrict__ phi, int32_t m, int32_t k,
                                                  uint64_t *__restrict__ ns) {
  constexpr int NW = KP > 64 ? 2 : 1;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t e = i / KP;
  const int b = (int)(i % KP);
  int32_t val = 0;
  if (e < m && b < k) val = (int32_t)phi[e * k + b];
  const uint64_t nz = ballot(val > 0), one = ballot(val == 1);
  if (e >= m) return;
  if (KP >= 64) {
    if (lane_id() == 0) {
      const int word = b / 64;
      ns[e * 2 * NW + word] = nz;
      ns[e * 2 * NW + NW + word] = one;
    }
  } else if (b == 0) {
    const int sh = lane_id();  // this net's field starts at this lane
    const uint64_t fm = (KP == 64) ? ~0ull : ((1ull << KP) - 1ull);
    ns[e * 2] = (nz >> sh) & fm;
    ns[e * 2 + 1] = (one >> sh) & fm;
  }
}

__global__ __launch_bounds__(256) void k_block_weights(const int32_t *__restrict__ part,
                                                       const int32_t *__restrict__ vw, int32_t n, int32_t k,
                                                       DevStatus *st, Union u) {
  if (u.vhg) {  // union: one atomic per vertex into its hypergraph's segment
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
      const int64_t sg = (int64_t)u.vhg[v] * k + part[v];
      atomicAdd((unsigned long long *)&st->bw[sg], (unsigned long long)(vw ? vw[v] : 1));
      atomicAdd(&st->bcnt[sg], 1);
    }
    return;
  }
  __shared__ unsigned long long sw[kMaxK];
  __shared__ int32_t sc[kMaxK];
  for (int b = threadIdx.x; b < k; b += blockDim.x) {
    sw[b] = 0;
    sc[b] = 0;
  }
  __syncthreads();
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    const int32_t b = part[v];
    atomicAdd(&sw[b], (unsigned long long)(vw ? vw[v] : 1));
    atomicAdd(&sc[b], 1);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < k; b += blockDim.x) {
    if (sw[b]) atomicAdd((unsigned long long *)&st->bw[b], sw[b]);
    if (sc[b]) atomicAdd(&st->bcnt[b], sc[b]);
  }
}

template <int NW>
__global__ __launch_bounds__(256) void k_km1(const uint64_t *__restrict__ ns, const int32_t *__restrict__ nw,
                                             int32_t m, DevStatus *st, Union u) {
  int64_t s = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    int lam = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) lam += __popcll(ns[e * 2 * NW + w]);
    const int64_t d = (int64_t)(lam - 1) * (nw ? nw[e] : 1);
    if (u.nhg) add_km1_hg(st, u.nhg[e], d);  // union: per hypergraph
    else s += d;
  }
  s = wave_sum(s);
  if (lane_id() == 0) add_km1(st, blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave, s);
}

// Level statistics for the learned temperature: over nets, the number and weight of cut nets
// (lambda >= 2), the net weight total and the largest net; over vertices, those with an incident
// cut net.  Integer sums, one atomic per block and counter.
template <int NW>
__global__ __launch_bounds__(256) void k_stats_nets(const int64_t *__restrict__ off, const uint64_t *__restrict__ ns,
                                                    const int32_t *__restrict__ nw, int32_t m,
                                                    int64_t *__restrict__ out) {
  int64_t cut = 0, cutw = 0, sw = 0, mx = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += (int64_t)gridDim.x * blockDim.x) {
    int lam = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) lam += __popcll(ns[e * 2 * NW + w]);
    const int64_t w = nw ? nw[e] : 1;
    sw += w;
    if (lam >= 2) {
      cut += 1;
      cutw += w;
    }
    const int64_t sz = off[e + 1] - off[e];
    mx = sz > mx ? sz : mx;
  }
  cut = wave_sum(cut);
  cutw = wave_sum(cutw);
  sw = wave_sum(sw);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const int64_t y = __shfl_xor(mx, o, kWave);
    mx = y > mx ? y : mx;
  }
  if (lane_id() == 0) {
    if (cut) atomicAdd((unsigned long long *)&out[0], (unsigned long long)cut);
    if (cutw) atomicAdd((unsigned long long *)&out[1], (unsigned long long)cutw);
    if (sw) atomicAdd((unsigned long long *)&out[2], (unsigned long long)sw);
    atomicMax((unsigned long long *)&out[3], (unsigned long long)mx);
  }
}

template <int NW>
__global__ __launch_bounds__(256) void k_stats_boundary(const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
                                                        const uint64_t *__restrict__ ns, int32_t n,
                                                        int64_t *__restrict__ out) {
  int64_t cnt = 0;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    for (int64_t q = voff[v]; q < voff[v + 1]; ++q) {
      const int64_t e = inc[q];
      int lam = 0;
#pragma unroll
      for (int w = 0; w < NW; ++w) lam += __popcll(ns[e * 2 * NW + w]);
      if (lam >= 2) {
        cnt += 1;
        break;
      }
    }
  }
  cnt = wave_sum(cnt);
  if (lane_id() == 0 && cnt) atomicAdd((unsigned long long *)&out[4], (unsigned long long)cnt);
}

inline unsigned grid_for(int64_t work, int block, int64_t cap) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_check_part(Ctx &c, const int32_t *part) {
  hipLaunchKernelGGL(k_check_part, dim3(grid_for(c.n, 256, 16384)), dim3(256), 0, c.stream, part, c.n, c.k, c.st);
  return hipGetLastError();
}

namespace {

template <typename T>
hipError_t build_phi(Ctx &c, const int32_t *part, T *phi) {
  // 16-bit tables (the context's own) are cleared with their padding; an int32 table may be a
  // caller's buffer of exactly m*k counts
  const size_t entries = (size_t)c.m * c.k + (sizeof(T) == 2 ? 1 : 0);
  hipError_t e = hipMemsetAsync(phi, 0, sizeof(T) * entries, c.stream);
  if (e != hipSuccess) return e;
  if (c.nchunks > 0)
    hipLaunchKernelGGL(k_phi_chunks<T>, dim3((unsigned)((c.nchunks + 3) / 4)), dim3(256), 0, c.stream, c.off, c.pins,
                       c.chunks, c.pnet, c.nchunks, part, c.k, phi);
  if (c.nmid > 0)
    hipLaunchKernelGGL(k_phi_large<T>, dim3((unsigned)c.nmid), dim3(256), 0, c.stream, c.off, c.pins, c.mid_nets,
                       part, c.k, phi);
  if (c.nbig > 0)
    hipLaunchKernelGGL(k_phi_large<T>, dim3((unsigned)c.nbig), dim3(256), 0, c.stream, c.off, c.pins, c.big_nets,
                       part, c.k, phi);
  return hipGetLastError();
}

template <typename T>
hipError_t build_ns(Ctx &c, const T *phi) {
  int kp = 1;
  while (kp < c.k) kp <<= 1;
  const int64_t threads = (int64_t)c.m * kp;
  const unsigned g = grid_for(threads, 256, INT32_MAX);
  switch (kp) {
  case 2: hipLaunchKernelGGL((k_build_ns<2, T>), dim3(g), dim3(256), 0, c.stream, phi, c.m, c.k, c.ns); break;
  case 4: hipLaunchKernelGGL((k_build_ns<4, T>), dim3(g), dim3(256), 0, c.stream, phi, c.m, c.k, c.ns); break;
  case 8: hipLaunchKernelGGL((k_build_ns<8, T>), dim3(g), dim3(256), 0, c.stream, phi, c.m, c.k, c.ns); break;
  case 16: hipLaunchKernelGGL((k_build_ns<16, T>), dim3(g), dim3(256), 0, c.stream, phi, c.m, c.k, c.ns); break;
  case 32: hipLaunchKernelGGL((k_build_ns<32, T>), dim3(g), dim3(256), 0, c.stream, phi, c.m, c.k, c.ns); break;
  case 64: hipLaunchKernelGGL((k_build_ns<64, T>), dim3(g), dim3(256), 0, c.stream, phi, c.m, c.k, c.ns); break;
  default: hipLaunchKernelGGL((k_build_ns<128, T>), dim3(g), dim3(256), 0, c.stream, phi, c.m, c.k, c.ns); break;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_build_phi(Ctx &c, const int32_t *part, int32_t *phi) { return build_phi(c, part, phi); }
hipError_t launch_build_phi(Ctx &c, const int32_t *part, uint16_t *phi) { return build_phi(c, part, phi); }

hipError_t launch_build_ns(Ctx &c) { return c.phi16 ? build_ns(c, c.phi16) : build_ns(c, c.phi); }

hipError_t launch_block_weights(Ctx &c, const int32_t *part) {
  const size_t nseg = (c.H > 1 ? (size_t)c.H + 1 : 1) * (size_t)c.k;  // a union's padding has its own segments
  hipError_t e = hipMemsetAsync(c.st->bw, 0, sizeof(int64_t) * nseg, c.stream);
  if (e == hipSuccess) e = hipMemsetAsync(c.st->bcnt, 0, sizeof(int32_t) * nseg, c.stream);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_block_weights, dim3(grid_for(c.n, 256, 2048)), dim3(256), 0, c.stream, part, c.vw, c.n, c.k,
                     c.st, union_of(c));
  return hipGetLastError();
}

hipError_t launch_km1_from_ns(Ctx &c) {
  hipError_t e = hipMemsetAsync(&c.st->km1, 0, sizeof(int64_t) * (1 + kKm1Slots), c.stream);
  if (e == hipSuccess && c.H > 1) e = hipMemsetAsync(c.st->hkm1, 0, sizeof(int64_t) * (size_t)c.H, c.stream);
  if (e != hipSuccess) return e;
  const unsigned g = grid_for(c.m, 256, 4096);
  if (c.nw_words == 1)
    hipLaunchKernelGGL(k_km1<1>, dim3(g), dim3(256), 0, c.stream, c.ns, c.nw, c.m, c.st, union_of(c));
  else
    hipLaunchKernelGGL(k_km1<2>, dim3(g), dim3(256), 0, c.stream, c.ns, c.nw, c.m, c.st, union_of(c));
  return hipGetLastError();
}

hipError_t launch_level_stats(Ctx &c, int64_t *out5) {
  hipError_t e = hipMemsetAsync(out5, 0, 5 * sizeof(int64_t), c.stream);
  if (e != hipSuccess) return e;
  const unsigned gm = grid_for(c.m, 256, 4096), gn = grid_for(c.n, 256, 4096);
  if (c.nw_words == 1) {
    hipLaunchKernelGGL(k_stats_nets<1>, dim3(gm), dim3(256), 0, c.stream, c.off, c.ns, c.nw, c.m, out5);
    hipLaunchKernelGGL(k_stats_boundary<1>, dim3(gn), dim3(256), 0, c.stream, c.voff, c.inc, c.ns, c.n, out5);
  } else {
    hipLaunchKernelGGL(k_stats_nets<2>, dim3(gm), dim3(256), 0, c.stream, c.off, c.ns, c.nw, c.m, out5);
    hipLaunchKernelGGL(k_stats_boundary<2>, dim3(gn), dim3(256), 0, c.stream, c.voff, c.inc, c.ns, c.n, out5);
  }
  return hipGetLastError();
}

}  // namespace jet
