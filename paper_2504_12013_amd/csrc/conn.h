// Per-vertex block connectivity, shared by the candidate and rebalancing kernels.
//
// G lanes cooperate on one vertex v; lane j of the group owns blocks 8j .. 8j+7 and accumulates
//     conn[b] = sum of w(e) over incident nets e that have a pin in block b
// from the nets' connectivity words; every lane also accumulates
//     benefit  = sum of w(e) over incident nets where v is the only pin in s.
// With aff = w(I(v)) - benefit (incident nets with at least two pins in s):
//     gain(v, b) = conn[b] - aff        for b != s
// (Section 2 metric; a net gains b when it had no pin there, loses s when v was its last pin there).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jet {

// Group-parallel form: lane lg of the group loads incident net (base + lg) of each batch of G
// consecutive incidences, so the group keeps G independent load chains in flight; the batch is
// then exchanged inside the group with cross-lane shuffles (each lane takes the 32-bit half of
// the mask word holding its byte).  Batches start at q0, q0 + stride, ... below q1.  The
// arguments are equal for the G lanes of a group, so the shuffles only ever read lanes of the
// same group that run the same iteration.
template <int G, bool UNIT>
__device__ __forceinline__ void conn_accumulate(const int32_t *__restrict__ inc, int64_t q0, int64_t q1,
                                                int64_t stride, const int32_t *__restrict__ nw,
                                                const uint64_t *__restrict__ ns, int lg, int32_t s,
                                                int32_t conn[8], int32_t &benefit) {
  constexpr int NW = (G == 16) ? 2 : 1;
  constexpr int U = 4;               // batches whose loads are issued before any is consumed
  const int word = lg >> 3;          // mask word holding this lane's blocks
  const int half = (lg & 7) >> 2;    // 32-bit half of that word
  const int shift = (lg & 3) * 8;    // byte inside the half
  const int sw = s >> 6;
  const uint64_t sbit = 1ull << (s & 63);
  for (int64_t b0 = q0; b0 < q1; b0 += U * stride) {
    int32_t e[U], w[U], own[U];
    uint32_t lo[U][NW], hi[U][NW];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t q = b0 + u * stride + lg;
      e[u] = q < q1 ? inc[q] : -1;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      w[u] = 0;
      own[u] = 0;
#pragma unroll
      for (int x = 0; x < NW; ++x) {
        lo[u][x] = 0u;
        hi[u][x] = 0u;
      }
      if (e[u] >= 0) {
        w[u] = UNIT ? 1 : nw[e[u]];
        const uint64_t *nse = ns + (int64_t)e[u] * (2 * NW);
#pragma unroll
        for (int x = 0; x < NW; ++x) {
          const uint64_t m = nse[x];
          lo[u][x] = (uint32_t)m;
          hi[u][x] = (uint32_t)(m >> 32);
        }
        own[u] = (nse[NW + sw] & sbit) ? w[u] : 0;  // v is this net's only pin in s
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (b0 + u * stride >= q1) break;  // uniform over the group
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const int32_t wj = __shfl(w[u], j, G);
        const int32_t oj = __shfl(own[u], j, G);
        uint32_t mine = 0u;
#pragma unroll
        for (int x = 0; x < NW; ++x) {
          const uint32_t l32 = (uint32_t)__shfl((int)lo[u][x], j, G);
          const uint32_t h32 = (uint32_t)__shfl((int)hi[u][x], j, G);
          if (x == word) mine = half ? h32 : l32;
        }
        const uint32_t byte = (mine >> shift) & 0xffu;
#pragma unroll
        for (int b = 0; b < 8; ++b) conn[b] += ((byte >> b) & 1u) ? wj : 0;
        benefit += oj;
      }
    }
  }
}

// Sequential form for one lane per vertex (G = 1): four incident nets per step.
template <bool UNIT>
__device__ __forceinline__ void conn_accumulate_lane(const int32_t *__restrict__ inc, int64_t q0, int64_t q1,
                                                     const int32_t *__restrict__ nw,
                                                     const uint64_t *__restrict__ ns, int32_t s, int32_t conn[8],
                                                     int32_t &benefit) {
  const uint64_t sbit = 1ull << (s & 63);
  auto add = [&](uint64_t mw, uint64_t ow, int32_t w) {
    const uint32_t byte = (uint32_t)mw & 0xffu;
#pragma unroll
    for (int j = 0; j < 8; ++j) conn[j] += ((byte >> j) & 1u) ? w : 0;
    if (ow & sbit) benefit += w;
  };
  int64_t q = q0;
  for (; q + 3 < q1; q += 4) {
    const int32_t e0 = inc[q], e1 = inc[q + 1], e2 = inc[q + 2], e3 = inc[q + 3];
    const uint64_t *n0 = ns + (int64_t)e0 * 2, *n1 = ns + (int64_t)e1 * 2;
    const uint64_t *n2 = ns + (int64_t)e2 * 2, *n3 = ns + (int64_t)e3 * 2;
    const uint64_t m0 = n0[0], m1 = n1[0], m2 = n2[0], m3 = n3[0];
    const uint64_t o0 = n0[1], o1 = n1[1], o2 = n2[1], o3 = n3[1];
    const int32_t w0 = UNIT ? 1 : nw[e0], w1 = UNIT ? 1 : nw[e1], w2 = UNIT ? 1 : nw[e2], w3 = UNIT ? 1 : nw[e3];
    add(m0, o0, w0);
    add(m1, o1, w1);
    add(m2, o2, w2);
    add(m3, o3, w3);
  }
  for (; q < q1; ++q) {
    const int32_t e = inc[q];
    add(ns[(int64_t)e * 2], ns[(int64_t)e * 2 + 1], UNIT ? 1 : nw[e]);
  }
}

// Strided form: each lane of the group walks q0, q0 + step, ... itself (all lanes of the group load
// the same incident net); four nets per step.  Used by the workgroup-per-vertex kernels with G = 1.
template <int G, bool UNIT>
__device__ __forceinline__ void conn_accumulate_strided(const int32_t *__restrict__ inc, int64_t q0, int64_t q1,
                                                        int64_t step, const int32_t *__restrict__ nw,
                                                        const uint64_t *__restrict__ ns, int lg, int32_t s,
                                                        int32_t conn[8], int32_t &benefit) {
  constexpr int NW = (G == 16) ? 2 : 1;
  const int word = lg >> 3;
  const int shift = (lg & 7) * 8;
  const int sw = s >> 6;
  const uint64_t sbit = 1ull << (s & 63);
  auto add = [&](uint64_t mw, uint64_t ow, int32_t w) {
    const uint32_t byte = (uint32_t)(mw >> shift) & 0xffu;
#pragma unroll
    for (int j = 0; j < 8; ++j) conn[j] += ((byte >> j) & 1u) ? w : 0;
    if (ow & sbit) benefit += w;
  };
  int64_t q = q0;
  for (; q + 3 * step < q1; q += 4 * step) {
    const int32_t e0 = inc[q], e1 = inc[q + step], e2 = inc[q + 2 * step], e3 = inc[q + 3 * step];
    const uint64_t *n0 = ns + (int64_t)e0 * (2 * NW), *n1 = ns + (int64_t)e1 * (2 * NW);
    const uint64_t *n2 = ns + (int64_t)e2 * (2 * NW), *n3 = ns + (int64_t)e3 * (2 * NW);
    const uint64_t m0 = n0[word], m1 = n1[word], m2 = n2[word], m3 = n3[word];
    const uint64_t o0 = n0[NW + sw], o1 = n1[NW + sw], o2 = n2[NW + sw], o3 = n3[NW + sw];
    const int32_t w0 = UNIT ? 1 : nw[e0], w1 = UNIT ? 1 : nw[e1], w2 = UNIT ? 1 : nw[e2], w3 = UNIT ? 1 : nw[e3];
    add(m0, o0, w0);
    add(m1, o1, w1);
    add(m2, o2, w2);
    add(m3, o3, w3);
  }
  for (; q < q1; q += step) {
    const int32_t e = inc[q];
    const uint64_t *nse = ns + (int64_t)e * (2 * NW);
    add(nse[word], nse[NW + sw], UNIT ? 1 : nw[e]);
  }
}

// Dispatch: conn[] and benefit of v over the incidences [q0, q1) walked in batches (see above).
template <int G, bool UNIT>
__device__ __forceinline__ void vertex_conn(const int32_t *__restrict__ inc, int64_t q0, int64_t q1, int64_t stride,
                                            const int32_t *__restrict__ nw, const uint64_t *__restrict__ ns, int lg,
                                            int32_t s, int32_t conn[8], int32_t &benefit) {
  if (G == 1) conn_accumulate_lane<UNIT>(inc, q0, q1, nw, ns, s, conn, benefit);
  else conn_accumulate<G, UNIT>(inc, q0, q1, stride, nw, ns, lg, s, conn, benefit);
}

// ---- bit-sliced counts (unit net weights, k <= 64) ----
// conn(v, b) for all 64 blocks is kept in nine 64-bit planes: plane p holds bit p of every
// block's count (a non-hub vertex has at most 256 incident nets, so nine bits suffice).  Adding a
// net's mask is a carry-save step over the planes.

__device__ __forceinline__ void plane_add(uint64_t pl[9], uint64_t c) {
#pragma unroll
  for (int p = 0; p < 9; ++p) {
    const uint64_t t = pl[p] & c;
    pl[p] ^= c;
    c = t;
  }
}

// Lane lg of a group of G lanes takes incidences q0 + lg, q0 + lg + G, ... (four in flight) and
// accumulates their masks into pl; benefit counts the nets where s is marked as holding one pin.
template <int G>
__device__ __forceinline__ void planes_accumulate(const int32_t *__restrict__ inc, int64_t q0, int64_t q1,
                                                  const uint64_t *__restrict__ ns, int lg, uint64_t sbit,
                                                  uint64_t pl[9], int32_t &benefit) {
  int64_t q = q0 + lg;
  for (; q + 3 * G < q1; q += 4 * G) {
    const int32_t e0 = inc[q], e1 = inc[q + G], e2 = inc[q + 2 * G], e3 = inc[q + 3 * G];
    const uint64_t m0 = ns[(int64_t)e0 * 2], m1 = ns[(int64_t)e1 * 2], m2 = ns[(int64_t)e2 * 2],
                   m3 = ns[(int64_t)e3 * 2];
    const uint64_t o0 = ns[(int64_t)e0 * 2 + 1], o1 = ns[(int64_t)e1 * 2 + 1], o2 = ns[(int64_t)e2 * 2 + 1],
                   o3 = ns[(int64_t)e3 * 2 + 1];
    plane_add(pl, m0);
    plane_add(pl, m1);
    plane_add(pl, m2);
    plane_add(pl, m3);
    benefit += ((o0 & sbit) != 0) + ((o1 & sbit) != 0) + ((o2 & sbit) != 0) + ((o3 & sbit) != 0);
  }
  for (; q < q1; q += G) {
    const int32_t e = inc[q];
    plane_add(pl, ns[(int64_t)e * 2]);
    benefit += (ns[(int64_t)e * 2 + 1] & sbit) != 0;
  }
}

// Sums the planes and benefits of the G lanes of each group (butterfly over the group, ripple
// adds of the bit-sliced numbers); every lane of the wave calls it.
template <int G>
__device__ __forceinline__ void planes_combine(uint64_t pl[9], int32_t &benefit) {
#pragma unroll
  for (int o = 1; o < G; o <<= 1) {
    uint64_t carry = 0ull;
#pragma unroll
    for (int p = 0; p < 9; ++p) {
      const uint64_t x = pl[p], y = __shfl_xor(pl[p], o, G);
      pl[p] = x ^ y ^ carry;
      carry = (x & y) | (carry & (x ^ y));
    }
    benefit += __shfl_xor(benefit, o, G);
  }
}

// Lowest block of largest count among the blocks of mask (counts of zero included): the mask is
// narrowed from the top plane down.  Returns the count, or -1 when mask is empty.
__device__ __forceinline__ int32_t planes_best(const uint64_t pl[9], uint64_t mask, int32_t &block) {
  block = 0;
  if (!mask) return -1;
#pragma unroll
  for (int p = 8; p >= 0; --p) {
    const uint64_t x = mask & pl[p];
    if (x) mask = x;
  }
  block = __ffsll((unsigned long long)mask) - 1;
  int32_t c = 0;
#pragma unroll
  for (int p = 0; p < 9; ++p) c |= (int32_t)((pl[p] >> block) & 1ull) << p;
  return c;
}

}  // namespace jet
