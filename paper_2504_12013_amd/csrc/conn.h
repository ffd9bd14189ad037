// Per-vertex block connectivity, shared by the candidate and rebalancing kernels.
//
// G lanes cooperate on one vertex v; lane j of the group owns blocks 8j .. 8j+7 and accumulates
//     conn[b] = sum of w(e) over incident nets e that have a pin in block b
// from the nets' connectivity words; the lane owning v's block s also accumulates
//     benefit  = sum of w(e) over incident nets where v is the only pin in s.
// With aff = w(I(v)) - benefit (incident nets with at least two pins in s):
//     gain(v, b) = conn[b] - aff        for b != s
// (Section 2 metric; a net gains b when it had no pin there, loses s when v was its last pin there).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jet {

template <int G, bool UNIT>
__device__ __forceinline__ void conn_accumulate(const int32_t *__restrict__ inc, int64_t q0, int64_t q1, int64_t step,
                                                const int32_t *__restrict__ nw, const uint64_t *__restrict__ ns,
                                                int lg, int32_t s, int32_t conn[8], int32_t &benefit) {
  constexpr int NW = (G == 16) ? 2 : 1;
  const int word = lg >> 3;
  const int shift = (lg & 7) * 8;
  const int sbit = s & 63;
  const bool owner = (s >> 3) == lg;
  auto add = [&](uint64_t mw, uint64_t ow, int32_t w) {
    const uint32_t byte = (uint32_t)(mw >> shift) & 0xffu;
#pragma unroll
    for (int j = 0; j < 8; ++j) conn[j] += ((byte >> j) & 1u) ? w : 0;
    if (owner && ((ow >> sbit) & 1ull)) benefit += w;
  };
  int64_t q = q0;
  // four incident nets per step: the index loads, then the word loads, are independent
  for (; q + 3 * step < q1; q += 4 * step) {
    const int32_t e0 = inc[q], e1 = inc[q + step], e2 = inc[q + 2 * step], e3 = inc[q + 3 * step];
    const uint64_t *n0 = ns + (int64_t)e0 * (2 * NW), *n1 = ns + (int64_t)e1 * (2 * NW);
    const uint64_t *n2 = ns + (int64_t)e2 * (2 * NW), *n3 = ns + (int64_t)e3 * (2 * NW);
    const uint64_t m0 = n0[word], m1 = n1[word], m2 = n2[word], m3 = n3[word];
    const uint64_t o0 = n0[NW + word], o1 = n1[NW + word], o2 = n2[NW + word], o3 = n3[NW + word];
    const int32_t w0 = UNIT ? 1 : nw[e0], w1 = UNIT ? 1 : nw[e1], w2 = UNIT ? 1 : nw[e2], w3 = UNIT ? 1 : nw[e3];
    add(m0, o0, w0);
    add(m1, o1, w1);
    add(m2, o2, w2);
    add(m3, o3, w3);
  }
  for (; q < q1; q += step) {
    const int32_t e = inc[q];
    const uint64_t *nse = ns + (int64_t)e * (2 * NW);
    add(nse[word], nse[NW + word], UNIT ? 1 : nw[e]);
  }
}

}  // namespace jet
