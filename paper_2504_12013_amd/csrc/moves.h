// Move-list helpers shared by the kernels that list moves (iteration and rebalancing).
#pragma once
#include "dev_util.h"
#include "jet_internal.h"

namespace jet {

// Records position `pos` of the move list in the high-degree list for the lanes with `big` set
// (one slot reservation per wave).  Must be called with every lane of the wave active.  The list
// order is irrelevant: applying the moves is order independent.
__device__ __forceinline__ void push_big_move(bool big, int32_t pos, DevStatus *st, int32_t *bigmv) {
  const uint64_t mm = ballot(big);
  if (!mm) return;
  int32_t base = 0;
  if (lane_id() == 0) base = atomicAdd(&st->n_bigmv, __popcll(mm));
  base = __shfl(base, 0, kWave);
  if (big) bigmv[base + rank_below(mm)] = pos;
}

}  // namespace jet
