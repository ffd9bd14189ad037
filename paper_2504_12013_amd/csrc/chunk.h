// Wave-per-chunk mapping for small nets.  A chunk is a run of consecutive nets with at most 64
// pins in total; one wave holds all of them, one pin per lane, so per-net work needs no atomics
// between waves and no segment search.
#pragma once
#include "dev_util.h"

namespace jet {

struct ChunkLane {
  int32_t net;    // net ID of this lane's pin (valid only if active)
  int64_t q;      // pin index
  bool active;    // lane holds a pin
};

// Called by all 64 lanes of every wave of the block (it contains block barriers).  `mark` points
// to 64 ints of LDS private to this wave.  has_chunk must be wave-uniform.
__device__ __forceinline__ ChunkLane chunk_lane(const int64_t *__restrict__ off, int2 cd, bool has_chunk,
                                                int32_t *mark) {
  const int l = lane_id();
  ChunkLane r;
  r.active = false;
  r.net = 0;
  r.q = 0;
  int64_t base = 0;
  int32_t npins = 0;
  if (has_chunk) {
    base = off[cd.x];
    npins = (int32_t)(off[cd.x + cd.y] - base);
  }
  mark[l] = 0;
  __syncthreads();
  if (has_chunk && l < cd.y) mark[(int)(off[cd.x + l] - base)] = 1;
  __syncthreads();
  const uint64_t starts = ballot(mark[l] != 0);
  if (has_chunk && l < npins) {
    const uint64_t upto = (l == 63) ? ~0ull : ((2ull << l) - 1ull);
    r.net = cd.x + __popcll(starts & upto) - 1;
    r.q = base + l;
    r.active = true;
  }
  return r;
}

}  // namespace jet
