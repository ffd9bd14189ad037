// Wave-per-chunk mapping for small nets.  A chunk is a run of consecutive nets with at most 64
// pins in total; one wave holds all of them, one pin per lane, so per-net work needs no atomics
// between waves and no segment search.
#pragma once
#include "dev_util.h"

namespace jet {

struct ChunkLane {
  int32_t net;      // net ID of this lane's pin (valid only if active)
  int64_t q;        // pin index
  bool active;      // lane holds a pin
  uint64_t starts;  // lanes that hold the first pin of a net (wave-uniform)
};

// Must be called by all 64 lanes of the wave (wave-level only: no LDS, no block barrier);
// has_chunk must be wave-uniform.  Lane x < cd.y reads the offset of net cd.x + x; the OR over the
// wave of one bit per offset marks the lanes where nets start.
__device__ __forceinline__ ChunkLane chunk_lane(const int64_t *__restrict__ off, int2 cd, bool has_chunk) {
  const int l = lane_id();
  ChunkLane r;
  r.active = false;
  r.net = 0;
  r.q = 0;
  int64_t base = 0;
  int32_t npins = 0;
  uint64_t bit = 0;
  if (has_chunk) {
    base = off[cd.x];
    npins = (int32_t)(off[cd.x + cd.y] - base);
    if (l < cd.y) bit = 1ull << (int)(off[cd.x + l] - base);
  }
  uint32_t lo = (uint32_t)bit, hi = (uint32_t)(bit >> 32);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    lo |= (uint32_t)__shfl_xor((int)lo, o, kWave);
    hi |= (uint32_t)__shfl_xor((int)hi, o, kWave);
  }
  r.starts = ((uint64_t)hi << 32) | lo;
  if (has_chunk && l < npins) {
    const uint64_t upto = (l == 63) ? ~0ull : ((2ull << l) - 1ull);
    r.net = cd.x + __popcll(r.starts & upto) - 1;
    r.q = base + l;
    r.active = true;
  }
  return r;
}

// Orders this wave's LDS accesses before the following ones (for LDS private to the wave).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

}  // namespace jet
