// Wave-per-chunk mapping for small nets.  A chunk is a run of consecutive nets with at most 64
// pins in total; one wave holds all of them, one pin per lane, so per-net work needs no atomics
// between waves and no segment search.  Chunk descriptors (first net, number of nets, number of
// pins, first pin) and every pin's net index inside its chunk are built once at set-up, so a lane
// finds its pin and net with one load each.
#pragma once
#include "dev_util.h"

namespace jet {

struct ChunkLane {
  int32_t net;      // net ID of this lane's pin (valid only if active)
  int64_t q;        // pin index
  bool active;      // lane holds a pin
  uint64_t starts;  // lanes that hold the first pin of a net (wave-uniform)
};

// Must be called by all 64 lanes of the wave (wave-level only); has_chunk must be wave-uniform.
__device__ __forceinline__ ChunkLane chunk_lane(int4 cd, const uint8_t *__restrict__ pnet, bool has_chunk) {
  const int l = lane_id();
  ChunkLane r;
  r.active = has_chunk && l < cd.z;
  r.net = 0;
  r.q = 0;
  int32_t j = -1;
  if (r.active) {
    r.q = (int64_t)cd.w + l;
    j = pnet[r.q];
    r.net = cd.x + j;
  }
  const int32_t jprev = __shfl_up(j, 1, kWave);
  r.starts = ballot(r.active && (l == 0 || jprev != j));
  return r;
}

// Orders this wave's LDS accesses before the following ones (for LDS private to the wave).
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

}  // namespace jet
