// Device helpers for gfx950 (wave64): reductions, scans and ballots used by the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jet {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// number of set bits of mask strictly below this lane
__device__ __forceinline__ int rank_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x += __shfl_xor(x, o, kWave);
  return x;
}

// inclusive prefix sum over the wave
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T x) {
  const int l = lane_id();
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    T y = __shfl_up(x, o, kWave);
    if (l >= o) x += y;
  }
  return x;
}

// Exclusive prefix sum over a block of BLOCK threads; returns the block total in *total.
// Uses `smem` of at least BLOCK/64 + 1 elements.  Must be called by every thread of the block.
template <int BLOCK, typename T>
__device__ __forceinline__ T block_excl_scan(T x, T *smem, T *total) {
  constexpr int NW = BLOCK / kWave;
  const int w = threadIdx.x / kWave, l = lane_id();
  T inc = wave_incl_scan(x);
  if (l == kWave - 1) smem[w] = inc;
  __syncthreads();
  if (threadIdx.x == 0) {
    T run = 0;
    for (int i = 0; i < NW; ++i) {
      T s = smem[i];
      smem[i] = run;
      run += s;
    }
    smem[NW] = run;
  }
  __syncthreads();
  T res = inc - x + smem[w];
  *total = smem[NW];
  __syncthreads();
  return res;
}

// read a 32-bit value held by lane `src` (wave-uniform src) into every lane
__device__ __forceinline__ int32_t read_lane_i32(int32_t v, int src) {
  return __builtin_amdgcn_readlane(v, src);
}
__device__ __forceinline__ uint32_t read_lane_u32(uint32_t v, int src) {
  return (uint32_t)__builtin_amdgcn_readlane((int)v, src);
}

}  // namespace jet
