// Per-vertex candidate records shared by the iteration kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jet {

// candidate bitmask test
__device__ __forceinline__ bool inm_bit(const uint32_t *__restrict__ inm, int32_t v) {
  return (inm[v >> 5] >> (v & 31)) & 1u;
}

// record: gain (bits 0-31), target block (32-39, 0xff = none), source block (40-47)
__device__ __forceinline__ uint64_t pack_rec(int32_t g, int32_t t, int32_t s) {
  return (uint64_t)(uint32_t)g | ((uint64_t)(uint32_t)(t & 0xff) << 32) | ((uint64_t)(uint32_t)(s & 0xff) << 40);
}
__device__ __forceinline__ int32_t rec_gain(uint64_t r) { return (int32_t)(uint32_t)r; }
__device__ __forceinline__ int32_t rec_target(uint64_t r) { return (int32_t)((r >> 32) & 0xff); }
__device__ __forceinline__ int32_t rec_source(uint64_t r) { return (int32_t)((r >> 40) & 0xff); }

// Execution order of the candidates (highest gain first, then lowest vertex ID) as an ascending
// 64-bit key: high word INT32_MAX - gain, low word the vertex ID.
__device__ __forceinline__ uint32_t order_hi(int32_t g) { return (uint32_t)((int64_t)INT32_MAX - (int64_t)g); }
__device__ __forceinline__ unsigned long long order_key(int32_t g, int32_t v) {
  return ((unsigned long long)order_hi(g) << 32) | (uint32_t)v;
}

}  // namespace jet
