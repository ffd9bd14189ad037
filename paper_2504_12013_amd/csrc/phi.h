// Pin counts phi_e[b] (Section 2), net-major, one row of k counts per net.  They are stored as
// int32, or as uint16 when no net has more than 65,535 pins: a count never exceeds its net's size,
// also while the moves of one application are half done (a pin adds to its target only once and
// subtracts from its source only once), so 16 bits suffice and a row of k = 64 counts fits one
// 128-byte line.  16-bit counts change through 32-bit atomics on the aligned word that holds
// them: a count is decremented only while positive and incremented only below 65,536, so no
// borrow or carry reaches the neighbouring count.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace jet {

// Adds d (+1 or -1) to count i and returns the count before the addition.
__device__ __forceinline__ int32_t phi_atomic_add(int32_t *phi, int64_t i, int32_t d) {
  return atomicAdd(phi + i, d);
}
__device__ __forceinline__ int32_t phi_atomic_add(uint16_t *phi, int64_t i, int32_t d) {
  uint32_t *word = reinterpret_cast<uint32_t *>(phi + (i & ~(int64_t)1));
  const int sh = (int)(i & 1) * 16;
  const uint32_t old = atomicAdd(word, (uint32_t)d << sh);
  return (int32_t)((old >> sh) & 0xffffu);
}

// Entries allocated for m*k counts (16-bit tables are padded to whole 32-bit words).
inline size_t phi_entries(int64_t m, int32_t k) { return (size_t)m * k + 1; }

}  // namespace jet
