// Allocation-free evaluation of the connectivity metric (Section 2): km1(part) = sum over nets of
// omega(e) * (lambda(e) - 1), lambda(e) the number of blocks holding a pin of e.  The same value as
// jet_km1, computed without a context: one wave per net ORs the blocks of the net's pins into a
// 128-bit mask held in registers, each workgroup writes the sum of its nets into one slot of a
// library-owned static device array, and one workgroup adds the slots in index order.  Nothing is
// allocated, nothing is synchronised: the call only enqueues two kernels on the caller's stream.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "dev_util.h"
#include "jet_internal.h"

namespace jet {

namespace {

constexpr int kStaticThreads = 256;                  // four waves per workgroup
constexpr int kStaticNetsPerWave = 16;
constexpr int kStaticNetsPerGroup = 4 * kStaticNetsPerWave;
constexpr int kStaticSlots = 65536;                  // one partial sum per workgroup
constexpr int64_t kStaticMaxNets = (int64_t)kStaticSlots * kStaticNetsPerGroup;  // 4,194,304
constexpr int kSumThreads = 1024;
// a slot written by a workgroup that met an invalid input (offsets out of order or beyond
// num_pins, a pin outside [0,n), a block outside [0,k)); the metric itself is never negative
constexpr long long kBadSlot = LLONG_MIN;

}  // namespace

}  // namespace jet

// Per-workgroup partial sums of the metric.  Every GPU holds its own copy until the process ends;
// host code reaches it only through the address hipGetSymbolAddress returns for the device.
static __device__ __align__(256) long long scratch[jet::kStaticSlots];

namespace jet {

namespace {

__device__ __forceinline__ uint64_t wave_or_u64(uint64_t x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, o, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), o, kWave);
    x |= ((uint64_t)hi << 32) | lo;
  }
  return x;
}

// Every read is guarded by the stated sizes (m + 1 offsets, num_pins pins, n part entries), so
// malformed inputs are reported through the slot, never read past.
__global__ __launch_bounds__(kStaticThreads) void k_static_km1(const int64_t *__restrict__ off,
                                                                const int32_t *__restrict__ pins,
                                                                const int32_t *__restrict__ nw,
                                                                const int32_t *__restrict__ part, int32_t n,
                                                                int32_t m, int64_t num_pins, int32_t k,
                                                                long long *__restrict__ slots) {
  __shared__ long long wsum[kStaticThreads / kWave];
  __shared__ int wbad[kStaticThreads / kWave];
  const int w = threadIdx.x / kWave, l = lane_id();
  long long acc = 0;
  bool bad = false;
  const int64_t e0 = (int64_t)blockIdx.x * kStaticNetsPerGroup + (int64_t)w * kStaticNetsPerWave;
  for (int j = 0; j < kStaticNetsPerWave; ++j) {
    const int64_t e = e0 + j;
    if (e >= m) break;  // wave-uniform
    int64_t q0 = off[e], q1 = off[e + 1];
    if (q0 < 0 || q1 < q0 || q1 > num_pins) {
      bad = true;
      q1 = q0;  // nothing of this net is read
    }
    uint64_t lo = 0ull, hi = 0ull;
    for (int64_t q = q0 + l; q < q1; q += kWave) {
      const int32_t v = pins[q];
      if (v < 0 || v >= n) {
        bad = true;
        continue;
      }
      const int32_t b = part[v];
      if (b < 0 || b >= k) {
        bad = true;
        continue;
      }
      if (b < 64) lo |= 1ull << b;
      else hi |= 1ull << (b - 64);
    }
    lo = wave_or_u64(lo);
    hi = wave_or_u64(hi);
    const int lambda = __popcll(lo) + __popcll(hi);
    if (l == 0 && lambda > 0) acc += (long long)(nw ? nw[e] : 1) * (lambda - 1);
  }
  const bool wave_bad = ballot(bad) != 0ull;
  if (l == 0) {
    wsum[w] = acc;
    wbad[w] = wave_bad ? 1 : 0;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    long long s = 0;
    int b = 0;
    for (int i = 0; i < kStaticThreads / kWave; ++i) {
      s += wsum[i];
      b |= wbad[i];
    }
    slots[blockIdx.x] = b ? kBadSlot : s;
  }
}

// Adds slots[0..count) in a fixed order (per thread by stride, then a fixed tree); -1 if any
// slot is marked bad.
__global__ __launch_bounds__(kSumThreads) void k_static_sum(const long long *__restrict__ slots, int32_t count,
                                                            int64_t *__restrict__ out) {
  __shared__ long long part_sum[kSumThreads];
  __shared__ int any_bad;
  if (threadIdx.x == 0) any_bad = 0;
  __syncthreads();
  long long s = 0;
  for (int32_t i = threadIdx.x; i < count; i += kSumThreads) {
    const long long x = slots[i];
    if (x == kBadSlot) any_bad = 1;
    else s += x;
  }
  part_sum[threadIdx.x] = s;
  __syncthreads();
  for (int h = kSumThreads / 2; h >= 1; h >>= 1) {
    if ((int)threadIdx.x < h) part_sum[threadIdx.x] += part_sum[threadIdx.x + h];
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = any_bad ? -1 : part_sum[0];
}

std::mutex g_static_mu;
constexpr int kMaxDevices = 64;
long long *g_static_ptr[kMaxDevices] = {};
thread_local std::string g_static_error;

}  // namespace

}  // namespace jet

extern "C" int jet_km1_static(int32_t n, int32_t m, int64_t num_pins, const int64_t *net_offsets, const int32_t *pins,
                              const int32_t *net_weights, const int32_t *part, int32_t k, int64_t *km1,
                              void *stream) {
  using namespace jet;
  g_static_error.clear();
  if (n < 1 || m < 1 || num_pins < 1 || num_pins > INT32_MAX) {
    g_static_error = "n, m and num_pins must be >= 1 and num_pins < 2^31";
    return JET_EINVAL;
  }
  if (k < 2 || k > kMaxK) {
    g_static_error = "k outside [2,128]";
    return JET_EINVAL;
  }
  if (!net_offsets || !pins || !part || !km1) {
    g_static_error = "net_offsets, pins, part or km1 is NULL";
    return JET_EINVAL;
  }
  if ((int64_t)m > kStaticMaxNets) {
    g_static_error = "m = " + std::to_string(m) + " exceeds the " + std::to_string(kStaticMaxNets) +
                     " nets the static partial-sum array covers";
    return JET_EUNSUPPORTED;
  }
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    g_static_error = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return JET_EHIP;
  }
  long long *slots = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_static_mu);
    if (!g_static_ptr[dev]) {
      void *p = nullptr;
      e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p) {
        g_static_error = std::string("hipGetSymbolAddress: ") + hipGetErrorString(e);
        return JET_EHIP;
      }
      g_static_ptr[dev] = (long long *)p;
    }
    slots = g_static_ptr[dev];
  }
  const int32_t groups = (int32_t)(((int64_t)m + kStaticNetsPerGroup - 1) / kStaticNetsPerGroup);
  hipStream_t s = (hipStream_t)stream;
  hipLaunchKernelGGL(k_static_km1, dim3((unsigned)groups), dim3(kStaticThreads), 0, s, net_offsets, pins, net_weights,
                     part, n, m, num_pins, k, slots);
  hipLaunchKernelGGL(k_static_sum, dim3(1), dim3(kSumThreads), 0, s, slots, groups, km1);
  e = hipGetLastError();
  if (e != hipSuccess) {
    g_static_error = std::string("launch: ") + hipGetErrorString(e);
    return JET_EHIP;
  }
  return JET_OK;
}

extern "C" const char *jet_km1_static_last_error(void) { return jet::g_static_error.c_str(); }
