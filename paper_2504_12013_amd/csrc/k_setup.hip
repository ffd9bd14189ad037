// Setup kernels (once per hypergraph): input validation, the incidence transpose I(v) (Section 2:
// incident nets of a vertex), incident weight sums, and a device exclusive scan.
#include "dev_util.h"
#include "jet_internal.h"

namespace jet {

namespace {

__device__ __forceinline__ void flag_error(DevStatus *st, int32_t code, int32_t arg) {
  if (atomicCAS(&st->err, 0, code) == 0) st->err_arg = arg;
}

__global__ void k_check_pins_degrees(const int32_t *__restrict__ pins, int64_t p, int32_t n,
                                     int32_t *__restrict__ deg, DevStatus *st) {
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < p; q += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = pins[q];
    if (v < 0 || v >= n) {
      flag_error(st, kErrPinRange, (int32_t)(q & 0x7fffffff));
      continue;
    }
    if (deg) atomicAdd(&deg[v], 1);
  }
}

// one wave per net; lanes stride over its pins and claim a slot in each pin's incidence list
__global__ void k_fill_incidence(const int64_t *__restrict__ off, const int32_t *__restrict__ pins, int32_t m,
                                 unsigned long long *__restrict__ cursor, int32_t *__restrict__ inc) {
  const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int l = lane_id();
  if (wid >= m) return;
  const int32_t e = (int32_t)wid;
  for (int64_t q = off[e] + l; q < off[e + 1]; q += kWave) {
    const int32_t v = pins[q];
    const unsigned long long pos = atomicAdd(&cursor[v], 1ull);
    inc[pos] = e;
  }
}

// Sort each incidence list ascending (deterministic layout) and detect repeated pins.  Lists up to
// 64 entries: insertion sort by one thread.  Longer lists are deferred to k_sort_long.
__global__ void k_sort_short(const int64_t *__restrict__ voff, int32_t *__restrict__ inc, int32_t n,
                             int32_t *__restrict__ long_list, int32_t *__restrict__ long_cnt, DevStatus *st) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t a = voff[v], b = voff[v + 1];
  const int64_t d = b - a;
  if (d > kSmallNet) {
    const int pos = atomicAdd(long_cnt, 1);
    long_list[pos] = (int32_t)v;
    return;
  }
  for (int64_t i = a + 1; i < b; ++i) {
    const int32_t x = inc[i];
    int64_t j = i - 1;
    while (j >= a && inc[j] > x) {
      inc[j + 1] = inc[j];
      --j;
    }
    inc[j + 1] = x;
  }
  for (int64_t i = a + 1; i < b; ++i)
    if (inc[i] == inc[i - 1]) flag_error(st, kErrDupPin, (int32_t)v);
}

// bitonic sort of one long incidence list in LDS (<= kMaxSortedDegree entries), one block per vertex
__global__ __launch_bounds__(1024) void k_sort_long(const int64_t *__restrict__ voff, int32_t *__restrict__ inc,
                                                    const int32_t *__restrict__ long_list, DevStatus *st) {
  __shared__ int32_t buf[kMaxSortedDegree];
  const int32_t v = long_list[blockIdx.x];
  const int64_t a = voff[v];
  const int32_t d = (int32_t)(voff[v + 1] - a);
  if (d > kMaxSortedDegree) return;  // sorted by k_sort_huge
  int32_t N = 1;
  while (N < d) N <<= 1;
  for (int32_t i = threadIdx.x; i < N; i += blockDim.x) buf[i] = i < d ? inc[a + i] : INT32_MAX;
  __syncthreads();
  for (int32_t size = 2; size <= N; size <<= 1) {
    for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (int32_t i = threadIdx.x; i < N / 2; i += blockDim.x) {
        const int32_t lo = 2 * i - (i & (stride - 1));
        const int32_t hi = lo + stride;
        const bool up = (lo & size) == 0;
        const int32_t x = buf[lo], y = buf[hi];
        if ((x > y) == up) {
          buf[lo] = y;
          buf[hi] = x;
        }
      }
      __syncthreads();
    }
  }
  for (int32_t i = threadIdx.x; i < d; i += blockDim.x) {
    inc[a + i] = buf[i];
    if (i > 0 && buf[i] == buf[i - 1]) flag_error(st, kErrDupPin, v);
  }
}

// Incidence lists longer than kMaxSortedDegree: LSD radix sort of the net IDs (8-bit digits) by
// one 1024-thread block per vertex, ping-ponging between the list and its slot range in `tmp`.
constexpr int kHugeThreads = 1024;
__global__ __launch_bounds__(kHugeThreads) void k_sort_huge(const int64_t *__restrict__ voff,
                                                            int32_t *__restrict__ inc, int32_t *__restrict__ tmp,
                                                            const int32_t *__restrict__ huge_list, DevStatus *st) {
  constexpr int NW = kHugeThreads / kWave;
  __shared__ uint32_t hist[256];
  __shared__ uint32_t wcnt[NW][256];
  const int tid = threadIdx.x, w = tid / kWave;
  const int32_t v = huge_list[blockIdx.x];
  const int64_t a = voff[v];
  const int32_t d = (int32_t)(voff[v + 1] - a);
  if (d <= kMaxSortedDegree) return;  // sorted in LDS by k_sort_long
  uint32_t *src = (uint32_t *)(inc + a), *dst = (uint32_t *)(tmp + a);
  for (int pass = 0; pass < 4; ++pass) {
    const int sh = 8 * pass;
    if (tid < 256) hist[tid] = 0;
    __syncthreads();
    for (int32_t i = tid; i < d; i += kHugeThreads) atomicAdd(&hist[(src[i] >> sh) & 0xffu], 1u);
    __syncthreads();
    if (tid == 0) {
      uint32_t run = 0;
      for (int x = 0; x < 256; ++x) {
        const uint32_t c = hist[x];
        hist[x] = run;
        run += c;
      }
    }
    __syncthreads();
    for (int32_t tb = 0; tb < d; tb += kHugeThreads) {
      const int32_t i = tb + tid;
      const bool valid = i < d;
      const uint32_t key = valid ? src[i] : 0u;
      const uint32_t dg = (key >> sh) & 0xffu;
      uint64_t same = ballot(valid);
#pragma unroll
      for (int bit = 0; bit < 8; ++bit) {
        const uint64_t b = ballot(valid && ((dg >> bit) & 1u));
        same &= ((dg >> bit) & 1u) ? b : ~b;
      }
      const int rank = rank_below(same);
      for (int j = tid; j < NW * 256; j += kHugeThreads) (&wcnt[0][0])[j] = 0;
      __syncthreads();
      if (valid && rank == __popcll(same) - 1) wcnt[w][dg] = (uint32_t)__popcll(same);
      __syncthreads();
      if (tid < 256) {
        uint32_t run = hist[tid];
        for (int ww = 0; ww < NW; ++ww) {
          const uint32_t c = wcnt[ww][tid];
          wcnt[ww][tid] = run;
          run += c;
        }
        hist[tid] = run;
      }
      __syncthreads();
      if (valid) dst[wcnt[w][dg] + rank] = key;
      __syncthreads();
    }
    uint32_t *t = src;
    src = dst;
    dst = t;
  }
  // four passes: the sorted list is back in inc
  for (int32_t i = tid + 1; i < d; i += kHugeThreads)
    if (src[i] == src[i - 1]) flag_error(st, kErrDupPin, v);
}

// omega(I(v)) with overflow detection
__global__ void k_sumw(const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
                       const int32_t *__restrict__ nw, int32_t n, int32_t *__restrict__ sumw, DevStatus *st) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  int64_t s = 0;
  for (int64_t q = voff[v]; q < voff[v + 1]; ++q) s += nw ? nw[inc[q]] : 1;
  if (s > INT32_MAX) {
    flag_error(st, kErrOverflow, (int32_t)v);
    s = INT32_MAX;
  }
  sumw[v] = (int32_t)s;
}

__global__ void k_check_weights(const int32_t *__restrict__ w, int64_t len, unsigned long long *__restrict__ total,
                                DevStatus *st) {
  int64_t s = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t x = w[i];
    if (x < 1) flag_error(st, kErrWeight, (int32_t)(i & 0x7fffffff));
    s += x;
  }
  s = wave_sum(s);
  if (lane_id() == 0 && total) atomicAdd(total, (unsigned long long)s);
}

// ---- exclusive scan int32 -> int64 (three phases)
constexpr int kScanBlock = 256, kScanItems = 8, kScanTile = kScanBlock * kScanItems;

__global__ __launch_bounds__(kScanBlock) void k_scan_partials(const int32_t *__restrict__ in, int64_t len,
                                                              int64_t *__restrict__ part) {
  __shared__ int64_t sm[kScanBlock / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + (int64_t)i * kScanBlock + threadIdx.x;
    if (idx < len) s += in[idx];
  }
  s = wave_sum(s);
  if (lane_id() == 0) sm[threadIdx.x / kWave] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t t = 0;
    for (int w = 0; w < kScanBlock / kWave; ++w) t += sm[w];
    part[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(1024) void k_scan_single(int64_t *__restrict__ part, int64_t cnt) {
  __shared__ int64_t sm[1024 / kWave + 1];
  int64_t carry = 0;
  for (int64_t base = 0; base < cnt; base += 1024) {
    const int64_t idx = base + threadIdx.x;
    const int64_t x = idx < cnt ? part[idx] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan<1024>(x, sm, &tot);
    if (idx < cnt) part[idx] = carry + ex;
    carry += tot;
  }
}

__global__ __launch_bounds__(kScanBlock) void k_scan_final(const int32_t *__restrict__ in, int64_t len,
                                                           const int64_t *__restrict__ part,
                                                           int64_t *__restrict__ out) {
  __shared__ int64_t sm[kScanBlock / kWave + 1];
  const int64_t base = (int64_t)blockIdx.x * kScanTile;
  int64_t carry = part[blockIdx.x];
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t idx = base + (int64_t)i * kScanBlock + threadIdx.x;
    const int64_t x = idx < len ? in[idx] : 0;
    int64_t tot;
    const int64_t ex = block_excl_scan<kScanBlock>(x, sm, &tot);
    if (idx < len) out[idx] = carry + ex;
    carry += tot;
  }
  // the element after the last one receives the grand total
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) out[len] = carry;
}

inline unsigned grid_for(int64_t work, int block, int64_t cap = 1 << 20) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

hipError_t launch_check_pins(Ctx &c) {
  hipLaunchKernelGGL(k_check_pins_degrees, dim3(grid_for(c.p, 256, 65536)), dim3(256), 0, c.stream, c.pins, c.p,
                     c.n, (int32_t *)nullptr, c.st);
  return hipGetLastError();
}

hipError_t launch_degrees(Ctx &c, int32_t *deg) {
  hipLaunchKernelGGL(k_check_pins_degrees, dim3(grid_for(c.p, 256, 65536)), dim3(256), 0, c.stream, c.pins, c.p,
                     c.n, deg, c.st);
  return hipGetLastError();
}

hipError_t launch_exclusive_scan_i32_to_i64(Ctx &c, const int32_t *in, int64_t *out, int64_t len) {
  const int64_t tiles = (len + kScanTile - 1) / kScanTile;
  const int64_t t = tiles < 1 ? 1 : tiles;
  if (c.scan_tmp_len < t) {
    if (c.scan_tmp) (void)hipFree(c.scan_tmp);
    c.scan_tmp = nullptr;
    c.scan_tmp_len = 0;
    hipError_t e = hipMalloc(&c.scan_tmp, sizeof(int64_t) * t);
    if (e != hipSuccess) return e;
    c.scan_tmp_len = t;
  }
  hipLaunchKernelGGL(k_scan_partials, dim3((unsigned)t), dim3(kScanBlock), 0, c.stream, in, len, c.scan_tmp);
  hipLaunchKernelGGL(k_scan_single, dim3(1), dim3(1024), 0, c.stream, c.scan_tmp, t);
  hipLaunchKernelGGL(k_scan_final, dim3((unsigned)t), dim3(kScanBlock), 0, c.stream, in, len, c.scan_tmp, out);
  return hipGetLastError();
}

hipError_t launch_fill_incidence(Ctx &c, int64_t *cursor) {
  const int64_t threads = (int64_t)c.m * kWave;
  hipLaunchKernelGGL(k_fill_incidence, dim3(grid_for(threads, 256, INT32_MAX)), dim3(256), 0, c.stream, c.off,
                     c.pins, c.m, (unsigned long long *)cursor, c.inc);
  return hipGetLastError();
}

hipError_t launch_sort_incidence(Ctx &c) {
  int32_t *long_list = nullptr, *long_cnt = nullptr;
  hipError_t e = hipMalloc(&long_list, sizeof(int32_t) * ((size_t)c.n + 1));
  if (e != hipSuccess) return e;
  long_cnt = long_list + c.n;
  e = hipMemsetAsync(long_cnt, 0, sizeof(int32_t), c.stream);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_sort_short, dim3(grid_for(c.n, 256, INT32_MAX)), dim3(256), 0, c.stream, c.voff, c.inc,
                       c.n, long_list, long_cnt, c.st);
    e = hipGetLastError();
  }
  int32_t cnt = 0;
  if (e == hipSuccess) e = hipMemcpyAsync(&cnt, long_cnt, sizeof(int32_t), hipMemcpyDeviceToHost, c.stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  if (e == hipSuccess && cnt > 0) {
    hipLaunchKernelGGL(k_sort_long, dim3((unsigned)cnt), dim3(1024), 0, c.stream, c.voff, c.inc, long_list, c.st);
    e = hipGetLastError();
    int32_t *tmp = nullptr;
    if (e == hipSuccess) e = hipMalloc(&tmp, sizeof(int32_t) * (size_t)c.p);
    if (e == hipSuccess) {
      hipLaunchKernelGGL(k_sort_huge, dim3((unsigned)cnt), dim3(kHugeThreads), 0, c.stream, c.voff, c.inc, tmp,
                         long_list, c.st);
      e = hipGetLastError();
      hipError_t e2 = hipStreamSynchronize(c.stream);
      if (e == hipSuccess) e = e2;
      (void)hipFree(tmp);
    }
  }
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_sumw, dim3(grid_for(c.n, 256, INT32_MAX)), dim3(256), 0, c.stream, c.voff, c.inc, c.nw,
                       c.n, c.sumw, c.st);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipStreamSynchronize(c.stream);
  (void)hipFree(long_list);
  return e;
}

hipError_t launch_check_weights(Ctx &c) {
  // total vertex weight lands in st->bw[0] as scratch (the status block is rebuilt before use)
  hipError_t e = hipMemsetAsync(&c.st->bw[0], 0, sizeof(int64_t), c.stream);
  if (e != hipSuccess) return e;
  if (c.vw) {
    hipLaunchKernelGGL(k_check_weights, dim3(grid_for(c.n, 256, 4096)), dim3(256), 0, c.stream, c.vw, (int64_t)c.n,
                       (unsigned long long *)&c.st->bw[0], c.st);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  if (c.nw) {
    hipLaunchKernelGGL(k_check_weights, dim3(grid_for(c.m, 256, 4096)), dim3(256), 0, c.stream, c.nw, (int64_t)c.m,
                       (unsigned long long *)nullptr, c.st);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace jet
