// Afterburner (Algorithm 2) for the rare large nets whose interleaved events do not fit in LDS.
//
// A block b of net e is interleaved when every pin of e in b is a candidate leaving b and other
// candidates arrive in b; then the order of b's events decides which ones change lambda(e).  One
// 1024-thread workgroup per such net:
//   1. recounts departures / arrivals per block and finds the interleaved blocks;
//   2. writes one event (block, execution-order key, kind) per candidate and interleaved block it
//      touches into global scratch;
//   3. sorts the events by (block, key) with a stable LSD radix sort (8-bit digits; passes whose
//      digit is constant are skipped);
//   4. walks each block's events in order with a segmented prefix sum: the count of b before an
//      event is phi_e[b] + (arrivals - departures) so far; a departure that finds 1 earns w(e), an
//      arrival that finds 0 costs w(e).
#include "dev_util.h"
#include "jet_internal.h"
#include "rec.h"

namespace jet {

namespace {

constexpr int kOT = 1024;
constexpr int kOW = kOT / kWave;

struct LsdShared {
  uint32_t hist[256];
  uint32_t wcnt[kOW][256];
  int32_t skip;
};

// One stable counting pass by the digit `pass` (0..7: byte of the key, 8: the block byte of the
// meta word).  Returns false (and writes nothing) if every event has the same digit.
__device__ bool lsd_pass(const unsigned long long *__restrict__ kin, const uint32_t *__restrict__ min,
                         unsigned long long *__restrict__ kout, uint32_t *__restrict__ mout, int32_t E, int pass,
                         LsdShared &sh) {
  const int tid = threadIdx.x, w = tid / kWave;
  auto digit = [&](int32_t i) -> uint32_t {
    return pass < 8 ? (uint32_t)(kin[i] >> (8 * pass)) & 0xffu : (min[i] & 0xffu);
  };
  if (tid < 256) sh.hist[tid] = 0;
  if (tid == 0) sh.skip = 0;
  __syncthreads();
  for (int32_t i = tid; i < E; i += kOT) atomicAdd(&sh.hist[digit(i)], 1u);
  __syncthreads();
  if (tid < 256 && sh.hist[tid] == (uint32_t)E) sh.skip = 1;
  __syncthreads();
  const bool skip = sh.skip != 0;
  __syncthreads();  // every thread has read the flag before the next pass clears it
  if (skip) return false;
  if (tid == 0) {
    uint32_t run = 0;
    for (int d = 0; d < 256; ++d) {
      const uint32_t c = sh.hist[d];
      sh.hist[d] = run;
      run += c;
    }
  }
  __syncthreads();
  for (int32_t tb = 0; tb < E; tb += kOT) {
    const int32_t i = tb + tid;
    const bool valid = i < E;
    unsigned long long key = 0;
    uint32_t meta = 0, d = 0;
    if (valid) {
      key = kin[i];
      meta = min[i];
      d = pass < 8 ? (uint32_t)(key >> (8 * pass)) & 0xffu : (meta & 0xffu);
    }
    uint64_t same = ballot(valid);
#pragma unroll
    for (int bit = 0; bit < 8; ++bit) {
      const uint64_t b = ballot(valid && ((d >> bit) & 1u));
      same &= ((d >> bit) & 1u) ? b : ~b;
    }
    const int rank = rank_below(same);
    for (int j = tid; j < kOW * 256; j += kOT) (&sh.wcnt[0][0])[j] = 0;
    __syncthreads();
    if (valid && rank == __popcll(same) - 1) sh.wcnt[w][d] = (uint32_t)__popcll(same);
    __syncthreads();
    if (tid < 256) {
      uint32_t run = sh.hist[tid];
      for (int ww = 0; ww < kOW; ++ww) {
        const uint32_t c = sh.wcnt[ww][tid];
        sh.wcnt[ww][tid] = run;
        run += c;
      }
      sh.hist[tid] = run;
    }
    __syncthreads();
    if (valid) {
      const uint32_t pos = sh.wcnt[w][d] + (uint32_t)rank;
      kout[pos] = key;
      mout[pos] = meta;
    }
    __syncthreads();
  }
  return true;
}

template <typename T>
__global__ __launch_bounds__(kOT) void k_ab_overflow(const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ pins,
                                                     const int32_t *__restrict__ nw,
                                                     const uint32_t *__restrict__ inm,
                                                     const uint64_t *__restrict__ rec,
                                                     const T *__restrict__ phi, int32_t k,
                                                     RgSink rg, const DevStatus *st,
                                                     const int2 *__restrict__ ovf_list,
                                                     const int64_t *__restrict__ ovf_off,
                                                     unsigned long long *__restrict__ ka,
                                                     unsigned long long *__restrict__ kb,
                                                     uint32_t *__restrict__ ma, uint32_t *__restrict__ mb,
                                                     const LoopCtl *lc) {
  JET_GATE(lc, kPhJet);
  __shared__ int32_t D[kMaxK], A[kMaxK], P0[kMaxK], seg_base[kMaxK];
  __shared__ uint8_t mixed[kMaxK];
  __shared__ int32_t sm[kOW + 1];
  __shared__ LsdShared sh;
  __shared__ int32_t s_carry;
  if ((int32_t)blockIdx.x >= st->n_ovf) return;
  const int tid = threadIdx.x;
  const int2 item = ovf_list[blockIdx.x];
  const int32_t e = item.y;
  const int64_t q0 = off[e], q1 = off[e + 1];
  const int32_t wgt = nw ? nw[e] : 1;
  const int64_t base = ovf_off[item.x];
  unsigned long long *K0 = ka + base, *K1 = kb + base;
  uint32_t *M0 = ma + base, *M1 = mb + base;

  for (int b = tid; b < k; b += kOT) {
    D[b] = 0;
    A[b] = 0;
  }
  __syncthreads();
  for (int64_t q = q0 + tid; q < q1; q += kOT) {
    const int32_t v = pins[q];
    if (inm_bit(inm, v)) {
      const uint64_t r = rec[v];
      atomicAdd(&D[rec_source(r)], 1);
      atomicAdd(&A[rec_target(r)], 1);
    }
  }
  __syncthreads();
  for (int b = tid; b < k; b += kOT) {
    const int32_t p0 = (int32_t)phi[(int64_t)e * k + b];
    P0[b] = p0;
    mixed[b] = (D[b] > 0 && A[b] > 0 && p0 == D[b]) ? 1 : 0;
  }
  __syncthreads();

  // events: departures from and arrivals into interleaved blocks
  int32_t E = 0;
  for (int64_t qb = q0; qb < q1; qb += kOT) {
    const int64_t q = qb + tid;
    int32_t v = 0, s = 0, t = 0, g = 0;
    bool dep = false, arr = false;
    if (q < q1) {
      v = pins[q];
      if (inm_bit(inm, v)) {
        const uint64_t r = rec[v];
        s = rec_source(r);
        t = rec_target(r);
        g = rec_gain(r);
        dep = mixed[s] != 0;
        arr = mixed[t] != 0;
      }
    }
    int32_t tot;
    const int32_t pos = E + block_excl_scan<kOT>((dep ? 1 : 0) + (arr ? 1 : 0), sm, &tot);
    const unsigned long long key = order_key(g, v);
    if (dep) {
      K0[pos] = key;
      M0[pos] = (uint32_t)s;
    }
    if (arr) {
      K0[pos + (dep ? 1 : 0)] = key;
      M0[pos + (dep ? 1 : 0)] = (uint32_t)t | 0x100u;
    }
    E += tot;
  }
  __syncthreads();

  // sort by (block, key)
  bool in0 = true;
  for (int pass = 0; pass < 9; ++pass) {
    const bool moved = in0 ? lsd_pass(K0, M0, K1, M1, E, pass, sh) : lsd_pass(K1, M1, K0, M0, E, pass, sh);
    if (moved) in0 = !in0;
  }
  const unsigned long long *KS = in0 ? K0 : K1;
  const uint32_t *MS = in0 ? M0 : M1;

  // segmented walk
  if (tid == 0) s_carry = 0;
  __syncthreads();
  for (int32_t tb = 0; tb < E; tb += kOT) {
    const int32_t i = tb + tid;
    const bool valid = i < E;
    uint32_t meta = 0;
    if (valid) meta = MS[i];
    const int32_t blk = (int32_t)(meta & 0xffu);
    const bool arrival = (meta >> 8) & 1u;
    const int32_t carry = s_carry;
    int32_t tot;
    const int32_t P = carry + block_excl_scan<kOT>(valid ? (arrival ? 1 : -1) : 0, sm, &tot);
    if (valid && (i == 0 || (int32_t)(MS[i - 1] & 0xffu) != blk)) seg_base[blk] = P;
    __syncthreads();
    if (valid) {
      const int32_t before = P0[blk] + P - seg_base[blk];
      const int32_t v = (int32_t)(uint32_t)KS[i];
      if (!arrival && before == 1) rg_add(rg, blockIdx.x, v, wgt);
      if (arrival && before == 0) rg_add(rg, blockIdx.x, v, -wgt);
    }
    __syncthreads();
    if (tid == 0) s_carry = carry + tot;
    __syncthreads();
  }
}

}  // namespace

hipError_t launch_afterburner_overflow(Ctx &c, RgSink sink, const LoopCtl *lc) {
  if (c.nbig_over == 0) return hipSuccess;
  if (c.phi16)
    hipLaunchKernelGGL(k_ab_overflow<uint16_t>, dim3((unsigned)c.nbig_over), dim3(kOT), 0, c.stream, c.off, c.pins,
                       c.nw, c.inm, c.rec, c.phi16, c.k, sink, c.st, c.ovf_list, c.ovf_off, c.ovf_ka, c.ovf_kb, c.ovf_ma,
                       c.ovf_mb, lc);
  else
    hipLaunchKernelGGL(k_ab_overflow<int32_t>, dim3((unsigned)c.nbig_over), dim3(kOT), 0, c.stream, c.off, c.pins,
                       c.nw, c.inm, c.rec, c.phi, c.k, sink, c.st, c.ovf_list, c.ovf_off, c.ovf_ka, c.ovf_kb, c.ovf_ma,
                       c.ovf_mb, lc);
  return hipGetLastError();
}

}  // namespace jet
