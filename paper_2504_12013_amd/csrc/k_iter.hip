// One Jet iteration on the device (Section 4.1, Algorithm 2):
//   candidates  -> best adjacent target, gain and temperature filter per vertex
//   afterburner -> recomputed gains by replaying the ordered candidates per net
//   select      -> kept moves X = {v in M : recomputed gain > 0}, locks
//   apply       -> partition, pin counts, block weights and metric, then connectivity words
// Every cross-thread combination is an integer sum (or an idempotent bit update derived from final
// counts), so the outcome does not depend on scheduling.
#include <algorithm>

#include "chunk.h"
#include "dev_util.h"
#include "moves.h"
#include "jet_internal.h"
#include "rec.h"
#include "conn.h"
#include "phi.h"

namespace jet {

namespace {

// ------------------------------------------------------------------ candidates (Section 4.1)
//
// Every unlocked vertex v of block s picks the adjacent foreign block t of largest conn (lowest ID
// on ties), i.e. of largest gain conn[t] - aff, and is a candidate iff
//     65536 gain + tau_q aff >= 0        (gain >= -tau aff with tau = tau_q / 65536).
// Vertices with at most kHubDegree incident nets: G lanes per vertex (conn.h).  Hubs: one
// workgroup per vertex (k_candidates_hub).

__device__ __forceinline__ void finish_candidate(int32_t v, int32_t s, int32_t bestc, int32_t bestb, int32_t sumw_v,
                                                 int32_t benefit, int32_t tau_q, uint64_t *__restrict__ rec,
                                                 bool *cand_out) {
  bool cand = false;
  uint64_t r;
  if (bestc > 0) {
    const int32_t aff = sumw_v - benefit;
    const int32_t g = bestc - aff;
    cand = 65536ll * (int64_t)g + (int64_t)tau_q * (int64_t)aff >= 0;
    r = pack_rec(g, bestb, s);
  } else {
    r = pack_rec(0, 0xff, s);
  }
  rec[v] = r;
  *cand_out = cand;
}

template <int G, bool UNIT>
__global__ __launch_bounds__(G == 16 ? 512 : 256) void k_candidates(
    const int32_t *__restrict__ part, const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
    const int32_t *__restrict__ nw, const uint64_t *__restrict__ ns, const int32_t *__restrict__ sumw,
    const int32_t *__restrict__ lockstamp, int32_t locked_stamp, const uint8_t *__restrict__ lock_bytes, int32_t n,
    int32_t tau_q, uint64_t *__restrict__ rec, uint32_t *__restrict__ inm, DevStatus *st, const LoopCtl *lc,
    Union u) {
  JET_GATE(lc, kPhJet);
  if (lc && !u.lcs) {
    locked_stamp = lc->stamp - 1;
    tau_q = lc->tau_q;
  }
  constexpr int BLOCK = (G == 16) ? 512 : 256;
  constexpr int VPB = BLOCK / G;
  __shared__ uint32_t words[VPB / 32];
  __shared__ unsigned long long scanned;
  __shared__ int32_t ncand;
  const int lg = threadIdx.x % G;
  const int vl = threadIdx.x / G;
  if (threadIdx.x == 0) {
    scanned = 0ull;
    ncand = 0;
  }
  // union: only the tiles of the hypergraphs in their Jet phase (VPB divides the tile size)
  const ActList *AL = u.lcs ? &u.act[kActJet] : nullptr;
  const int64_t nv = AL ? (int64_t)AL->tpref[AL->cnt] * kUnionTile : (int64_t)n;
  const int64_t ntiles = (nv + VPB - 1) / VPB;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {  // block-uniform trip count
    const int64_t vb = AL ? act_tile_base(*AL, u.ht0, (int32_t)(tile * VPB / kUnionTile)) + (tile * VPB) % kUnionTile
                          : tile * VPB;
    const int64_t v = vb + vl;
    if (threadIdx.x < VPB / 32) words[threadIdx.x] = 0u;
    __syncthreads();
    const bool valid = v < n;
    int32_t s = 0, tq = tau_q;
    bool skip = true, hub = false;
    int64_t q0 = 0, q1 = 0;
    if (valid) {
      s = part[v];
      q0 = voff[v];
      q1 = voff[v + 1];
      hub = q1 - q0 > kHubDegree;
      int32_t ls = locked_stamp;
      bool off = false;
      if (u.lcs) {  // the vertex's own hypergraph decides (union)
        const LoopCtl &h = u.lcs[u.vhg[v]];
        off = h.phase != kPhJet;
        ls = h.stamp - 1;
        tq = h.tau_q;
      }
      const bool locked = lock_bytes ? (lock_bytes[v] != 0) : (lockstamp[v] == ls);
      skip = locked || hub || off;
    }
    int32_t conn[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) conn[j] = 0;
    int32_t benefit = 0;
    if (!skip) vertex_conn<G, UNIT>(inc, q0, q1, G, nw, ns, lg, s, conn, benefit);
    int32_t bestc = 0, bestb = INT32_MAX;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      const int32_t b = lg * 8 + j;
      if (b != s && conn[j] > bestc) {
        bestc = conn[j];
        bestb = b;
      }
    }
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      const int32_t oc = __shfl_xor(bestc, o, G);
      const int32_t ob = __shfl_xor(bestb, o, G);
      if (oc > bestc || (oc == bestc && ob < bestb)) {
        bestc = oc;
        bestb = ob;
      }
    }
    if (valid && !hub && lg == 0) {
      bool cand = false;
      finish_candidate((int32_t)v, s, skip ? 0 : bestc, bestb, sumw[v], benefit, tq, rec, &cand);
      if (cand) atomicOr(&words[vl >> 5], 1u << (vl & 31));
      if (!skip) atomicAdd(&scanned, (unsigned long long)(q1 - q0));
    }
    __syncthreads();
    if (threadIdx.x < VPB / 32) {
      const uint32_t wv = words[threadIdx.x];
      inm[vb / 32 + threadIdx.x] = wv;
      if (wv) atomicAdd(&ncand, __popc(wv));
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (ncand) atomicAdd(&st->n_cand, ncand);
    if (scanned) atomicAdd((unsigned long long *)&st->inc_low, scanned);
  }
}

// Unit net weights and k <= 64: G lanes per vertex (G = 1 on light levels), each accumulating
// the bit-sliced counts of its share of the incident nets (conn.h), summed over the group at the
// end.  The best target is the lowest block of largest count among the adjacent blocks other than
// s.  Same records and flags as k_candidates (exact integer counts, same tie rule), with no
// per-net shuffles and no barriers.  With G = 1 a wave writes its two candidate words itself;
// otherwise it ORs its bits into a word cleared before the launch.
template <int G>
__global__ __launch_bounds__(256) void k_candidates_bits(
    const int32_t *__restrict__ part, const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
    const uint64_t *__restrict__ ns, const int32_t *__restrict__ sumw, const int32_t *__restrict__ lockstamp,
    int32_t locked_stamp, const uint8_t *__restrict__ lock_bytes, int32_t n, int32_t tau_q,
    uint64_t *__restrict__ rec, uint32_t *__restrict__ inm, DevStatus *st, const LoopCtl *lc, Union u,
    int32_t xcd) {
  JET_GATE(lc, kPhJet);
  if (lc && !u.lcs) {
    locked_stamp = lc->stamp - 1;
    tau_q = lc->tau_q;
  }
  constexpr int VPW = kWave / G;  // vertices per wave and step
  __shared__ unsigned long long wscan[4];
  __shared__ int32_t wcand[4];
  const int l = lane_id(), w = threadIdx.x / kWave, lg = l % G;
  unsigned long long scanned = 0ull;
  int32_t ncand = 0;
  // union: only the tiles of the hypergraphs in their Jet phase (VPW divides the tile size)
  const ActList *AL = u.lcs ? &u.act[kActJet] : nullptr;
  const int64_t nv = AL ? (int64_t)AL->tpref[AL->cnt] * kUnionTile : (int64_t)n;
  // Workgroups go to the eight XCDs round robin.  With xcd set, the workgroups of one XCD walk one
  // contiguous eighth of the vertex range, so the nets of neighbouring vertices are fetched into
  // that XCD's L2 once instead of into all eight.
  int64_t vstart = ((int64_t)blockIdx.x * 4 + w) * VPW, vend = nv, vstep = (int64_t)gridDim.x * 4 * VPW;
  if (xcd && !AL && gridDim.x % 8 == 0) {
    const int64_t span = 4 * VPW;                      // vertices of one workgroup step
    const int64_t steps = (nv + span - 1) / span;
    const int64_t per = (steps + 7) / 8;               // workgroup steps of one XCD
    const int64_t x = blockIdx.x % 8, j = blockIdx.x / 8;
    vstart = (x * per + j) * span + w * VPW;
    vend = std::min<int64_t>(nv, (x + 1) * per * span);
    vstep = (int64_t)(gridDim.x / 8) * span;
  }
  for (int64_t vbase = vstart; vbase < vend; vbase += vstep) {  // wave-uniform trip count
    const int64_t base =
        AL ? act_tile_base(*AL, u.ht0, (int32_t)(vbase / kUnionTile)) + vbase % kUnionTile : vbase;
    const int64_t v = base + l / G;
    const bool valid = v < n;
    int32_t s = 0, tq = tau_q;
    bool skip = true, hub = false;
    int64_t q0 = 0, q1 = 0;
    if (valid) {
      s = part[v];
      q0 = voff[v];
      q1 = voff[v + 1];
      hub = q1 - q0 > kHubDegree;
      int32_t ls = locked_stamp;
      bool off = false;
      if (u.lcs) {  // the vertex's own hypergraph decides (union)
        const LoopCtl &h = u.lcs[u.vhg[v]];
        off = h.phase != kPhJet;
        ls = h.stamp - 1;
        tq = h.tau_q;
      }
      const bool locked = lock_bytes ? (lock_bytes[v] != 0) : (lockstamp[v] == ls);
      skip = locked || hub || off;
    }
    uint64_t pl[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) pl[p] = 0ull;
    int32_t benefit = 0;
    const uint64_t sbit = 1ull << s;
    if (!skip) planes_accumulate<G>(inc, q0, q1, ns, lg, sbit, pl, benefit);
    planes_combine<G>(pl, benefit);
    uint64_t any = 0ull;
#pragma unroll
    for (int p = 0; p < 9; ++p) any |= pl[p];
    int32_t bestb;
    const int32_t bestc = planes_best(pl, any & ~sbit, bestb);  // adjacent blocks other than s
    bool cand = false;
    if (valid && !hub && lg == 0) {
      finish_candidate((int32_t)v, s, skip ? 0 : (bestc > 0 ? bestc : 0), bestb, sumw[v], benefit, tq, rec, &cand);
      if (!skip) scanned += (unsigned long long)(q1 - q0);
    }
    const uint64_t cm = ballot(cand);
    if (G == 1) {
      if (l == 0) {
        inm[base >> 5] = (uint32_t)cm;
        inm[(base >> 5) + 1] = (uint32_t)(cm >> 32);
      }
      ncand += __popcll(cm);
    } else {
      uint32_t bits = 0u;  // bit j = vertex base + j (lane j * G)
#pragma unroll
      for (int j = 0; j < VPW; ++j) bits |= (uint32_t)((cm >> (j * G)) & 1ull) << j;
      if (l == 0 && bits) atomicOr(&inm[base >> 5], bits << (base & 31));
      ncand += __popc(bits);
    }
  }
  scanned = wave_sum(scanned);
  if (l == 0) {
    wscan[w] = scanned;
    wcand[w] = ncand;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long ts = 0ull;
    int32_t tc = 0;
    for (int i = 0; i < 4; ++i) {
      ts += wscan[i];
      tc += wcand[i];
    }
    if (tc) atomicAdd(&st->n_cand, tc);
    if (ts) atomicAdd((unsigned long long *)&st->inc_low, ts);
  }
}

// max over 64 lanes of a 64-bit key
__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)x, o, kWave);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(x >> 32), o, kWave);
    const unsigned long long y = ((unsigned long long)hi << 32) | lo;
    x = y > x ? y : x;
  }
  return x;
}

// One 256-thread workgroup per hub vertex: the incident nets are split over 256/G lane groups,
// whose per-block sums are added in LDS.  Runs after k_candidates (which leaves hub bits clear).
template <int G, bool UNIT>
__global__ __launch_bounds__(256) void k_candidates_hub(
    const int32_t *__restrict__ part, const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
    const int32_t *__restrict__ nw, const uint64_t *__restrict__ ns, const int32_t *__restrict__ sumw,
    const int32_t *__restrict__ lockstamp, int32_t locked_stamp, const uint8_t *__restrict__ lock_bytes,
    const int32_t *__restrict__ hubs, int32_t nhubs, int32_t k, int32_t tau_q, uint64_t *__restrict__ rec,
    uint32_t *__restrict__ inm, DevStatus *st, const LoopCtl *lc, Union u) {
  JET_GATE(lc, kPhJet);
  if (lc && !u.lcs) {
    locked_stamp = lc->stamp - 1;
    tau_q = lc->tau_q;
  }
  constexpr int NG = 256 / G;
  __shared__ int32_t cs[NG][8 * G];
  __shared__ int32_t bsum[NG];
  __shared__ unsigned long long wbest[4];
  const int tid = threadIdx.x, gi = tid / G, lg = tid % G;
  int32_t ncand = 0;
  unsigned long long scanned = 0ull;
  for (int32_t hi = blockIdx.x; hi < nhubs; hi += gridDim.x) {  // block-uniform trip count
  const int32_t v = hubs[hi];
  const int32_t s = part[v];
  int32_t ls = locked_stamp, tq = tau_q;
  bool off = false;
  if (u.lcs) {  // the vertex's own hypergraph decides (union)
    const LoopCtl &h = u.lcs[u.vhg[v]];
    off = h.phase != kPhJet;
    ls = h.stamp - 1;
    tq = h.tau_q;
  }
  const bool locked = off || (lock_bytes ? (lock_bytes[v] != 0) : (lockstamp[v] == ls));
  if (locked) {
    if (tid == 0) rec[v] = pack_rec(0, 0xff, s);
    continue;
  }
  int32_t conn[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) conn[j] = 0;
  int32_t benefit = 0;
  if (G == 1) conn_accumulate_strided<G, UNIT>(inc, voff[v] + gi, voff[v + 1], NG, nw, ns, lg, s, conn, benefit);
  else conn_accumulate<G, UNIT>(inc, voff[v] + (int64_t)gi * G, voff[v + 1], (int64_t)NG * G, nw, ns, lg, s, conn,
                                benefit);
#pragma unroll
  for (int j = 0; j < 8; ++j) cs[gi][lg * 8 + j] = conn[j];
  if ((s >> 3) == lg) bsum[gi] = benefit;
  __syncthreads();
  unsigned long long key = 0;
  if (tid < k && tid != s) {
    int32_t tot = 0;
    for (int g = 0; g < NG; ++g) tot += cs[g][tid];
    if (tot > 0) key = ((unsigned long long)(uint32_t)tot << 32) | (uint32_t)(0xffffffffu - (uint32_t)tid);
  }
  key = wave_max_u64(key);
  if (lane_id() == 0) wbest[tid / kWave] = key;
  __syncthreads();
  if (tid == 0) {
    unsigned long long bk = wbest[0];
    for (int w = 1; w < 4; ++w) bk = wbest[w] > bk ? wbest[w] : bk;
    int32_t ben = 0;
    for (int g = 0; g < NG; ++g) ben += bsum[g];
    const int32_t bestc = (int32_t)(uint32_t)(bk >> 32);
    const int32_t bestb = (int32_t)(0xffffffffu - (uint32_t)bk);
    bool cand = false;
    finish_candidate(v, s, bestc, bestb, sumw[v], ben, tq, rec, &cand);
    if (cand) {
      atomicOr(&inm[v >> 5], 1u << (v & 31));
      ncand += 1;
    }
    scanned += (unsigned long long)(voff[v + 1] - voff[v]);
  }
  __syncthreads();  // LDS reused by the next hub
  }  // hub loop
  if (tid == 0) {
    if (ncand) atomicAdd(&st->n_cand, ncand);
    if (scanned) atomicAdd((unsigned long long *)&st->inc_hub, scanned);
  }
}

__global__ void k_export_candidates(const uint64_t *__restrict__ rec, const uint32_t *__restrict__ inm, int32_t n,
                                    int32_t *__restrict__ t, int32_t *__restrict__ g, uint8_t *__restrict__ in_m) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const uint64_t r = rec[v];
  const int32_t tt = rec_target(r);
  t[v] = tt == 0xff ? -1 : tt;
  g[v] = rec_gain(r);
  in_m[v] = inm_bit(inm, (int32_t)v) ? 1 : 0;
}

__global__ void k_import_candidates(const int32_t *__restrict__ part, const int32_t *__restrict__ t,
                                    const int32_t *__restrict__ g, const uint8_t *__restrict__ in_m, int32_t n,
                                    int32_t k, int64_t nwords, uint64_t *__restrict__ rec,
                                    uint32_t *__restrict__ inm, DevStatus *st) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    rec[i] = pack_rec(g[i], t[i] < 0 ? 0xff : t[i], part[i]);
    if (in_m[i] && (t[i] < 0 || t[i] >= k || t[i] == part[i]))
      if (atomicCAS(&st->err, 0, kErrTarget) == 0) st->err_arg = (int32_t)i;
  }
  if (i < nwords) {
    uint32_t wv = 0;
    for (int b = 0; b < 32; ++b) {
      const int64_t v = i * 32 + b;
      if (v < n && in_m[v]) wv |= 1u << b;
    }
    inm[i] = wv;
  }
}

// ------------------------------------------------------------------ afterburner (Algorithm 2)
//
// Replay of the ordered candidates L = e intersect M on net e, decomposed per block: the count of
// block b only changes at events on b (a candidate leaving b or arriving in b), so
//   a departure of v from s earns omega(e) iff  phi_e[s] + A_s(<v) - D_s(<v) == 1
//   an arrival of v in t costs omega(e) iff      phi_e[t] + A_t(<v) - D_t(<v) == 0
// where D_b(<v) / A_b(<v) count candidates before v (in execution order) that leave / enter b.

// Small nets, one wave per chunk.  The whole net is in the wave, so each candidate lane takes the
// net's pins in its source and target blocks (phi_e[s], phi_e[t]) from byte counters of (net of
// the chunk, block) that every pin of the chunk adds one to in the wave's LDS table (a chunk holds
// at most 64 pins, so a byte never carries): no pin count or connectivity word is read.  Only the
// candidates of nets with two or more candidates have predecessors to count; a candidate alone on
// its net skips that step.  The pins clear their counter words again at the end, so the table is
// zero between chunks.
// One chunk of the afterburner for small nets (all lanes of the wave call it; the chunk's
// descriptor, each lane's pin and its net index in the chunk are loaded by the caller).  KW: counter
// words per net (k / 4 rounded up to 16 or 32).
template <int KW>
__device__ __forceinline__ void ab_chunk(int4 cd, int32_t pin, int32_t pj, const int32_t *__restrict__ nw,
                                         const int32_t *__restrict__ part, const uint32_t *__restrict__ inm,
                                         const uint64_t *__restrict__ rec, RgSink rg, int32_t slot,
                                         uint32_t (*cnt)[KW], uint32_t *ncand) {
  const int l = lane_id();
  ChunkLane cl;
  cl.active = l < cd.z;
  cl.q = (int64_t)cd.w + l;
  cl.net = cd.x + pj;
  const int32_t jprev = __shfl_up(pj, 1, kWave);
  cl.starts = ballot(cl.active && (l == 0 || jprev != pj));
  const int32_t v = pin;
  const bool cand = cl.active && inm_bit(inm, v);
  const uint64_t cm = ballot(cand);
  if (cm == 0) return;
  uint32_t khi = 0xffffffffu, klo = 0xffffffffu;
  int32_t s = 0, t = 0, pv = 0;
  if (cl.active) pv = part[v];
  if (cand) {
    const uint64_t r = rec[v];
    khi = order_hi(rec_gain(r));
    klo = (uint32_t)v;
    s = rec_source(r);
    t = rec_target(r);
  }
  if (cl.active) atomicAdd(&cnt[pj][pv >> 2], 1u << (8 * (pv & 3)));
  if (cand) atomicAdd(&ncand[pj], 1u);
  wave_lds_sync();
  int32_t phs = 0, pht = 0;  // pins of the net in s (this one included) and in t
  if (cand) {
    phs = (int32_t)((cnt[pj][s >> 2] >> (8 * (s & 3))) & 0xffu);
    pht = (int32_t)((cnt[pj][t >> 2] >> (8 * (t & 3))) & 0xffu);
  }
  const bool multi = cl.active && ncand[pj] >= 2u;  // this lane's net has two or more candidates
  const uint64_t cm2 = ballot(cand && multi);
  int32_t Ds = 0, As = 0, Dt = 0, At = 0;
  if (cm2) {
    const int32_t st_pack = s | (t << 8);
    // Every candidate of such a net needs the candidates of its net that precede it in the order.
    // Two ways to visit the pairs, chosen per wave: broadcast each of those candidates in turn (one
    // step per candidate), or rotate the lanes of every such net past each other (one step per pin
    // of the longest of them).
    const uint64_t starts = cl.starts;
    const uint64_t upto = (l == 63) ? ~0ull : ((2ull << l) - 1ull);
    const int seg0 = 63 - __clzll((long long)(starts & upto));  // first lane of this lane's net
    const uint64_t later = starts & ~upto;
    const int npins = __popcll(ballot(cl.active));  // outside any branch: a ballot sees active lanes only
    const int seg_end = later ? __ffsll((unsigned long long)later) - 1 : npins;
    const int segn = cl.active ? seg_end - seg0 : 0;
    int maxseg = multi ? segn : 0;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) maxseg = max(maxseg, __shfl_xor(maxseg, o, kWave));
    auto count = [&](uint32_t hj, uint32_t lj, int32_t pk) {
      if (hj < khi || (hj == khi && lj < klo)) {  // non-candidates carry the largest key
        const int32_t sj = pk & 0xff, tj = pk >> 8;
        Ds += sj == s;
        As += tj == s;
        Dt += sj == t;
        At += tj == t;
      }
    };
    if (__popcll(cm2) <= maxseg - 1) {
      uint64_t rem = cm2;
      while (rem) {
        const int j = __ffsll((unsigned long long)rem) - 1;
        rem &= rem - 1;
        const int32_t ej = read_lane_i32(cl.net, j);
        const uint32_t hj = read_lane_u32(khi, j), lj = read_lane_u32(klo, j);
        const int32_t pk = read_lane_i32(st_pack, j);
        if (cand && ej == cl.net) count(hj, lj, pk);
      }
    } else {
      for (int d = 1; d < maxseg; ++d) {
        int r = l - seg0 + d;
        if (r >= segn) r -= segn;
        const int src = d < segn ? seg0 + r : l;
        const uint32_t hj = (uint32_t)__shfl((int)khi, src, kWave), lj = (uint32_t)__shfl((int)klo, src, kWave);
        const int32_t pk = __shfl(st_pack, src, kWave);
        if (cand && d < segn) count(hj, lj, pk);
      }
    }
  }
  if (cand) {
    // v's turn: s empties iff exactly v is left in it; t fills iff it is empty before v arrives
    const int32_t wgt = nw ? nw[cl.net] : 1;
    const bool dep = phs + As - Ds == 1;
    const bool arr = pht + At - Dt == 0;
    const int32_t delta = (dep ? wgt : 0) - (arr ? wgt : 0);
    if (delta) rg_add(rg, slot, v, delta);
  }
  wave_lds_sync();  // every lane has read its counters
  if (cl.active) cnt[pj][pv >> 2] = 0u;  // every nonzero counter word has a pin here
  if (cand) ncand[pj] = 0u;
}

template <int KW>
__global__ __launch_bounds__(256) void k_ab_chunks(const int32_t *__restrict__ pins, const int4 *__restrict__ chunks,
                                                   const uint8_t *__restrict__ pnet, int32_t nchunks,
                                                   const int32_t *__restrict__ nw, const int32_t *__restrict__ part,
                                                   const uint32_t *__restrict__ inm,
                                                   const uint64_t *__restrict__ rec, RgSink rg,
                                                   const LoopCtl *lc, Union u, int32_t xcd) {
  JET_GATE(lc, kPhJet);
  // union: only the chunks of the hypergraphs in their Jet phase
  const ActList *AL = u.lcs ? &u.act[kActJet] : nullptr;
  const int32_t nvc = AL ? AL->cpref[AL->cnt] : nchunks;
  __shared__ uint32_t cnt[4][64][KW];
  __shared__ uint32_t ncand[4][64];
  const int l = lane_id();
  const int w = threadIdx.x / kWave;
  const int32_t wid = blockIdx.x * 4 + w, nwv = gridDim.x * 4;
  for (int x = 0; x < 64 * KW; x += kWave) (&cnt[w][0][0])[x + l] = 0u;
  ncand[w][l] = 0u;
  wave_lds_sync();
  auto fetch = [&](int32_t cc, int4 &d, int32_t &p, int32_t &j) {
    d = cc < nvc ? chunks[AL ? act_chunk(*AL, u.hch0, cc) : cc] : make_int4(0, 0, 0, 0);
    p = 0;
    j = -1;
    if (l < d.z) {
      const int64_t q = (int64_t)d.w + l;
      j = pnet[q];
      p = pins[q];
    }
  };
  // with xcd set, the workgroups of one XCD (round robin by workgroup) walk one contiguous eighth of
  // the chunks, so the records of neighbouring pins are fetched into that XCD's L2 only
  int32_t c0 = wid, cend = nvc, cstep = nwv;
  if (xcd && !AL && gridDim.x % 8 == 0) {
    const int32_t per = (nvc + 7) / 8, x = (int32_t)(blockIdx.x % 8);
    c0 = x * per + (int32_t)(blockIdx.x / 8) * 4 + w;
    cend = min(nvc, (x + 1) * per);
    cstep = (int32_t)(gridDim.x / 8) * 4;
  }
  int4 cd;
  int32_t pin, pj;
  fetch(c0 < cend ? c0 : nvc, cd, pin, pj);
  for (int32_t c = c0; c < cend; c += cstep) {  // wave-uniform trip count
    int4 ncd;
    int32_t npin, npj;
    fetch(c + cstep < cend ? c + cstep : nvc, ncd, npin, npj);  // the next chunk's loads overlap this chunk's work
    ab_chunk<KW>(cd, pin, pj, nw, part, inm, rec, rg, wid, cnt[w], ncand[w]);
    cd = ncd;
    pin = npin;
    pj = npj;
  }
}

enum : uint8_t { kNone = 0, kInert = 1, kArrOnly = 2, kDepOnly = 3, kMixed = 4 };
constexpr int kAbU = 4;  // slices of a net whose loads one thread keeps in flight in the first pass
// interleaved blocks: prefix sums while (blocks x padded events) <= kScanMixed x events, else walks
constexpr int kScanMixed = 24;

// Larger nets, one block per net.  Per block b of the net, with D = candidates leaving b and
// A = candidates entering b:
//   phi_e[b] > D            -> some pin of b stays: the count never reaches 0, no event fires
//   phi_e[b] = 0 (so D = 0) -> only the first arrival (smallest key) finds b empty
//   phi_e[b] = D, A = 0     -> only the last departure (largest key) empties b
//   phi_e[b] = D, A > 0     -> departures and arrivals interleave: walk b's events in key order
// The candidates live in LDS when they fit; otherwise the pins are streamed again and only the
// candidates touching interleaved blocks are kept (at most CAP of them).
template <int THREADS, int CAP, int NW, typename T>
__global__ __launch_bounds__(THREADS) void k_ab_nets(const int64_t *__restrict__ off,
                                                     const int32_t *__restrict__ pins,
                                                     const int32_t *__restrict__ nets,
                                                     const int32_t *__restrict__ nw,
                                                     const uint32_t *__restrict__ inm,
                                                     const uint64_t *__restrict__ rec,
                                                     const T *__restrict__ phi,
                                                     const uint64_t *__restrict__ ns, int32_t k,
                                                     RgSink rg, DevStatus *st,
                                                     int2 *__restrict__ ovf_list, const LoopCtl *lc, Union u) {
  JET_GATE(lc, kPhJet);
  if (u.lcs && u.lcs[u.nhg[nets[blockIdx.x]]].phase != kPhJet) return;  // union: a net of an idle hypergraph
  __shared__ int32_t D[kMaxK], A[kMaxK], P0[kMaxK];
  __shared__ uint8_t cls[kMaxK];
  __shared__ unsigned long long bestdep[kMaxK], bestarr[kMaxK];
  __shared__ unsigned long long Lkey[CAP];
  __shared__ uint16_t Lst[CAP];
  __shared__ uint8_t fdep[CAP], farr[CAP];
  __shared__ int32_t cntL, cntX, flags, nmix;
  __shared__ int32_t scan_sm[THREADS / kWave + 1];
  const int tid = threadIdx.x;
  const int32_t e = nets[blockIdx.x];
  const int64_t q0 = off[e], q1 = off[e + 1];
  const int32_t wgt = nw ? nw[e] : 1;
  for (int b = tid; b < k; b += THREADS) {
    D[b] = 0;
    A[b] = 0;
  }
  if (tid == 0) {
    cntL = 0;
    cntX = 0;
    flags = 0;
    nmix = 0;
  }
  __syncthreads();
  // pass 1: histograms, candidates into LDS while they fit.  kAbU slices of the net at a time, each
  // level of their dependent loads (pin, candidate bit, record) issued for all before any is used.
  for (int64_t qb = q0; qb < q1; qb += THREADS * kAbU) {
    int32_t v[kAbU];
    bool cand[kAbU];
    uint64_t r[kAbU];
#pragma unroll
    for (int u = 0; u < kAbU; ++u) {
      const int64_t q = qb + u * THREADS + tid;
      v[u] = q < q1 ? pins[q] : -1;
    }
#pragma unroll
    for (int u = 0; u < kAbU; ++u) cand[u] = v[u] >= 0 && inm_bit(inm, v[u]);
#pragma unroll
    for (int u = 0; u < kAbU; ++u) r[u] = cand[u] ? rec[v[u]] : 0ull;
#pragma unroll
    for (int u = 0; u < kAbU; ++u) {
      const uint64_t cm = ballot(cand[u]);
      int32_t base = 0;
      if (cm) {
        if (lane_id() == 0) base = atomicAdd(&cntL, __popcll(cm));
        base = __shfl(base, 0, kWave);
      }
      if (cand[u]) {
        const int32_t s = rec_source(r[u]), t = rec_target(r[u]);
        atomicAdd(&D[s], 1);
        atomicAdd(&A[t], 1);
        const int32_t pos = base + rank_below(cm);
        if (pos < CAP) {
          Lkey[pos] = order_key(rec_gain(r[u]), v[u]);
          Lst[pos] = (uint16_t)(s | (t << 8));
        }
      }
    }
  }
  __syncthreads();
  for (int b = tid; b < k; b += THREADS) {
    const int32_t d = D[b], a = A[b];
    uint8_t cb = kNone;
    if (d + a > 0) {
      // count of b: 0 / 1 from the connectivity words; read exactly only if it can equal d >= 2
      const uint64_t *nse = ns + (int64_t)e * (2 * NW);
      const bool nz = (nse[b >> 6] >> (b & 63)) & 1ull, one = (nse[NW + (b >> 6)] >> (b & 63)) & 1ull;
      const int32_t p0 = !nz ? 0 : one ? 1 : d < 2 ? 2 : (int32_t)phi[(int64_t)e * k + b];
      P0[b] = p0;
      if (p0 > d) cb = kInert;
      else if (d == 0) cb = kArrOnly;
      else if (a == 0) cb = kDepOnly;
      else cb = kMixed;
    }
    cls[b] = cb;
    bestdep[b] = 0ull;
    bestarr[b] = ~0ull;
    if (cb == kArrOnly || cb == kDepOnly) atomicOr(&flags, 1);
    if (cb == kMixed) {
      atomicOr(&flags, 2);
      atomicAdd(&nmix, 1);
    }
  }
  __syncthreads();
  const int32_t fl = flags;
  if (fl == 0) return;
  const int32_t total = cntL;
  const bool in_lds = total <= CAP;
  // pass 2: extreme keys per block; interleaved events when the candidates did not fit
  if (in_lds) {
    for (int32_t i = tid; i < total; i += THREADS) {
      const unsigned long long key = Lkey[i];
      const int32_t s = Lst[i] & 0xff, t = Lst[i] >> 8;
      if (cls[s] == kDepOnly) atomicMax(&bestdep[s], key);
      if (cls[t] == kArrOnly) atomicMin(&bestarr[t], key);
    }
  } else {
    for (int64_t qb = q0; qb < q1; qb += THREADS) {
      const int64_t q = qb + tid;
      bool cand = false;
      int32_t v = 0;
      if (q < q1) {
        v = pins[q];
        cand = inm_bit(inm, v);
      }
      int32_t s = 0, t = 0;
      unsigned long long key = 0;
      bool mixed = false;
      if (cand) {
        const uint64_t r = rec[v];
        s = rec_source(r);
        t = rec_target(r);
        key = order_key(rec_gain(r), v);
        if (cls[s] == kDepOnly) atomicMax(&bestdep[s], key);
        if (cls[t] == kArrOnly) atomicMin(&bestarr[t], key);
        mixed = cls[s] == kMixed || cls[t] == kMixed;
      }
      const uint64_t mm = ballot(mixed);
      int32_t base = 0;
      if (mm) {
        if (lane_id() == 0) base = atomicAdd(&cntX, __popcll(mm));
        base = __shfl(base, 0, kWave);
      }
      if (mixed) {
        const int32_t pos = base + rank_below(mm);
        if (pos < CAP) {
          Lkey[pos] = key;
          Lst[pos] = (uint16_t)(s | (t << 8));
        }
      }
    }
  }
  __syncthreads();
  for (int b = tid; b < k; b += THREADS) {
    if (cls[b] == kDepOnly) rg_add(rg, blockIdx.x, (int32_t)(uint32_t)bestdep[b], wgt);
    if (cls[b] == kArrOnly) rg_add(rg, blockIdx.x, (int32_t)(uint32_t)bestarr[b], -wgt);
  }
  if (!(fl & 2)) return;
  const int32_t cnt = in_lds ? total : cntX;
  if (cnt > CAP) {  // too many interleaved events for LDS: resolved by k_ab_overflow
    if (tid == 0) {
      if (ovf_list) ovf_list[atomicAdd(&st->n_ovf, 1)] = make_int2(blockIdx.x, e);
      else if (atomicCAS(&st->err, 0, kErrMixedOverflow) == 0) st->err_arg = e;
    }
    return;
  }
  // bitonic sort of (key, source|target) by key
  int32_t N = 1;
  while (N < cnt) N <<= 1;
  for (int32_t i = cnt + tid; i < N; i += THREADS) {
    Lkey[i] = ~0ull;
    Lst[i] = 0;
  }
  for (int32_t i = tid; i < N; i += THREADS) {
    fdep[i] = 0;
    farr[i] = 0;
  }
  __syncthreads();
  for (int32_t size = 2; size <= N; size <<= 1) {
    for (int32_t stride = size >> 1; stride > 0; stride >>= 1) {
      for (int32_t i = tid; i < N / 2; i += THREADS) {
        const int32_t lo = 2 * i - (i & (stride - 1));
        const int32_t hi = lo + stride;
        const bool up = (lo & size) == 0;
        const unsigned long long x = Lkey[lo], y = Lkey[hi];
        if ((x > y) == up) {
          Lkey[lo] = y;
          Lkey[hi] = x;
          const uint16_t tmp = Lst[lo];
          Lst[lo] = Lst[hi];
          Lst[hi] = tmp;
        }
      }
      __syncthreads();
    }
  }
  // The count of an interleaved block b before each event (execution order) is P0[b] plus the
  // block's steps so far (+1 arrival, -1 departure).  Few such blocks: a block-wide prefix sum per
  // block; many: one thread per block walks all events.
  if ((int64_t)nmix * ((cnt + THREADS - 1) / THREADS) * THREADS <= (int64_t)kScanMixed * cnt) {
    for (int b = 0; b < k; ++b) {  // block-uniform: cls is in LDS
      if (cls[b] != kMixed) continue;
      int32_t carry = P0[b];
      for (int32_t i0 = 0; i0 < cnt; i0 += THREADS) {
        const int32_t i = i0 + tid;
        bool dep = false, arr = false;
        if (i < cnt) {
          dep = (Lst[i] & 0xff) == b;
          arr = (Lst[i] >> 8) == b;
        }
        int32_t tot;
        const int32_t before = carry + block_excl_scan<THREADS>((int32_t)arr - (int32_t)dep, scan_sm, &tot);
        if (dep && before == 1) fdep[i] = 1;
        if (arr && before == 0) farr[i] = 1;
        carry += tot;
      }
    }
  } else {
    for (int b = tid; b < k; b += THREADS) {
      if (cls[b] != kMixed) continue;
      int32_t cur = P0[b];
      for (int32_t i = 0; i < cnt; ++i) {
        const int32_t s = Lst[i] & 0xff, t = Lst[i] >> 8;
        if (s == b) {
          if (cur == 1) fdep[i] = 1;
          --cur;
        }
        if (t == b) {
          if (cur == 0) farr[i] = 1;
          ++cur;
        }
      }
    }
  }
  __syncthreads();
  for (int32_t i = tid; i < cnt; i += THREADS) {
    const int32_t s = Lst[i] & 0xff, t = Lst[i] >> 8;
    int32_t delta = 0;
    if (fdep[i] && cls[s] == kMixed) delta += wgt;
    if (farr[i] && cls[t] == kMixed) delta -= wgt;
    if (delta) rg_add(rg, blockIdx.x, (int32_t)(uint32_t)Lkey[i], delta);
  }
}

// ------------------------------------------------------------------ kept moves and locks

// Compaction helper: each block takes tiles of kSelBlock * kCompactPer vertices, kCompactPer per
// thread (strided, so the loads coalesce), each predicate evaluated once and kept in registers;
// one block scan and one atomic per tile reserve the slots (list order does not matter: applying
// a move list is order independent).
constexpr int kSelBlock = 256;
constexpr int kCompactPer = 8;

struct NoPost {
  __device__ void operator()(const int64_t *, uint32_t) const {}
};

// post(sub, mask): called by every thread of the block once the tile's predicates are evaluated,
// with the first vertex of each of its kCompactPer sub-tiles (n for a sub-tile past the end) and
// the thread's mask of selected sub-tile vertices.
template <typename Pred, typename Emit, typename Post = NoPost>
__device__ __forceinline__ void block_compact(int64_t n, Pred pred, Emit emit, DevStatus *st, int32_t *bigmv,
                                              const ActList *AL = nullptr, const int32_t *ht0 = nullptr,
                                              Post post = Post()) {
  __shared__ int32_t sm[kSelBlock / kWave + 1];
  __shared__ int32_t s_base;
  __shared__ unsigned long long s_deg;
  const int tid = threadIdx.x;
  if (tid == 0) s_deg = 0ull;
  __syncthreads();
  unsigned long long deg = 0ull;
  constexpr int64_t kTile = (int64_t)kSelBlock * kCompactPer;
  static_assert(kSelBlock == kUnionTile, "a union's sub-tiles are its hypergraphs' tiles");
  // union: virtual vertices = the tiles of the listed hypergraphs, each sub-tile j mapped on its own
  const int32_t ntv = AL ? AL->tpref[AL->cnt] : 0;
  const int64_t nv = AL ? (int64_t)ntv * kUnionTile : n;
  const int64_t ntiles = (nv + kTile - 1) / kTile;
  __shared__ int64_t s_sb[kCompactPer];
  auto sub_base = [&](int64_t tile, int j) -> int64_t {
    if (!AL) return tile * kTile + j * kSelBlock;
    const int64_t t = tile * kCompactPer + j;
    return t < ntv ? act_tile_base(*AL, ht0, (int32_t)t) : n;
  };
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {  // block-uniform trip count
    uint32_t mask = 0;
    int32_t cnt = 0;
    int64_t sb[kCompactPer], vv[kCompactPer];
    if (AL) {  // one search per sub-tile by the first wave, shared by the block
      if (tid < kWave)
        for (int j = 0; j < kCompactPer; ++j) {
          const int64_t b = sub_base(tile, j);
          if (tid == 0) s_sb[j] = b;
        }
      __syncthreads();
    }
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) {
      sb[j] = AL ? s_sb[j] : sub_base(tile, j);
      const int64_t v = sb[j] < n ? sb[j] + tid : n;
      vv[j] = v;
      if (v < n && pred(v)) {
        mask |= 1u << j;
        ++cnt;
      }
    }
    int32_t tot;
    const int32_t rk = block_excl_scan<kSelBlock>(cnt, sm, &tot);  // ends with a barrier
    post(sb, mask);
    if (tot == 0) continue;  // block-uniform
    if (tid == 0) s_base = atomicAdd(&st->n_moves, tot);
    __syncthreads();
    int32_t pos = s_base + rk;
#pragma unroll
    for (int j = 0; j < kCompactPer; ++j) {
      const bool mv = (mask >> j) & 1u;
      unsigned long long d = 0ull;
      if (mv) d = emit(vv[j], pos);
      deg += d;
      push_big_move(mv && d > (unsigned long long)kLaneDegree, pos, st, bigmv);
      pos += mv ? 1 : 0;
    }
    __syncthreads();  // s_base is rewritten by the next tile
  }
  deg = wave_sum(deg);
  if (lane_id() == 0 && deg) atomicAdd(&s_deg, deg);
  __syncthreads();
  if (tid == 0 && s_deg) atomicAdd((unsigned long long *)&st->mv_inc, s_deg);
}

__global__ __launch_bounds__(kSelBlock) void k_select_moves(const int32_t *__restrict__ part,
                                                            uint32_t *__restrict__ inm,
                                                            const uint64_t *__restrict__ rec,
                                                            int32_t *__restrict__ rg,
                                                            const int32_t *__restrict__ vw, int32_t n, int32_t stamp,
                                                            int32_t *__restrict__ lockstamp,
                                                            int4 *__restrict__ moves, uint8_t *__restrict__ mvto,
                                                            const int64_t *__restrict__ voff, DevStatus *st,
                                                            int32_t *__restrict__ bigmv, const LoopCtl *lc,
                                                            Union u) {
  JET_GATE(lc, kPhJet);
  if (lc && !u.lcs) stamp = lc->stamp;
  // recomputed gains start from zero in the next iteration: each candidate's entry is cleared here
  auto pred = [&](int64_t v) {
    if (!inm_bit(inm, (int32_t)v)) return false;
    const int32_t g = rg[v];
    rg[v] = 0;
    return g > 0;
  };
  auto emit = [&](int64_t v, int32_t pos) -> unsigned long long {
    const int32_t t = rec_target(rec[v]);
    moves[pos] = make_int4((int32_t)v, part[v], t, vw ? vw[v] : 1);
    mvto[v] = (uint8_t)t;
    if (u.lcs) {  // union: the hypergraph's own stamp (its move count is added per sub-tile)
      lockstamp[v] = u.lcs[u.vhg[v]].stamp;
    } else {
      lockstamp[v] = stamp;
    }
    return (unsigned long long)(voff[v + 1] - voff[v]);
  };
  // the candidate bits of the walked tiles are cleared once read, so a hypergraph that leaves its
  // Jet phase (union) leaves none behind for the kernels that walk every net
  // union: the moves of every sub-tile (one hypergraph's vertices) counted with one atomic
  __shared__ int32_t s_cnt[kSelBlock / kWave][kCompactPer];
  auto clear_bits = [&](const int64_t *sb, uint32_t mask) {
    if (u.lcs) {
      const int w = threadIdx.x / kWave;
#pragma unroll
      for (int j = 0; j < kCompactPer; ++j) {
        const int32_t c = __popcll(ballot((mask >> j) & 1u));
        if (lane_id() == 0) s_cnt[w][j] = c;
      }
      __syncthreads();
      if (threadIdx.x < kCompactPer && sb[threadIdx.x] < n) {
        int32_t c = 0;
        for (int x = 0; x < kSelBlock / kWave; ++x) c += s_cnt[x][threadIdx.x];
        if (c) atomicAdd(&st->hmoves[u.vhg[sb[threadIdx.x]]], c);
      }
      __syncthreads();
    }
    if (threadIdx.x < kCompactPer * (kSelBlock / 32)) {
      const int j = threadIdx.x / (kSelBlock / 32), x = threadIdx.x % (kSelBlock / 32);
      if (sb[j] < n) inm[sb[j] / 32 + x] = 0u;
    }
  };
  if (u.lcs) block_compact(n, pred, emit, st, bigmv, &u.act[kActJet], u.ht0, clear_bits);
  else block_compact(n, pred, emit, st, bigmv, nullptr, nullptr, clear_bits);
}

__global__ __launch_bounds__(kSelBlock) void k_diff_moves(const int32_t *__restrict__ part,
                                                          const int32_t *__restrict__ target,
                                                          const int32_t *__restrict__ vw, int32_t n,
                                                          int4 *__restrict__ moves, uint8_t *__restrict__ mvto,
                                                          const int64_t *__restrict__ voff, DevStatus *st,
                                                          int32_t *__restrict__ bigmv, const LoopCtl *lc,
                                                          Union u) {
  JET_GATE(lc, kPhRoll);
  // union: only the hypergraphs whose round ended roll back
  auto pred = [&](int64_t v) {
    return part[v] != target[v] && (!u.lcs || u.lcs[u.vhg[v]].phase == kPhRoll);
  };
  auto emit = [&](int64_t v, int32_t pos) -> unsigned long long {
    moves[pos] = make_int4((int32_t)v, part[v], target[v], vw ? vw[v] : 1);
    mvto[v] = (uint8_t)target[v];
    return (unsigned long long)(voff[v + 1] - voff[v]);
  };
  if (u.lcs) block_compact(n, pred, emit, st, bigmv, &u.act[kActRoll], u.ht0);
  else block_compact(n, pred, emit, st, bigmv);
}

// ------------------------------------------------------------------ applying a move list
//
// Two ways to bring pin counts, connectivity words, block weights and the metric up to date; the
// device picks one from the number of listed moves (no host round trip):
//
// Many moves (>= n / kNetCentricDivisor): net-centric.  Every net is owned by one wave (small
// nets, chunked) or one workgroup (larger nets), which recounts the blocks its moving pins leave
// and enter and rewrites those counts, its connectivity words and its metric contribution with
// plain stores; the partition entries are then updated from the move list.
//
// Few moves: vertex-centric.  Each move walks its incident nets and moves the counts by +-1 with
// atomics.  The counter values of one (net, block) form a sequence of +-1 steps in the atomics'
// order (never below zero), and every atomic sees exactly one step, so a 0->1 step adds w(e) and a
// 1->0 step removes it (the sum telescopes to the exact change), and the bits [count > 0] (flips at
// 0<->1) and [count == 1] (flips at 0<->1 and 1<->2) are kept by atomic XOR toggles, which commute.
// A move with many incident nets gets a whole block whose threads stride over its nets.

// divisor 0: always vertex-centric; otherwise net-centric when the moves' incident nets, times the
// divisor, reach the number of pins
__device__ __forceinline__ bool net_centric(const DevStatus *st, int64_t p, int32_t divisor) {
  return divisor > 0 && st->mv_inc * divisor >= p;
}

// One +-1 step on (net, block) given the value the atomic returned.
template <int NW>
__device__ __forceinline__ int64_t after_step(int32_t old, bool up, int32_t b, int32_t w,
                                              unsigned long long *__restrict__ nse) {
  int64_t dk = 0;
  const unsigned long long bit = 1ull << (b & 63);
  if (up) {  // old -> old + 1
    if (old == 0) {
      dk = w;
      atomicXor(&nse[b >> 6], bit);
    }
    if (old <= 1) atomicXor(&nse[NW + (b >> 6)], bit);
  } else {   // old -> old - 1
    if (old == 1) {
      dk = -w;
      atomicXor(&nse[b >> 6], bit);
    }
    if (old <= 2) atomicXor(&nse[NW + (b >> 6)], bit);
  }
  return dk;
}

// The incident nets q0, q0 + step, ... < q1 of one move s -> t; four nets per round so that eight
// counter atomics are in flight before any returned value is used.
template <int NW, typename T>
__device__ __forceinline__ int64_t apply_nets_of_move(const int32_t *__restrict__ inc, int64_t q0, int64_t q1,
                                                      int64_t step, int32_t s, int32_t t, int32_t k,
                                                      const int32_t *__restrict__ nw, T *__restrict__ phi,
                                                      uint64_t *__restrict__ ns) {
  int64_t dk = 0;
  int64_t q = q0;
  for (; q + 3 * step < q1; q += 4 * step) {
    int32_t e[4], os[4], ot[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) e[i] = inc[q + i * step];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      os[i] = phi_atomic_add(phi, (int64_t)e[i] * k + s, -1);
      ot[i] = phi_atomic_add(phi, (int64_t)e[i] * k + t, 1);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int32_t w = nw ? nw[e[i]] : 1;
      unsigned long long *nse = (unsigned long long *)(ns + (int64_t)e[i] * (2 * NW));
      dk += after_step<NW>(os[i], false, s, w, nse);
      dk += after_step<NW>(ot[i], true, t, w, nse);
    }
  }
  for (; q < q1; q += step) {
    const int32_t e = inc[q];
    const int32_t os = phi_atomic_add(phi, (int64_t)e * k + s, -1);
    const int32_t ot = phi_atomic_add(phi, (int64_t)e * k + t, 1);
    const int32_t w = nw ? nw[e] : 1;
    unsigned long long *nse = (unsigned long long *)(ns + (int64_t)e * (2 * NW));
    dk += after_step<NW>(os, false, s, w, nse);
    dk += after_step<NW>(ot, true, t, w, nse);
  }
  return dk;
}

// Partition entries and block weights from the move list; in the vertex-centric case also the
// incident nets of every move.
constexpr int kApplyLanes = 8;
template <int NW, typename T>
__global__ __launch_bounds__(256) void k_apply(const int4 *__restrict__ moves, const int64_t *__restrict__ voff,
                                               const int32_t *__restrict__ inc, const int32_t *__restrict__ nw,
                                               int64_t p, int32_t k, int32_t *__restrict__ part,
                                               T *__restrict__ phi, uint64_t *__restrict__ ns,
                                               uint8_t *__restrict__ mvto, const int32_t *__restrict__ bigmv,
                                               int32_t divisor, DevStatus *st, const LoopCtl *lc, int32_t want,
                                               Union u, int32_t xcd) {
  JET_GATE(lc, want);
  __shared__ unsigned long long dw[kMaxK];
  __shared__ int32_t dc[kMaxK];
  __shared__ int64_t sdk[256 / kWave];
  for (int b = threadIdx.x; b < k; b += blockDim.x) {
    dw[b] = 0;
    dc[b] = 0;
  }
  __syncthreads();
  const int32_t cnt = st->n_moves;
  const bool by_vertex = !net_centric(st, p, divisor);
  int64_t dk = 0;
  // kApplyLanes lanes per move, each taking every kApplyLanes-th incident net of a move with few
  // nets, so a move's chain of dependent atomics is that many times shorter.  A union gives every
  // workgroup a contiguous range of the list (moves are listed by vertex, so by hypergraph): the
  // moves of the range's first hypergraph ("home") add into the workgroup's sums, the others (a
  // range crossing into the next hypergraph) straight into their segments.
  const int lg = threadIdx.x % kApplyLanes;
  const bool un = u.vhg != nullptr;
  int64_t i0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kApplyLanes, i1 = cnt;
  int64_t istep = (int64_t)gridDim.x * blockDim.x / kApplyLanes;
  int32_t home = 0;
  if (un) {
    const int64_t per = ((int64_t)cnt + gridDim.x - 1) / gridDim.x;
    const int64_t first = (int64_t)blockIdx.x * per;
    i0 = first + threadIdx.x / kApplyLanes;
    i1 = first + per < cnt ? first + per : cnt;
    istep = blockDim.x / kApplyLanes;
    if (first < cnt) home = u.vhg[moves[first].x];
  } else if (xcd && gridDim.x % 8 == 0) {
    // the workgroups of one XCD (round robin by workgroup) take one contiguous eighth of the list
    // (moves are listed by vertex: neighbouring moves share nets' lines in that XCD's L2)
    const int64_t span = blockDim.x / kApplyLanes, steps = (cnt + span - 1) / span, per = (steps + 7) / 8;
    const int64_t x = blockIdx.x % 8;
    i0 = (x * per + blockIdx.x / 8) * span + threadIdx.x / kApplyLanes;
    i1 = min((int64_t)cnt, (x + 1) * per * span);
    istep = (int64_t)(gridDim.x / 8) * span;
  }
  for (int64_t i = i0; i < i1; i += istep) {
    const int4 mv = moves[i];
    const int32_t hg = un ? (int32_t)u.vhg[mv.x] : 0;
    const bool local = !un || hg == home;
    if (lg == 0) {
      part[mv.x] = mv.z;
      mvto[mv.x] = 0xff;
      if (local) {
        atomicAdd(&dw[mv.y], (unsigned long long)(-(int64_t)mv.w));
        atomicAdd(&dw[mv.z], (unsigned long long)mv.w);
        atomicAdd(&dc[mv.y], -1);
        atomicAdd(&dc[mv.z], 1);
      } else {  // union: another hypergraph's segments
        const int64_t sg = (int64_t)hg * k;
        atomicAdd((unsigned long long *)&st->bw[sg + mv.y], (unsigned long long)(-(int64_t)mv.w));
        atomicAdd((unsigned long long *)&st->bw[sg + mv.z], (unsigned long long)mv.w);
        atomicAdd(&st->bcnt[sg + mv.y], -1);
        atomicAdd(&st->bcnt[sg + mv.z], 1);
      }
    }
    if (by_vertex) {
      const int64_t q0 = voff[mv.x], q1 = voff[mv.x + 1];
      if (q1 - q0 <= kLaneDegree) {
        const int64_t d = apply_nets_of_move<NW>(inc, q0 + lg, q1, kApplyLanes, mv.y, mv.z, k, nw, phi, ns);
        if (local) dk += d;
        else add_km1_hg(st, hg, d);
      }
    }
  }
  if (by_vertex) {
    // high-degree moves: an equal share of the grid each (several blocks per move while there are
    // fewer such moves than blocks), the threads of the share striding over the move's nets
    const int32_t nb = st->n_bigmv;
    if (nb > 0 && nb <= (int32_t)gridDim.x) {
      const int32_t per = (int32_t)gridDim.x / nb;
      const int32_t j = (int32_t)blockIdx.x / per, sub = (int32_t)blockIdx.x % per;
      if (j < nb) {
        const int4 mv = moves[bigmv[j]];
        const int64_t q0 = voff[mv.x], q1 = voff[mv.x + 1];
        const int64_t d = apply_nets_of_move<NW>(inc, q0 + (int64_t)sub * blockDim.x + threadIdx.x, q1,
                                                 (int64_t)per * blockDim.x, mv.y, mv.z, k, nw, phi, ns);
        if (u.vhg) add_km1_hg(st, u.vhg[mv.x], d);
        else dk += d;
      }
    } else {
      for (int32_t j = blockIdx.x; j < nb; j += gridDim.x) {
        const int4 mv = moves[bigmv[j]];
        const int64_t q0 = voff[mv.x], q1 = voff[mv.x + 1];
        const int64_t d = apply_nets_of_move<NW>(inc, q0 + threadIdx.x, q1, blockDim.x, mv.y, mv.z, k, nw, phi, ns);
        if (u.vhg) add_km1_hg(st, u.vhg[mv.x], d);
        else dk += d;
      }
    }
  }
  dk = wave_sum(dk);
  if (lane_id() == 0) sdk[threadIdx.x / kWave] = dk;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t tt = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) tt += sdk[w];
    if (un) add_km1_hg(st, home, tt);
    else add_km1(st, blockIdx.x, tt);
  }
  const int64_t sg0 = (int64_t)home * k;  // segments of the home hypergraph (the blocks for one)
  for (int b = threadIdx.x; b < k; b += blockDim.x) {
    if (dw[b]) atomicAdd((unsigned long long *)&st->bw[sg0 + b], dw[b]);
    if (dc[b]) atomicAdd(&st->bcnt[sg0 + b], dc[b]);
  }
}

// Net-centric, small nets: one wave per chunk.  Each pin's new block is its move target or its
// block; per net the new connectivity words come from LDS OR-accumulation (a second OR collects
// blocks seen twice), and each moving pin rewrites the counts of the two blocks it touches from
// the pins of its net now in them (no count is read): every pin adds one to a byte counter of
// (its net, its new block) in the wave's LDS table, and a moving pin reads the two it needs.  A
// chunk holds at most 64 pins, so a byte never carries; the pins clear their counter words again
// once the chunk is done, so the table is zero between chunks.  A wave takes kApplyU chunks at a time and
// issues each level of their dependent loads (descriptor, pin, move target, block and words) for
// all of them before using any, so the latency chain is paid once per group.
constexpr int kApplyU = 4;

template <int NW, typename T>
__global__ __launch_bounds__(256) void k_apply_chunks(const int64_t *__restrict__ off,
                                                      const int32_t *__restrict__ pins,
                                                      const int4 *__restrict__ chunks,
                                                      const uint8_t *__restrict__ pnet, int32_t nchunks,
                                                      const int32_t *__restrict__ nw,
                                                      const int32_t *__restrict__ part,
                                                      const uint8_t *__restrict__ mvto, int64_t p, int32_t k,
                                                      T *__restrict__ phi, uint64_t *__restrict__ ns,
                                                      int32_t divisor, DevStatus *st, const LoopCtl *lc,
                                                      int32_t want, Union un, int32_t xcd) {
  JET_GATE(lc, want);
  constexpr int U = kApplyU;
  __shared__ unsigned long long once[4][64][NW], twice[4][64][NW];
  __shared__ uint32_t cnt[4][64][16 * NW];  // per wave: byte counters of (chunk net, block)
  if (!net_centric(st, p, divisor)) return;
  const int w = threadIdx.x / kWave, l = lane_id();
  for (int x = 0; x < 64 * 16 * NW; x += kWave) (&cnt[w][0][0])[x + l] = 0u;
  const int32_t wid = blockIdx.x * 4 + w, nwaves = gridDim.x * 4;
  int64_t dk = 0;
  // each wave walks its own groups of chunks; the LDS slots are private to the wave.  With xcd set,
  // the workgroups of one XCD (round robin by workgroup) take one contiguous eighth of the chunks
  // (ranges aligned to groups of U chunks).
  int32_t cstart = wid * U, cend = nchunks, cstep = nwaves * U;
  if (xcd && !un.vhg && gridDim.x % 8 == 0) {
    const int32_t span = 4 * U, steps = (nchunks + span - 1) / span, per = (steps + 7) / 8;
    const int32_t x = (int32_t)(blockIdx.x % 8);
    cstart = (x * per + (int32_t)(blockIdx.x / 8)) * span + w * U;
    cend = min(nchunks, (x + 1) * per * span);
    cstep = (int32_t)(gridDim.x / 8) * span;
  }
  for (int32_t c0 = cstart; c0 < cend; c0 += cstep) {  // wave-uniform trip count
    int4 cd[U];
#pragma unroll
    for (int u = 0; u < U; ++u) cd[u] = c0 + u < cend ? chunks[c0 + u] : make_int4(0, 0, 0, 0);
    int32_t v[U], j[U];
    bool act[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      act[u] = l < cd[u].z;
      v[u] = 0;
      j[u] = 0;
      if (act[u]) {
        const int64_t q = (int64_t)cd[u].w + l;
        j[u] = pnet[q];
        v[u] = pins[q];
      }
    }
    uint8_t mt[U];
#pragma unroll
    for (int u = 0; u < U; ++u) mt[u] = act[u] ? mvto[v[u]] : (uint8_t)0xff;
    uint64_t movers[U];
#pragma unroll
    for (int u = 0; u < U; ++u) movers[u] = ballot(mt[u] != 0xff);
    // blocks of the pins and connectivity words of the nets in chunks with movers
    int32_t ob[U], nb[U];
    uint64_t wd[U][2 * NW];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ob[u] = 0;
      if (movers[u] && act[u]) ob[u] = part[v[u]];
#pragma unroll
      for (int x = 0; x < 2 * NW; ++x) wd[u][x] = 0ull;
      if (movers[u] && l < cd[u].y) {
        const uint64_t *nse = ns + (int64_t)(cd[u].x + l) * (2 * NW);
#pragma unroll
        for (int x = 0; x < 2 * NW; ++x) wd[u][x] = nse[x];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) nb[u] = mt[u] != 0xff ? (int32_t)mt[u] : ob[u];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (!movers[u]) continue;  // wave-uniform
      const bool moved = mt[u] != 0xff;
#pragma unroll
      for (int x = 0; x < NW; ++x) {
        once[w][l][x] = 0ull;
        twice[w][l][x] = 0ull;
      }
      wave_lds_sync();
      if (act[u]) {
        const unsigned long long bit = 1ull << (nb[u] & 63);
        const unsigned long long old = atomicOr(&once[w][j[u]][nb[u] >> 6], bit);
        if (old & bit) atomicOr(&twice[w][j[u]][nb[u] >> 6], bit);
        atomicAdd(&cnt[w][j[u]][nb[u] >> 2], 1u << (8 * (nb[u] & 3)));
      }
      wave_lds_sync();
      // The whole net is in the wave, so the new counts of the two blocks a moving pin touches
      // are those of its net's counters: pins of the net whose new block is that block.
      if (moved) {
        const int32_t co = (cnt[w][j[u]][ob[u] >> 2] >> (8 * (ob[u] & 3))) & 0xff;
        const int32_t cn = (cnt[w][j[u]][nb[u] >> 2] >> (8 * (nb[u] & 3))) & 0xff;
        const int64_t row = (int64_t)(cd[u].x + j[u]) * k;
        phi[row + ob[u]] = (T)co;
        phi[row + nb[u]] = (T)cn;
      }
      // per net: new words and metric change (lane x of the wave handles net x of the chunk)
      if (l < cd[u].y) {
        const int64_t e = cd[u].x + l;
        uint64_t *nse = ns + e * (2 * NW);
        int lam_old = 0, lam_new = 0;
#pragma unroll
        for (int x = 0; x < NW; ++x) {
          const uint64_t a = once[w][l][x], bb = twice[w][l][x];
          lam_old += __popcll(wd[u][x]);
          lam_new += __popcll(a);
          if (a != wd[u][x]) nse[x] = a;
          if ((a & ~bb) != wd[u][NW + x]) nse[NW + x] = a & ~bb;
        }
        if (lam_new != lam_old) {
          const int64_t d = (int64_t)(lam_new - lam_old) * (nw ? nw[e] : 1);
          if (un.nhg) add_km1_hg(st, un.nhg[e], d);
          else dk += d;
        }
      }
      wave_lds_sync();  // the LDS slots are reused by the next chunk
      if (act[u]) cnt[w][j[u]][nb[u] >> 2] = 0u;  // every nonzero counter word has a pin here
    }
  }  // chunk-group loop
  dk = wave_sum(dk);
  if (l == 0) add_km1(st, wid, dk);
}

// Net-centric, larger nets: one block per net; per-block count changes gathered in LDS, then the
// block rewrites the changed counts, the connectivity words and its metric contribution.
template <int NW, typename T, int THREADS>
__global__ __launch_bounds__(THREADS) void k_apply_nets(const int64_t *__restrict__ off, const int32_t *__restrict__ pins,
                                                    const int32_t *__restrict__ nets, int32_t nnets,
                                                    const int32_t *__restrict__ nw,
                                                    const int32_t *__restrict__ part,
                                                    const uint8_t *__restrict__ mvto, int64_t p, int32_t k,
                                                    T *__restrict__ phi, uint64_t *__restrict__ ns,
                                                    int32_t divisor, DevStatus *st, const LoopCtl *lc,
                                                    int32_t want, Union u) {
  JET_GATE(lc, want);
  __shared__ int32_t delta[kMaxK];
  __shared__ unsigned long long words[2 * NW];
  __shared__ int32_t any;
  if (!net_centric(st, p, divisor)) return;
  int64_t dk = 0;  // metric change of this block's nets (thread 0)
  for (int32_t bi = blockIdx.x; bi < nnets; bi += gridDim.x) {  // block-uniform trip count
  const int32_t e = nets[bi];
  const int64_t q0 = off[e], q1 = off[e + 1];
  for (int b = threadIdx.x; b < k; b += blockDim.x) delta[b] = 0;
  if (threadIdx.x == 0) any = 0;
  if (threadIdx.x < 2 * NW) words[threadIdx.x] = ns[(int64_t)e * (2 * NW) + threadIdx.x];
  __syncthreads();
  // four slices of the net at a time, each level of their dependent loads (pin, move target,
  // block) issued for all before any is used
  for (int64_t qb = q0; qb < q1; qb += 4 * THREADS) {
    int32_t v[4], pv[4];
    uint8_t mt[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t q = qb + u * THREADS + threadIdx.x;
      v[u] = q < q1 ? pins[q] : -1;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) mt[u] = v[u] >= 0 ? mvto[v[u]] : (uint8_t)0xff;
#pragma unroll
    for (int u = 0; u < 4; ++u) pv[u] = mt[u] != 0xff ? part[v[u]] : 0;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (mt[u] != 0xff) {
        atomicSub(&delta[pv[u]], 1);
        atomicAdd(&delta[mt[u]], 1);
        any = 1;
      }
    }
  }
  __syncthreads();
  if (any) {
  for (int b = threadIdx.x; b < k; b += blockDim.x) {
    const int32_t d = delta[b];
    if (d == 0) continue;
    const int64_t idx = (int64_t)e * k + b;
    const int32_t nv = (int32_t)phi[idx] + d;
    phi[idx] = (T)nv;
    const unsigned long long bit = 1ull << (b & 63);
    if (nv > 0) atomicOr(&words[b >> 6], bit);
    else atomicAnd(&words[b >> 6], ~bit);
    if (nv == 1) atomicOr(&words[NW + (b >> 6)], bit);
    else atomicAnd(&words[NW + (b >> 6)], ~bit);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t *nse = ns + (int64_t)e * (2 * NW);
    int lam_old = 0, lam_new = 0;
    for (int x = 0; x < NW; ++x) {
      lam_old += __popcll(nse[x]);
      lam_new += __popcll(words[x]);
    }
    for (int x = 0; x < 2 * NW; ++x) nse[x] = words[x];
    if (lam_new != lam_old) {
      const int64_t d = (int64_t)(lam_new - lam_old) * (nw ? nw[e] : 1);
      if (u.nhg) add_km1_hg(st, u.nhg[e], d);
      else dk += d;
    }
  }
  }  // any
  __syncthreads();  // LDS reused by the next net
  }  // net loop
  if (threadIdx.x == 0) add_km1(st, blockIdx.x, dk);
}

inline unsigned grid_for(int64_t work, int block, int64_t cap) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}


template <int G, bool UNIT>
hipError_t cand_launch(Ctx &c, const int32_t *part, int32_t locked_stamp, const uint8_t *lock_bytes, int32_t tau_q,
                       const LoopCtl *lc) {
  constexpr int BLOCK = (G == 16) ? 512 : 256;
  constexpr int VPB = BLOCK / G;
  const unsigned grid = (unsigned)std::min<int64_t>(c.grid_cap, (c.n + VPB - 1) / VPB);
  // algorithmic bytes: per vertex part, lock, offsets, record, flag; per incidence the net ID, one
  // pin count and the net's connectivity mask (and its weight when weighted)
  const double per_inc = 8.0 + (c.k + 7) / 8 + (UNIT ? 0.0 : 4.0);
  const int32_t want = lc ? (int32_t)kPhJet : (int32_t)kPhAny;
  int tok = prof_begin(c, kProfCandidates, lc, want);
  // unit net weights, k <= 64: bit-sliced counts, one lane per vertex while the vertices are light
  // (mean degree below lane_degree), eight otherwise
  if (UNIT && c.k <= 64 && c.p_low < (int64_t)c.lane_degree * c.n_low) {
    hipLaunchKernelGGL(k_candidates_bits<1>, dim3((unsigned)std::min<int64_t>(c.grid_cap, (c.n + 255) / 256)),
                       dim3(256), 0, c.stream, part, c.voff, c.inc, c.ns, c.sumw, c.lockstamp, locked_stamp,
                       lock_bytes, c.n, tau_q, c.rec, c.inm, c.st, lc, union_of(c), c.cand_xcd);
  } else if (UNIT && c.k <= 64) {
    // the groups OR their bits into cleared words (a fill kernel: no memset node in a captured graph)
    const int64_t words = ((int64_t)c.n + 255) / 256 * 8;
    hipError_t fe = launch_fill_u32(c, c.inm, words, 0u, lc, want);
    if (fe != hipSuccess) return fe;
    hipLaunchKernelGGL(k_candidates_bits<8>, dim3((unsigned)std::min<int64_t>(c.grid_cap, (c.n + 31) / 32)),
                       dim3(256), 0, c.stream, part, c.voff, c.inc, c.ns, c.sumw, c.lockstamp, locked_stamp,
                       lock_bytes, c.n, tau_q, c.rec, c.inm, c.st, lc, union_of(c), c.cand_xcd);
  } else
    hipLaunchKernelGGL((k_candidates<G, UNIT>), dim3(grid), dim3(BLOCK), 0, c.stream, part, c.voff, c.inc, c.nw, c.ns,
                       c.sumw, c.lockstamp, locked_stamp, lock_bytes, c.n, tau_q, c.rec, c.inm, c.st, lc,
                       union_of(c));
  prof_end(c, tok, lc, want, 18.0 * c.n_low, per_inc);  // plus per_inc per scanned incidence (device count)
  if (c.nhubs > 0) {
    tok = prof_begin(c, kProfCandidatesHub, lc, want);
    hipLaunchKernelGGL((k_candidates_hub<G, UNIT>), dim3((unsigned)std::min<int64_t>(c.grid_cap, c.nhubs)),
                       dim3(256), 0, c.stream, part, c.voff, c.inc, c.nw, c.ns, c.sumw, c.lockstamp, locked_stamp,
                       lock_bytes, c.hubs, c.nhubs, c.k, tau_q, c.rec, c.inm, c.st, lc, union_of(c));
    prof_end(c, tok, lc, want, 18.0 * (c.n - c.n_low), per_inc);
  }
  return hipGetLastError();
}

template <bool UNIT>
hipError_t cand_dispatch(Ctx &c, const int32_t *part, int32_t locked_stamp, const uint8_t *lock_bytes,
                         int32_t tau_q, const LoopCtl *lc) {
  if (c.k <= 8) return cand_launch<1, UNIT>(c, part, locked_stamp, lock_bytes, tau_q, lc);
  if (c.k <= 16) return cand_launch<2, UNIT>(c, part, locked_stamp, lock_bytes, tau_q, lc);
  if (c.k <= 32) return cand_launch<4, UNIT>(c, part, locked_stamp, lock_bytes, tau_q, lc);
  if (c.k <= 64) return cand_launch<8, UNIT>(c, part, locked_stamp, lock_bytes, tau_q, lc);
  return cand_launch<16, UNIT>(c, part, locked_stamp, lock_bytes, tau_q, lc);
}

constexpr int kApplyGrid = 2048;

}  // namespace

// One launch clears the per-iteration counters (instead of a fill per field).
__global__ void k_reset_counters(DevStatus *st, int32_t what, const LoopCtl *lc, int32_t want, int32_t H) {
  JET_GATE(lc, want);
  if ((what & kResetMoves) && H > 1)  // union: per-hypergraph move counts
    for (int32_t i = threadIdx.x; i < H; i += blockDim.x) st->hmoves[i] = 0;
  if (threadIdx.x != 0) return;
  if (what & kResetCandidates) {
    st->n_cand = 0;
    st->inc_low = 0;
    st->inc_hub = 0;
    st->ab_inc = 0;
    st->n_ovf = 0;
  }
  if (what & kResetMoves) {
    st->n_moves = 0;
    st->n_bigmv = 0;
    st->mv_inc = 0;
  }
}

hipError_t launch_reset_counters(Ctx &c, int32_t what, const LoopCtl *lc, int32_t want) {
  hipLaunchKernelGGL(k_reset_counters, dim3(1), dim3(256), 0, c.stream, c.st, what, lc, want, c.H);
  return hipGetLastError();
}

hipError_t launch_candidates(Ctx &c, const int32_t *part, int32_t locked_stamp, const uint8_t *lock_bytes,
                             int32_t tau_q, const LoopCtl *lc) {
  // every counter of the iteration (candidates, afterburner overflow list, move list) starts at 0
  hipError_t e = launch_reset_counters(c, kResetCandidates | kResetMoves, lc, lc ? (int32_t)kPhJet : (int32_t)kPhAny);
  if (e != hipSuccess) return e;
  return c.unit_nw ? cand_dispatch<true>(c, part, locked_stamp, lock_bytes, tau_q, lc)
                   : cand_dispatch<false>(c, part, locked_stamp, lock_bytes, tau_q, lc);
}

hipError_t launch_export_candidates(Ctx &c, int32_t *t, int32_t *g, uint8_t *in_m) {
  hipLaunchKernelGGL(k_export_candidates, dim3(grid_for(c.n, 256, INT32_MAX)), dim3(256), 0, c.stream, c.rec, c.inm,
                     c.n, t, g, in_m);
  return hipGetLastError();
}

hipError_t launch_import_candidates(Ctx &c, const int32_t *part, const int32_t *t, const int32_t *g,
                                    const uint8_t *in_m) {
  const int64_t nwords = ((int64_t)c.n + 255) / 256 * 8;
  const int64_t work = nwords > c.n ? nwords : c.n;
  hipLaunchKernelGGL(k_import_candidates, dim3(grid_for(work, 256, INT32_MAX)), dim3(256), 0, c.stream, part, t, g,
                     in_m, c.n, c.k, nwords, c.rec, c.inm, c.st);
  return hipGetLastError();
}

// Sums the private copies of the recomputed gains into rg and clears them.
__global__ void k_rg_reduce(int32_t *__restrict__ rgx, int32_t copies, int32_t n, int32_t *__restrict__ rg,
                            const LoopCtl *lc) {
  JET_GATE(lc, kPhJet);
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x) {
    int32_t s = 0;
    for (int32_t r = 0; r < copies; ++r) {
      int32_t *p = rgx + (size_t)r * n + v;
      s += *p;
      *p = 0;
    }
    rg[v] = s;
  }
}

// Larger nets of the afterburner: 1,024-entry LDS lists for medium nets above 256 pins, 256-entry
// ones below, and the big-net kernel with its global-scratch overflow list.
template <int NW, typename T>
void ab_nets_launch(Ctx &c, RgSink sink, const T *phi, const LoopCtl *lc) {
  if (c.nmid_large > 0)
    hipLaunchKernelGGL((k_ab_nets<128, kMediumNet, NW, T>), dim3((unsigned)c.nmid_large), dim3(128), 0, c.stream, c.off,
                       c.pins, c.mid_nets, c.nw, c.inm, c.rec, phi, c.ns, c.k, sink, c.st, (int2 *)nullptr, lc, union_of(c));
  if (c.nmid > c.nmid_large)
    hipLaunchKernelGGL((k_ab_nets<64, kMediumSmall, NW, T>), dim3((unsigned)(c.nmid - c.nmid_large)), dim3(64), 0,
                       c.stream, c.off, c.pins, c.mid_nets + c.nmid_large, c.nw, c.inm, c.rec, phi, c.ns, c.k, sink,
                       c.st, (int2 *)nullptr, lc, union_of(c));
  if (c.nbig > 0)
    hipLaunchKernelGGL((k_ab_nets<512, kBigCap, NW, T>), dim3((unsigned)c.nbig), dim3(512), 0, c.stream, c.off, c.pins,
                       c.big_nets, c.nw, c.inm, c.rec, phi, c.ns, c.k, sink, c.st, c.ovf_list, lc, union_of(c));
}

hipError_t launch_afterburner(Ctx &c, const int32_t *part, const LoopCtl *lc) {
  // n_ovf was cleared with the candidate counters
  const RgSink sink = c.rg_copies > 1 ? RgSink{c.rgx, c.n, c.rg_copies} : RgSink{c.rg, c.n, 1};
  // algorithmic bytes (streaming part): net offsets, pins, candidate flag per pin, gains per vertex
  const int32_t want = lc ? (int32_t)kPhJet : (int32_t)kPhAny;
  const int tok = prof_begin(c, kProfAfterburner, lc, want);
  if (graph_afterburner(c)) {
    // every net has two pins: the vertex-centric form (k_graph.hip); 4 B per vertex (gain written)
    // plus, on the device, per scanned incidence of a candidate the neighbour, its block and
    // candidate bit (and the net weight), and 24 B per candidate (record, offsets)
    const hipError_t e = launch_ab_graph(c, part, lc, want);
    prof_end(c, tok, lc, want, 4.125 * c.n, 8.125 + (c.unit_nw ? 0.0 : 8.0));
    return e;
  }
  if (c.nchunks > 0) {
    const dim3 grid((unsigned)std::min<int64_t>(c.grid_cap, (c.nchunks + 3) / 4));
    if (c.k <= 64)
      hipLaunchKernelGGL(k_ab_chunks<16>, grid, dim3(256), 0, c.stream, c.pins, c.chunks, c.pnet, c.nchunks, c.nw,
                         part, c.inm, c.rec, sink, lc, union_of(c), c.cand_xcd);
    else
      hipLaunchKernelGGL(k_ab_chunks<kMaxK / 4>, grid, dim3(256), 0, c.stream, c.pins, c.chunks, c.pnet, c.nchunks,
                         c.nw, part, c.inm, c.rec, sink, lc, union_of(c), c.cand_xcd);
  }
  if (c.nw_words == 1) {
    if (c.phi16) ab_nets_launch<1>(c, sink, c.phi16, lc);
    else ab_nets_launch<1>(c, sink, c.phi, lc);
  } else {
    if (c.phi16) ab_nets_launch<2>(c, sink, c.phi16, lc);
    else ab_nets_launch<2>(c, sink, c.phi, lc);
  }
  hipError_t err = hipGetLastError();
  if (err != hipSuccess) return err;
  err = launch_afterburner_overflow(c, sink, lc);
  if (err == hipSuccess && c.rg_copies > 1) {
    // rg holds 0 for every vertex here (select clears the candidates' entries): plain stores
    hipLaunchKernelGGL(k_rg_reduce, dim3((unsigned)std::min<int64_t>(1024, (c.n + 255) / 256)), dim3(256), 0,
                       c.stream, c.rgx, c.rg_copies, c.n, c.rg, lc);
    err = hipGetLastError();
  }
  prof_end(c, tok, lc, want, 4.0 * c.m + 5.0 * c.p + 8.0 * c.n, 0.0);
  return err;
}

hipError_t launch_select_moves(Ctx &c, const int32_t *part, int32_t stamp, const LoopCtl *lc) {
  // the move counters were cleared with the candidate counters
  const int32_t want = lc ? (int32_t)kPhJet : (int32_t)kPhAny;
  const int tok = prof_begin(c, kProfSelect, lc, want);
  hipLaunchKernelGGL(k_select_moves, dim3(grid_for(c.n, kSelBlock * kCompactPer, c.grid_cap)), dim3(kSelBlock), 0,
                     c.stream, part, c.inm, c.rec,
                     c.rg, c.vw, c.n, stamp, c.lockstamp, c.moves, c.mvto, c.voff, c.st, c.bigmv, lc, union_of(c));
  prof_end(c, tok, lc, want, 8.5 * c.n, 0.0);
  return hipGetLastError();
}

hipError_t launch_diff_moves(Ctx &c, const int32_t *part, const int32_t *target, const LoopCtl *lc) {
  hipError_t e = launch_reset_counters(c, kResetMoves, lc, lc ? (int32_t)kPhRoll : (int32_t)kPhAny);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_diff_moves, dim3(grid_for(c.n, kSelBlock * kCompactPer, c.grid_cap)), dim3(kSelBlock), 0, c.stream,
                     part, target, c.vw,
                     c.n, c.moves, c.mvto, c.voff, c.st, c.bigmv, lc, union_of(c));
  return hipGetLastError();
}

template <int NW, typename T>
void apply_launch(Ctx &c, int32_t *part, bool wide, T *phi, const LoopCtl *lc, int32_t want) {
  // The net-centric kernels read the old blocks, so they run before k_apply writes the new ones.
  // The device decides which path runs; `wide` only sizes their grids: one wave per chunk and one
  // block per net when the host expects the net-centric path, a small grid that exits at once
  // otherwise (either grid gives the same result).
  const unsigned cap = wide ? 0x7fffffffu : 2048u;
  if (c.nchunks > 0)
    hipLaunchKernelGGL((k_apply_chunks<NW, T>),
                       dim3(std::min(cap, (unsigned)((c.nchunks + 4 * kApplyU - 1) / (4 * kApplyU)))), dim3(256), 0,
                       c.stream, c.off, c.pins, c.chunks, c.pnet, c.nchunks, c.nw, part, c.mvto, c.p, c.k, phi, c.ns,
                       c.apply_divisor, c.st, lc, want, union_of(c), c.apply_xcd);
  if (c.nmid > 0)
    hipLaunchKernelGGL((k_apply_nets<NW, T, 128>), dim3(std::min(cap, (unsigned)c.nmid)), dim3(128), 0, c.stream,
                       c.off, c.pins, c.mid_nets, c.nmid, c.nw, part, c.mvto, c.p, c.k, phi, c.ns, c.apply_divisor,
                       c.st, lc, want, union_of(c));
  if (c.nbig > 0)
    hipLaunchKernelGGL((k_apply_nets<NW, T, 256>), dim3(std::min(cap, (unsigned)c.nbig)), dim3(256), 0, c.stream,
                       c.off, c.pins, c.big_nets, c.nbig, c.nw, part, c.mvto, c.p, c.k, phi, c.ns, c.apply_divisor,
                       c.st, lc, want, union_of(c));
  hipLaunchKernelGGL((k_apply<NW, T>), dim3(kApplyGrid), dim3(256), 0, c.stream, c.moves, c.voff, c.inc, c.nw, c.p, c.k,
                     part, phi, c.ns, c.mvto, c.bigmv, c.apply_divisor, c.st, lc, want, union_of(c), c.apply_xcd);
}

hipError_t launch_apply_moves(Ctx &c, int32_t *part, bool wide, const LoopCtl *lc, int32_t want) {
  const int tok = prof_begin(c, kProfApply, lc, want);
  if (c.nw_words == 1) {
    if (c.phi16) apply_launch<1>(c, part, wide, c.phi16, lc, want);
    else apply_launch<1>(c, part, wide, c.phi, lc, want);
  } else {
    if (c.phi16) apply_launch<2>(c, part, wide, c.phi16, lc, want);
    else apply_launch<2>(c, part, wide, c.phi, lc, want);
  }
  prof_end(c, tok, lc, want, 0.0, 0.0);  // bytes from the move and moved-incidence counts (device)
  return hipGetLastError();
}

}  // namespace jet
