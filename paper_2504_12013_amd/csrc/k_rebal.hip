// Deterministic rebalancing round (Section 4.3) on the device.
//
//  prepare : per overloaded block the weight that must leave (bw - Lmax) and its list region
//  gain    : per vertex of an overloaded block that passes the heavy-vertex rule, the best valid
//            target (balanced after adding v, not in the deadzone; adjacency not required; lowest
//            block on ties) and an exact 160-bit order key
//  select  : per overloaded block, radix selection of the minimal prefix (in priority order) whose
//            weight reaches the needed amount -- the same set as sort + prefix sum + binary search
//  apply   : shared with the Jet moves (all selected vertices move at once)
//
// Order key, descending = (priority desc, vertex ID asc), priority gain*c for gain >= 0 and gain/c
// for gain < 0.  Words (most significant first):
//   w0      a 32-bit code that never decreases with the priority (bit length + leading 24 bits of
//           an exact integer image of it), so the first passes split the list well;
//   w1..w3  K + 2^95 where K = gain*c for gain >= 0 and K = -ceil(|gain| 2^62 / c) for gain < 0:
//           distinct rationals with c < 2^31 differ by more than 2^-62, so K orders them exactly;
//   w4      0xffffffff - v.
#include <algorithm>
#include <climits>

#include "conn.h"
#include "dev_util.h"
#include "jet_internal.h"
#include "moves.h"

namespace jet {

namespace {

__device__ __forceinline__ uint32_t mono_code(unsigned __int128 x) {
  if (x == 0) return 0u;
  const uint64_t hi = (uint64_t)(x >> 64), lo = (uint64_t)x;
  const int L = hi ? 128 - __clzll(hi) : 64 - __clzll(lo);  // bit length, 1..128
  uint32_t mant;
  if (L - 1 >= 24) mant = (uint32_t)(x >> (L - 1 - 24)) & 0xffffffu;
  else mant = (uint32_t)(x << (24 - (L - 1))) & 0xffffffu;
  return ((uint32_t)L << 24) | mant;
}

__device__ __forceinline__ void order_key(int32_t g, int32_t c, int32_t v, uint32_t key[5]) {
  const unsigned __int128 bias = (unsigned __int128)1 << 95;
  unsigned __int128 U;
  if (g >= 0) {
    const unsigned __int128 gc = (unsigned __int128)((uint64_t)(uint32_t)g * (uint64_t)(uint32_t)c);
    U = bias + gc;
    key[0] = 0x80000000u | mono_code(gc);
  } else {
    const uint64_t a = (uint64_t)(-(int64_t)g), cc = (uint64_t)(uint32_t)c;
    const uint64_t q0 = a / cc, r0 = a % cc;
    const uint64_t x1 = r0 << 31, f1 = x1 / cc, r1 = x1 % cc;
    const uint64_t x2 = r1 << 31, f2 = x2 / cc, r2 = x2 % cc;
    const unsigned __int128 ce =
        ((unsigned __int128)q0 << 62) + ((unsigned __int128)f1 << 31) + (unsigned __int128)f2 + (r2 != 0 ? 1 : 0);
    U = bias - ce;
    key[0] = 0x7fffffffu - mono_code(ce);
  }
  key[1] = (uint32_t)(U >> 64);
  key[2] = (uint32_t)(U >> 32);
  key[3] = (uint32_t)U;
  key[4] = 0xffffffffu - (uint32_t)v;
}

// The key of an entry in the order jet_params.rb_unweighted names: 0 the priority of Section 4.3,
// 1 the gain alone (the original Jet's priority), 2 the original's bucket order of the loss
// (Section 4.3 contrasts it with the sort): a move that does not lose goes to bucket 0, a loss
// L >= 1 to bucket 1 + floor(log2 L); lower buckets first, and inside a bucket vertex-ID order
// stands in for the original's arrival order.  Bucket words: w0 = (255 - bucket) << 24,
// w1..w3 = 0 (so the selection skips their passes), w4 = 0xffffffff - v as for the priorities.
// The bucket words replace the others by selects, so the key stays in registers.
__device__ __forceinline__ void entry_key(int32_t g, int32_t c, int32_t v, int32_t order, uint32_t key[5]) {
  order_key(g, order ? 1 : c, v, key);
  const bool bk = order == 2;
  const int32_t bucket = g >= 0 ? 0 : 64 - __clzll((unsigned long long)(-(int64_t)g));
  key[0] = bk ? (uint32_t)(255 - bucket) << 24 : key[0];
  key[1] = bk ? 0u : key[1];
  key[2] = bk ? 0u : key[2];
  key[3] = bk ? 0u : key[3];
}

// entry layout: 8 words = key[0..4], v, target, weight
constexpr int kEntryWords = 8;

__global__ void k_rb_prepare(int32_t k, int64_t lmax, DevStatus *st, const LoopCtl *lc) {
  JET_GATE(lc, kPhRb);
  __shared__ int64_t cnts[kMaxK];
  const int b = threadIdx.x;
  if (b < k) {
    const int64_t over = st->bw[b] - lmax;
    st->rb_need[b] = over > 0 ? over : 0;
    st->rb_count[b] = 0;
    st->rb_kept[b] = 0;
    cnts[b] = over > 0 ? st->bcnt[b] : 0;
  }
  __syncthreads();
  if (b == 0) {
    int64_t run = 0;
    for (int i = 0; i < k; ++i) {
      st->rb_off[i] = run;
      run += cnts[i];
    }
    st->rb_off[k] = run;
    st->n_moves = 0;
    st->n_bigmv = 0;
    st->mv_inc = 0;
    st->rb_inc = 0;
    st->rb_elig = 0;
    st->rb_ent = 0;
    st->rb_nlist = 0;
    st->rb_nhub = 0;
  }
}

// Union contexts (many hypergraphs, segments hg * k + b): the need and list region of every
// segment of a hypergraph in the rebalancing phase, its move count cleared, one workgroup scanning
// the segments in order.
constexpr int kPrepThreads = 1024;
__global__ __launch_bounds__(kPrepThreads) void k_rb_prepare_union(int32_t k, int32_t H, DevStatus *st,
                                                                   const LoopCtl *lc, Union u) {
  JET_GATE(lc, kPhRb);
  __shared__ int64_t sm[kPrepThreads / kWave + 1];
  __shared__ int64_t carry, scarry;
  if (threadIdx.x == 0) carry = scarry = 0;
  const int32_t nseg = H * k;
  for (int32_t base = 0; base < nseg; base += kPrepThreads) {  // block-uniform trip count
    const int32_t sg = base + threadIdx.x;
    int64_t cnt = 0;
    if (sg < nseg) {
      const int32_t hg = sg / k;
      const LoopCtl &h = u.lcs[hg];
      int64_t need = 0;
      if (h.phase == kPhRb) {
        const int64_t over = st->bw[sg] - h.lmax;
        need = over > 0 ? over : 0;
        if (sg % k == 0) st->hmoves[hg] = 0;
      }
      st->rb_need[sg] = need;
      st->rb_count[sg] = 0;
      st->rb_kept[sg] = 0;
      cnt = need > 0 ? st->bcnt[sg] : 0;
    }
    int64_t tot;
    const int64_t ex = block_excl_scan<kPrepThreads>(cnt, sm, &tot);
    if (sg < nseg) st->rb_off[sg] = carry + ex;
    // the overloaded segments, in order, for the selection
    int64_t ntot;
    const int64_t nex = block_excl_scan<kPrepThreads>((int64_t)(cnt > 0 ? 1 : 0), sm, &ntot);
    if (cnt > 0) st->rb_seg[scarry + nex] = sg;
    __syncthreads();
    if (threadIdx.x == 0) {
      carry += tot;
      scarry += ntot;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    st->rb_off[nseg] = carry;
    st->rb_nseg = (int32_t)scarry;
    st->n_moves = 0;
    st->n_bigmv = 0;
    st->mv_inc = 0;
    st->rb_inc = 0;
    st->rb_elig = 0;
    st->rb_ent = 0;
    st->rb_nlist = 0;
    st->rb_nhub = 0;
  }
}

// Union: movable non-hub vertices of overloaded segments (heavy-vertex rule with the hypergraph's
// own ceil(W/k)), each with an entry slot in its segment's region (order inside a region does not
// matter: entries are selected by exact keys).  A workgroup takes kListPer tiles of the listed
// hypergraphs at a time (each tile one hypergraph's), counts per (tile, block) in LDS and reserves
// list positions and region slots with one atomic per workgroup and per (tile, overloaded block).
__global__ __launch_bounds__(kUnionTile) void k_rb_list_union(const int32_t *__restrict__ part,
                                                              const int32_t *__restrict__ vw,
                                                              const int64_t *__restrict__ voff, int32_t n, int32_t k,
                                                              DevStatus *st, int32_t *__restrict__ list,
                                                              int32_t *__restrict__ slot, const LoopCtl *lctl,
                                                              Union u) {
  JET_GATE(lctl, kPhRb);
  constexpr int T = 8;  // tiles per workgroup step
  __shared__ int64_t s_vb[T], s_lmax[T], s_A[T];
  __shared__ int32_t s_hg[T];
  __shared__ int64_t sbw[T][kMaxK];
  __shared__ int32_t lcnt[T][kMaxK], lbase[T][kMaxK];
  __shared__ int32_t sm[kUnionTile / kWave + 1];
  __shared__ int32_t s_base;
  const int tid = threadIdx.x;
  const ActList &L = u.act[kActRb];
  const int32_t nt = L.tpref[L.cnt];
  for (int32_t t0 = blockIdx.x * T; t0 < nt; t0 += gridDim.x * T) {  // block-uniform trip count
    if (tid < kWave)  // the first wave finds every tile's first vertex and hypergraph
      for (int j = 0; j < T; ++j) {
        int32_t hg = 0;
        const int64_t vb = t0 + j < nt ? act_tile_base(L, u.ht0, t0 + j, &hg) : (int64_t)n;
        if (tid == 0) {
          s_vb[j] = vb;
          s_hg[j] = hg;
          s_lmax[j] = u.lcs[hg].lmax;
          s_A[j] = u.lcs[hg].A;
        }
      }
    __syncthreads();
    for (int x = tid; x < T * k; x += kUnionTile) {
      const int j = x / k, b = x % k;
      sbw[j][b] = s_vb[j] < n ? st->bw[(int64_t)s_hg[j] * k + b] : 0;
      lcnt[j][b] = 0;
    }
    __syncthreads();
    uint32_t mask = 0;
    int32_t cnt = 0, sv[T];
    int32_t loc[T];
#pragma unroll
    for (int j = 0; j < T; ++j) {
      sv[j] = 0;
      loc[j] = 0;
      const int64_t v = s_vb[j] + tid;
      if (s_vb[j] >= n || v >= n) continue;
      const int32_t s = part[v];
      const int64_t bs = sbw[j][s];
      if (bs <= s_lmax[j] || u.vhg[v] != s_hg[j]) continue;  // not overloaded, or a padding vertex
      const int64_t c = vw ? vw[v] : 1;
      if (2 * c <= 3 * (bs - s_A[j]) && voff[v + 1] - voff[v] <= kHubDegree) {
        mask |= 1u << j;
        ++cnt;
        sv[j] = s;
        loc[j] = atomicAdd(&lcnt[j][s], 1);
      }
    }
    int32_t tot;
    const int32_t rk = block_excl_scan<kUnionTile>(cnt, sm, &tot);
    if (tid == 0) s_base = tot ? atomicAdd(&st->rb_nlist, tot) : 0;
    for (int x = tid; x < T * k; x += kUnionTile) {
      const int j = x / k, b = x % k;
      const int32_t c = lcnt[j][b];
      if (c) {
        const int64_t sg = (int64_t)s_hg[j] * k + b;
        lbase[j][b] = (int32_t)(st->rb_off[sg] + atomicAdd(&st->rb_count[sg], c));
      }
    }
    __syncthreads();
    int32_t out = s_base + rk;
#pragma unroll
    for (int j = 0; j < T; ++j) {
      if ((mask >> j) & 1u) {
        list[out] = (int32_t)(s_vb[j] + tid);
        slot[out] = lbase[j][sv[j]] + loc[j];
        ++out;
      }
    }
    __syncthreads();  // LDS is rewritten by the next step
  }
}

// Rebalancing candidates of the round (Section 4.3): movable non-hub vertices of overloaded blocks
// (eligible under the heavy-vertex rule), listed so that the gain pass touches only them, with
// the entry slot each one owns in its block's region of the entry array.  Each workgroup takes
// kListPer vertices per thread (strided, so the loads coalesce), all loads in flight at once:
// it counts per block, one atomic per block reserves the slots (the block's count of listed
// vertices, after which hub entries are appended), and the threads write their vertices from
// registers.  The order inside a region does not matter: entries are selected by exact keys.
constexpr int kListBlock = 256;
constexpr int kListPer = 8;
__global__ __launch_bounds__(kListBlock) void k_rb_list(const int32_t *__restrict__ part,
                                                        const int32_t *__restrict__ vw,
                                                        const int64_t *__restrict__ voff, int32_t n, int32_t k,
                                                        int64_t lmax, int64_t A, DevStatus *st,
                                                        int32_t *__restrict__ list, int32_t *__restrict__ slot,
                                                        const LoopCtl *lctl) {
  JET_GATE(lctl, kPhRb);
  __shared__ int64_t bw[kMaxK];
  __shared__ int32_t lc[kMaxK], lbase[kMaxK];
  __shared__ int32_t sm[kListBlock / kWave + 1];
  __shared__ int32_t s_base;
  const int tid = threadIdx.x;
  for (int b = tid; b < k; b += kListBlock) {
    bw[b] = st->bw[b];
    lc[b] = 0;
  }
  __syncthreads();
  const int64_t r0 = (int64_t)blockIdx.x * (kListBlock * kListPer) + tid;
  int32_t pv[kListPer];
#pragma unroll
  for (int j = 0; j < kListPer; ++j) {
    const int64_t v = r0 + j * kListBlock;
    pv[j] = v < n ? part[v] : -1;
  }
  // vertices of overloaded blocks: weight and degree (loaded only for them)
  bool over[kListPer];
  int64_t bs[kListPer], c[kListPer], d0[kListPer], d1[kListPer];
#pragma unroll
  for (int j = 0; j < kListPer; ++j) {
    bs[j] = pv[j] >= 0 ? bw[pv[j]] : 0;
    over[j] = pv[j] >= 0 && bs[j] > lmax;
  }
#pragma unroll
  for (int j = 0; j < kListPer; ++j) {
    c[j] = 1;
    d0[j] = 0;
    d1[j] = 0;
    if (over[j]) {
      const int64_t v = r0 + j * kListBlock;
      if (vw) c[j] = vw[v];
      d0[j] = voff[v];
      d1[j] = voff[v + 1];
    }
  }
  uint32_t mask = 0;
  int32_t cnt = 0;
#pragma unroll
  for (int j = 0; j < kListPer; ++j) {
    if (over[j] && 2 * c[j] <= 3 * (bs[j] - A) && d1[j] - d0[j] <= kHubDegree) {  // hubs: listed separately
      mask |= 1u << j;
      ++cnt;
      atomicAdd(&lc[pv[j]], 1);
    }
  }
  int32_t tot;
  const int32_t rk = block_excl_scan<kListBlock>(cnt, sm, &tot);
  if (tid == 0) s_base = tot ? atomicAdd(&st->rb_nlist, tot) : 0;
  for (int b = tid; b < k; b += kListBlock) {
    const int32_t x = lc[b];
    lbase[b] = x ? (int32_t)st->rb_off[b] + atomicAdd(&st->rb_count[b], x) : 0;
    lc[b] = 0;
  }
  __syncthreads();
  if (tot == 0) return;
  int32_t out = s_base + rk;
#pragma unroll
  for (int j = 0; j < kListPer; ++j) {
    if ((mask >> j) & 1u) {
      list[out] = (int32_t)(r0 + j * kListBlock);
      slot[out] = lbase[pv[j]] + atomicAdd(&lc[pv[j]], 1);
      ++out;
    }
  }
}

// One rebalancing entry: the exact order key, vertex, target and weight; a vertex without a valid
// target leaves weight 0 (the selection skips such entries).
// order: jet_params.rb_unweighted (entry_key); the entry keeps the real weight c
__device__ __forceinline__ void write_entry(uint32_t *ent, bool ok, int32_t g, int32_t c, int32_t v, int32_t t,
                                            int32_t order) {
  uint32_t key[5] = {0u, 0u, 0u, 0u, 0u};
  if (ok) entry_key(g, c, v, order, key);
#pragma unroll
  for (int i = 0; i < 5; ++i) ent[i] = key[i];
  ent[5] = (uint32_t)v;
  ent[6] = ok ? (uint32_t)t : 0xffu;
  ent[7] = ok ? (uint32_t)c : 0u;
}

// Adds the thread's counts (scanned incidences, examined vertices, written entries) to the status,
// one atomic per workgroup and counter.  Every thread of the block calls it.
template <int NWV>
__device__ __forceinline__ void flush_rb_counters(unsigned long long a, unsigned long long b, unsigned long long c,
                                                  unsigned long long (*wsum)[3], DevStatus *st) {
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int w = threadIdx.x / kWave;
  if (lane_id() == 0) {
    wsum[w][0] = a;
    wsum[w][1] = b;
    wsum[w][2] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t0 = 0ull, t1 = 0ull, t2 = 0ull;
    for (int i = 0; i < NWV; ++i) {
      t0 += wsum[i][0];
      t1 += wsum[i][1];
      t2 += wsum[i][2];
    }
    if (t1) {
      atomicAdd((unsigned long long *)&st->rb_inc, t0);
      atomicAdd((unsigned long long *)&st->rb_elig, t1);
      if (t2) atomicAdd((unsigned long long *)&st->rb_ent, t2);
    }
  }
}

template <int G, bool UNIT>
__global__ __launch_bounds__(G == 16 ? 512 : 256) void k_rb_gain(
    const int32_t *__restrict__ part, const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
    const int32_t *__restrict__ nw, const uint64_t *__restrict__ ns, const int32_t *__restrict__ sumw,
    const int32_t *__restrict__ vw, const int32_t *__restrict__ list, const int32_t *__restrict__ slot, int32_t k,
    int64_t lmax, int64_t dz, DevStatus *st, uint32_t *__restrict__ entries, const LoopCtl *lc, Union u,
    int32_t xcd) {
  JET_GATE(lc, kPhRb);
  if (lc && !u.lcs) dz = lc->dz;
  constexpr int BLOCK = (G == 16) ? 512 : 256;
  constexpr int VPB = BLOCK / G;
  __shared__ int64_t bw[kMaxK];
  __shared__ unsigned long long wsum[BLOCK / kWave][3];
  for (int b = threadIdx.x; b < k; b += BLOCK) bw[b] = st->bw[b];
  __syncthreads();
  const int lg = threadIdx.x % G;
  const int64_t nl = st->rb_nlist;  // listed by k_rb_list: every entry is eligible
  const int64_t ntiles = (nl + VPB - 1) / VPB;
  unsigned long long scanned = 0ull, examined = 0ull, emitted = 0ull;
  // with xcd set, the workgroups of one XCD (round robin by workgroup) take one contiguous eighth of
  // the list, whose vertices are neighbours: their nets' words are fetched into one L2
  int64_t t0 = blockIdx.x, tend = ntiles, tstep = gridDim.x;
  if (xcd && !u.lcs && gridDim.x % 8 == 0) {
    const int64_t per = (ntiles + 7) / 8, x = blockIdx.x % 8;
    t0 = x * per + blockIdx.x / 8;
    tend = min(ntiles, (x + 1) * per);
    tstep = gridDim.x / 8;
  }
  for (int64_t tile = t0; tile < tend; tile += tstep) {  // no barriers: each vertex owns its slot
    const int64_t i = tile * VPB + threadIdx.x / G;
    const bool elig = i < nl;
    int64_t v = 0;
    int32_t s = 0, c = 1;
    int64_t q0 = 0, q1 = 0;
    int64_t lm = lmax, dzz = dz, sg0 = 0;  // union: the vertex's hypergraph's limits and segments
    int32_t unw = (lc && !u.lcs) ? lc->rb_unw : 0;
    if (elig) {
      v = list[i];
      s = part[v];
      c = vw ? vw[v] : 1;
      q0 = voff[v];
      q1 = voff[v + 1];
      if (u.lcs) {
        const int32_t hg = u.vhg[v];
        lm = u.lcs[hg].lmax;
        dzz = u.lcs[hg].dz;
        sg0 = (int64_t)hg * k;
        unw = u.lcs[hg].rb_unw;
      }
    }
    int32_t conn[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) conn[j] = 0;
    int32_t benefit = 0;
    if (elig) vertex_conn<G, UNIT>(inc, q0, q1, G, nw, ns, lg, s, conn, benefit);
    // best valid target by conn (gain = conn - aff), lowest block on ties; -1 = none
    int32_t bestc = -1, bestb = INT32_MAX;
    if (elig) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int32_t b = lg * 8 + j;
        if (b >= k) continue;
        const int64_t bwb = u.lcs ? st->bw[sg0 + b] : bw[b];
        if (b != s && bwb + c <= lm && bwb < dzz && conn[j] > bestc) {
          bestc = conn[j];
          bestb = b;
        }
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
    if (elig && lg == 0) {
      uint32_t *ent = entries + (int64_t)slot[i] * kEntryWords;
      write_entry(ent, bestc >= 0, bestc - (sumw[v] - benefit), c, (int32_t)v, bestb, unw);
      scanned += (unsigned long long)(q1 - q0);
      examined += 1ull;
      emitted += bestc >= 0 ? 1ull : 0ull;
    }
  }
  flush_rb_counters<BLOCK / kWave>(scanned, examined, emitted, wsum, st);
}

// Unit net weights and k <= 64: G lanes per listed vertex (G = 1 on light levels), the block
// counts conn(v, b) bit-sliced as in the candidate pass (conn.h).  The valid targets form a mask
// (b != s, room for v's weight, outside the deadzone); the best is the lowest block of largest
// count in it (counts of zero included, as for the lane-group kernel).
template <int G>
__global__ __launch_bounds__(256) void k_rb_gain_bits(
    const int32_t *__restrict__ part, const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
    const uint64_t *__restrict__ ns, const int32_t *__restrict__ sumw, const int32_t *__restrict__ vw,
    const int32_t *__restrict__ list, const int32_t *__restrict__ slot, int32_t k, int64_t lmax, int64_t dz,
    DevStatus *st, uint32_t *__restrict__ entries, const LoopCtl *lc, int32_t xcd) {
  JET_GATE(lc, kPhRb);
  if (lc) dz = lc->dz;  // one hypergraph (unions take the lane-group kernel)
  const int32_t unw = lc ? lc->rb_unw : 0;
  constexpr int VPW = kWave / G;
  __shared__ int64_t slack[kMaxK];
  __shared__ unsigned long long s_okdz;
  __shared__ long long s_minslack;
  __shared__ unsigned long long wsum[4][3];
  if (threadIdx.x == 0) {
    s_okdz = 0ull;
    s_minslack = LLONG_MAX;
  }
  __syncthreads();
  for (int b = threadIdx.x; b < k; b += 256) {
    const int64_t bwb = st->bw[b];
    slack[b] = lmax - bwb;
    if (bwb < dz) {
      atomicOr(&s_okdz, 1ull << b);
      atomicMin(&s_minslack, (long long)(lmax - bwb));
    }
  }
  __syncthreads();
  const uint64_t okdz = s_okdz;
  const int64_t minslack = s_minslack;
  const int64_t nl = st->rb_nlist;
  const int l = lane_id(), lg = l % G;
  unsigned long long scanned = 0ull, examined = 0ull, emitted = 0ull;
  // with xcd set, the workgroups of one XCD take one contiguous eighth of the list (as k_rb_gain)
  int64_t bstart = ((int64_t)blockIdx.x * 4 + threadIdx.x / kWave) * VPW, bend = nl;
  int64_t bstep = (int64_t)gridDim.x * 4 * VPW;
  if (xcd && gridDim.x % 8 == 0) {
    const int64_t span = 4 * VPW, steps = (nl + span - 1) / span, per = (steps + 7) / 8, x = blockIdx.x % 8;
    bstart = (x * per + blockIdx.x / 8) * span + (threadIdx.x / kWave) * VPW;
    bend = min(nl, (x + 1) * per * span);
    bstep = (int64_t)(gridDim.x / 8) * span;
  }
  for (int64_t base = bstart; base < bend; base += bstep) {  // wave-uniform trip count
    const int64_t i = base + l / G;
    const bool elig = i < nl;
    int32_t v = 0, s = 0, c = 1;
    int64_t q0 = 0, q1 = 0;
    if (elig) {
      v = list[i];
      s = part[v];
      c = vw ? vw[v] : 1;
      q0 = voff[v];
      q1 = voff[v + 1];
    }
    const uint64_t sbit = 1ull << s;
    uint64_t pl[9];
#pragma unroll
    for (int p = 0; p < 9; ++p) pl[p] = 0ull;
    int32_t benefit = 0;
    if (elig) planes_accumulate<G>(inc, q0, q1, ns, lg, sbit, pl, benefit);
    planes_combine<G>(pl, benefit);
    if (!elig || lg != 0) continue;
    // valid targets: room for c (every block outside the deadzone has it when c <= the smallest
    // slack there), outside the deadzone, not s
    uint64_t valid = okdz;
    if ((int64_t)c > minslack) {
      valid = 0ull;
      for (int b = 0; b < k; ++b)
        if (slack[b] >= (int64_t)c) valid |= 1ull << b;
      valid &= okdz;
    }
    int32_t bestb;
    const int32_t bestc = planes_best(pl, valid & ~sbit, bestb);
    write_entry(entries + (int64_t)slot[i] * kEntryWords, bestc >= 0, bestc - (sumw[v] - benefit), c, v, bestb,
                unw);
    scanned += (unsigned long long)(q1 - q0);
    examined += 1ull;
    emitted += bestc >= 0 ? 1ull : 0ull;
  }
  flush_rb_counters<4>(scanned, examined, emitted, wsum, st);
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

// Hub vertices of overloaded blocks (more than kHubDegree incident nets).  A round has few of them
// but each has many nets, so their nets are spread over the whole grid:
//   k_rb_hub_list    lists the hubs the heavy-vertex rule lets move;
//   k_rb_hub_accum   gives every listed hub an equal share of the workgroups, each summing the
//                    per-block connectivity and the benefit of its slice of incident nets into the
//                    hub's column of rb_hacc ([k + 1][nhubs], integer atomics: exact);
//   k_rb_hub_finish  one thread per listed hub: best valid target from the column, order key,
//                    entry (slots reserved per workgroup); clears the column for the next round.
__global__ __launch_bounds__(256) void k_rb_hub_list(const int32_t *__restrict__ part,
                                                     const int32_t *__restrict__ vw,
                                                     const int32_t *__restrict__ hubs, int32_t nhubs,
                                                     int64_t lmax, int64_t A, DevStatus *st,
                                                     int32_t *__restrict__ hlist, const LoopCtl *lc, int32_t k, Union u) {
  JET_GATE(lc, kPhRb);
  const int32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  bool e = false;
  int32_t v = 0;
  if (i < nhubs) {
    v = hubs[i];
    int64_t sg = part[v], lm = lmax, a = A;
    bool on = true;
    if (u.lcs) {  // union: the hub's hypergraph
      const int32_t hg = u.vhg[v];
      on = u.lcs[hg].phase == kPhRb;
      sg += (int64_t)hg * k;
      lm = u.lcs[hg].lmax;
      a = u.lcs[hg].A;
    }
    const int64_t bs = st->bw[sg];
    const int64_t c = vw ? vw[v] : 1;
    e = on && bs > lm && 2 * c <= 3 * (bs - a);
  }
  const uint64_t mm = ballot(e);
  if (!mm) return;
  int32_t base = 0;
  if (lane_id() == 0) base = atomicAdd(&st->rb_nhub, __popcll(mm));
  base = __shfl(base, 0, kWave);
  if (e) hlist[base + rank_below(mm)] = v;
}

template <int G, bool UNIT>
__global__ __launch_bounds__(256) void k_rb_hub_accum(
    const int32_t *__restrict__ part, const int64_t *__restrict__ voff, const int32_t *__restrict__ inc,
    const int32_t *__restrict__ nw, const uint64_t *__restrict__ ns, const int32_t *__restrict__ hlist, int32_t k,
    int32_t H, const DevStatus *st, int32_t *__restrict__ acc, const LoopCtl *lc) {
  JET_GATE(lc, kPhRb);
  constexpr int NG = 256 / G;
  __shared__ int32_t cs[NG][8 * G];
  __shared__ int32_t bsum[NG];
  const int32_t nh = st->rb_nhub;
  if (nh == 0) return;
  const int tid = threadIdx.x, gi = tid / G, lg = tid % G;
  const int32_t per = nh >= (int32_t)gridDim.x ? 1 : (int32_t)gridDim.x / nh;  // blocks per hub
  const int32_t first = (int32_t)blockIdx.x / per, sub = (int32_t)blockIdx.x % per;
  const int32_t step = nh >= (int32_t)gridDim.x ? (int32_t)gridDim.x : nh;
  for (int32_t j = first; j < nh; j += step) {  // block-uniform trip count
    const int32_t v = hlist[j];
    const int32_t s = part[v];
    int32_t conn[8];
#pragma unroll
    for (int x = 0; x < 8; ++x) conn[x] = 0;
    int32_t benefit = 0;
    const int64_t q0 = voff[v], q1 = voff[v + 1];
    if (G == 1)
      conn_accumulate_strided<G, UNIT>(inc, q0 + (int64_t)sub * NG + gi, q1, (int64_t)per * NG, nw, ns, lg, s, conn,
                                       benefit);
    else
      conn_accumulate<G, UNIT>(inc, q0 + ((int64_t)sub * NG + gi) * G, q1, (int64_t)per * NG * G, nw, ns, lg, s,
                               conn, benefit);
#pragma unroll
    for (int x = 0; x < 8; ++x) cs[gi][lg * 8 + x] = conn[x];
    if ((s >> 3) == lg) bsum[gi] = benefit;
    __syncthreads();
    if (tid < k) {
      int32_t tot = 0;
      for (int g = 0; g < NG; ++g) tot += cs[g][tid];
      if (tot) atomicAdd(&acc[(size_t)tid * H + j], tot);
    }
    if (tid == k) {
      int32_t ben = 0;
      for (int g = 0; g < NG; ++g) ben += bsum[g];
      if (ben) atomicAdd(&acc[(size_t)k * H + j], ben);
    }
    __syncthreads();  // LDS reused by the next hub
  }
}

__global__ __launch_bounds__(256) void k_rb_hub_finish(
    const int32_t *__restrict__ part, const int64_t *__restrict__ voff, const int32_t *__restrict__ sumw,
    const int32_t *__restrict__ vw, const int32_t *__restrict__ hlist, int32_t k, int32_t H, int64_t lmax, int64_t dz,
    DevStatus *st, int32_t *__restrict__ acc, uint32_t *__restrict__ entries, const LoopCtl *lc, Union u) {
  JET_GATE(lc, kPhRb);
  if (lc && !u.lcs) dz = lc->dz;
  __shared__ int64_t bw[kMaxK];
  __shared__ int32_t lcnt[kMaxK], lbase[kMaxK];
  __shared__ unsigned long long scanned, examined, emitted;
  const int32_t nh = st->rb_nhub;
  if (nh == 0) return;
  const int tid = threadIdx.x;
  for (int b = tid; b < k; b += 256) bw[b] = st->bw[b];
  if (tid == 0) {
    scanned = 0ull;
    examined = 0ull;
    emitted = 0ull;
  }
  const int32_t ntiles = (nh + 255) / 256;
  for (int32_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {  // block-uniform trip count
    for (int b = tid; b < k; b += 256) lcnt[b] = 0;
    __syncthreads();
    const int32_t j = tile * 256 + tid;
    const bool e = j < nh;
    int32_t v = 0, s = 0, c = 1, ben = 0;
    int64_t lm = lmax, dzz = dz, sg0 = 0;  // union: the hub's hypergraph's limits and segments
    int32_t unw = (lc && !u.lcs) ? lc->rb_unw : 0;
    // best valid target (balanced with v added, outside the deadzone) by conn, lowest block on ties
    int32_t bestc = -1, bestb = 0;
    if (e) {
      v = hlist[j];
      s = part[v];
      c = vw ? vw[v] : 1;
      if (u.lcs) {
        const int32_t hg = u.vhg[v];
        lm = u.lcs[hg].lmax;
        dzz = u.lcs[hg].dz;
        sg0 = (int64_t)hg * k;
        unw = u.lcs[hg].rb_unw;
      }
      for (int32_t b0 = 0; b0 < k; b0 += 16) {  // 16 loads in flight before any is used
        int32_t cb[16];
#pragma unroll
        for (int x = 0; x < 16; ++x) cb[x] = b0 + x < k ? acc[(size_t)(b0 + x) * H + j] : -1;
#pragma unroll
        for (int x = 0; x < 16; ++x) {
          const int32_t b = b0 + x;
          if (b < k) acc[(size_t)b * H + j] = 0;
          const int64_t bwb = b < k ? (u.lcs ? st->bw[sg0 + b] : bw[b]) : 0;
          if (b < k && b != s && bwb + c <= lm && bwb < dzz && cb[x] > bestc) {
            bestc = cb[x];
            bestb = b;
          }
        }
      }
      ben = acc[(size_t)k * H + j];
      acc[(size_t)k * H + j] = 0;
    }
    const bool emit = e && bestc >= 0;
    int32_t local = 0;
    int64_t uslot = 0;
    if (emit) {
      if (u.lcs) uslot = st->rb_off[sg0 + s] + atomicAdd(&st->rb_count[sg0 + s], 1);  // union: per segment
      else local = atomicAdd(&lcnt[s], 1);
      atomicAdd(&emitted, 1ull);
    }
    if (e) {
      atomicAdd(&scanned, (unsigned long long)(voff[v + 1] - voff[v]));
      atomicAdd(&examined, 1ull);
    }
    __syncthreads();
    for (int b = tid; b < k; b += 256)
      if (lcnt[b]) lbase[b] = atomicAdd(&st->rb_count[b], lcnt[b]);
    __syncthreads();
    if (emit) {
      const int32_t g = bestc - (sumw[v] - ben);
      uint32_t key5[5];
      entry_key(g, c, v, unw, key5);
      uint32_t *ent = entries + (u.lcs ? uslot : st->rb_off[s] + lbase[s] + local) * kEntryWords;
#pragma unroll
      for (int i = 0; i < 5; ++i) ent[i] = key5[i];
      ent[5] = (uint32_t)v;
      ent[6] = (uint32_t)bestb;
      ent[7] = (uint32_t)c;
    }
  }
  __syncthreads();
  if (tid == 0 && examined) {
    atomicAdd((unsigned long long *)&st->rb_inc, scanned);
    atomicAdd((unsigned long long *)&st->rb_elig, examined);
    if (emitted) atomicAdd((unsigned long long *)&st->rb_ent, emitted);
  }
}

constexpr int kSelThreads = 1024;
constexpr int kSelPer = 4;  // list entries per thread and tile in the selection's emit / keep sweeps

__device__ __forceinline__ uint32_t digit_of(const uint32_t *key, int d) {
  return (key[d >> 2] >> (8 * (3 - (d & 3)))) & 0xffu;
}

// Writes one selected entry as a move of vertex ent[5] from block `from` to ent[6].
__device__ __forceinline__ void put_move(const uint32_t *ent, int32_t from, int32_t pos, int4 *moves,
                                         int32_t *sel_target, uint8_t *mvto) {
  moves[pos] = make_int4((int32_t)ent[5], from, (int32_t)ent[6], (int32_t)ent[7]);
  mvto[ent[5]] = (uint8_t)ent[6];
  if (sel_target) sel_target[ent[5]] = (int32_t)ent[6];
}

// Threshold of one radix pass, computed by the 64 lanes of one wave: the largest digit dg whose
// weight at or above it, sum_{j >= dg} hw[j], reaches the remaining need nr.  Lane l holds the four
// bins of group 63 - l, so an inclusive scan over the lanes gives each group's suffix sum; the
// first lane whose suffix reaches the need owns the threshold.  When the whole weight is at most
// the need (only possible before the first selection), every entry with a weight is emitted:
// thr 0, done.  Otherwise done when the threshold digit's weight is exactly the rest of the need
// or a single entry holds it.  One lane writes the results.
__device__ __forceinline__ void pass_threshold(const unsigned long long *hw, const int32_t *hc, int64_t nr,
                                               int32_t *s_thr, int64_t *s_need, int32_t *s_done) {
  const int lane = lane_id();
  const int g = kWave - 1 - lane;
  int64_t h[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) h[j] = (int64_t)hw[4 * g + j];
  const int64_t sg = h[0] + h[1] + h[2] + h[3];
  const int64_t suf = wave_incl_scan(sg);
  const int64_t total = __shfl(suf, kWave - 1, kWave);
  const uint64_t reach = ballot(suf >= nr);
  if (total <= nr) {
    if (lane == 0) {
      *s_thr = 0;
      *s_done = 1;
    }
  } else if (lane == (int)__builtin_ctzll(reach)) {
    int64_t cum = suf - sg;
    int thr = 4 * g;
#pragma unroll
    for (int j = 3; j >= 0; --j) {
      if (cum + h[j] >= nr) {
        thr = 4 * g + j;
        break;
      }
      cum += h[j];
    }
    const int64_t rem = nr - cum;
    *s_thr = thr;
    *s_need = rem;
    *s_done = ((int64_t)hw[thr] == rem || hc[thr] == 1) ? 1 : 0;
  }
}

// ---- the first radix pass over all CUs (large levels) ----
// The first pass of the selection over an overloaded block's entries runs on S workgroups per
// block (slice s of the block's list each, grid S x k; blocks without need exit at once):
// k_rb_sel_hist adds the histogram of the first key byte into hist[b]; k_rb_sel_split derives the
// same threshold from it in every workgroup, emits the entries above the threshold byte (and on
// it, when that completes the selection) and compacts the entries on the threshold byte into the
// block's region of keep2.  The single-workgroup selection then continues from the second byte
// over the kept entries; it clears hist[b] again.
constexpr int kSplitThreads = 256;  // one thread per histogram bin

__device__ __forceinline__ void slice_range(int32_t len, int s, int S, int32_t &lo, int32_t &hi) {
  lo = (int32_t)((int64_t)len * s / S);
  hi = (int32_t)((int64_t)len * (s + 1) / S);
}

__global__ __launch_bounds__(kSplitThreads) void k_rb_sel_hist(const uint32_t *__restrict__ entries,
                                                               const DevStatus *st, unsigned long long *__restrict__ gw,
                                                               uint32_t *__restrict__ gc, const LoopCtl *lc) {
  JET_GATE(lc, kPhRb);
  __shared__ unsigned long long hw[256];
  __shared__ uint32_t hc[256];
  const int b = blockIdx.y, tid = threadIdx.x;
  if (st->rb_need[b] <= 0) return;
  int32_t lo, hi;
  slice_range(st->rb_count[b], blockIdx.x, gridDim.x, lo, hi);
  if (lo >= hi) return;
  const uint32_t *list = entries + st->rb_off[b] * kEntryWords;
  hw[tid] = 0ull;
  hc[tid] = 0u;
  __syncthreads();
  for (int32_t ib = lo + tid; ib < hi; ib += kSplitThreads * 4) {  // four entries' loads in flight
    uint32_t wt[4], k0[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int32_t i = ib + u * kSplitThreads;
      wt[u] = 0u;
      k0[u] = 0u;
      if (i < hi) {
        wt[u] = list[(int64_t)i * kEntryWords + 7];
        k0[u] = list[(int64_t)i * kEntryWords];
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (wt[u] == 0u) continue;  // a vertex without a valid target (or past the slice)
      atomicAdd(&hw[k0[u] >> 24], (unsigned long long)wt[u]);
      atomicAdd(&hc[k0[u] >> 24], 1u);
    }
  }
  __syncthreads();
  if (hc[tid]) {
    atomicAdd(&gw[(int64_t)b * 256 + tid], hw[tid]);
    atomicAdd(&gc[(int64_t)b * 256 + tid], hc[tid]);
  }
}

__global__ __launch_bounds__(kSplitThreads) void k_rb_sel_split(
    const uint32_t *__restrict__ entries, uint32_t *__restrict__ keep2, DevStatus *st,
    const unsigned long long *__restrict__ gw, const uint32_t *__restrict__ gc, int4 *__restrict__ moves,
    int32_t *__restrict__ sel_target, uint8_t *__restrict__ mvto, const int64_t *__restrict__ voff,
    int32_t *__restrict__ bigmv, const LoopCtl *lc) {
  JET_GATE(lc, kPhRb);
  __shared__ unsigned long long hw[256];
  __shared__ int32_t hc[256];
  __shared__ int32_t s_thr, s_done, s_ebase, s_kbase;
  __shared__ int64_t s_need;
  __shared__ int32_t sm[kSplitThreads / kWave + 1];
  __shared__ unsigned long long s_deg;
  const int b = blockIdx.y, tid = threadIdx.x;
  const int64_t need = st->rb_need[b];
  if (need <= 0) return;
  int32_t lo, hi;
  slice_range(st->rb_count[b], blockIdx.x, gridDim.x, lo, hi);
  if (lo >= hi) return;
  const uint32_t *list = entries + st->rb_off[b] * kEntryWords;
  uint32_t *kept = keep2 + st->rb_off[b] * kEntryWords;
  hw[tid] = gw[(int64_t)b * 256 + tid];
  hc[tid] = (int32_t)gc[(int64_t)b * 256 + tid];
  if (tid == 0) s_deg = 0ull;
  __syncthreads();
  if (tid < kWave) pass_threshold(hw, hc, need, &s_thr, &s_need, &s_done);
  __syncthreads();
  const uint32_t thr = (uint32_t)s_thr;
  const bool done = s_done != 0;
  unsigned long long deg = 0ull;
  for (int32_t tb = lo; tb < hi; tb += kSplitThreads * kSelPer) {  // block-uniform trip count
    uint32_t ent[kSelPer][kEntryWords];
    uint32_t emit = 0u, keep = 0u;
#pragma unroll
    for (int j = 0; j < kSelPer; ++j) {
      const int32_t i = tb + j * kSplitThreads + tid;
      if (i < hi) {
#pragma unroll
        for (int w = 0; w < kEntryWords; ++w) ent[j][w] = list[(int64_t)i * kEntryWords + w];
        if (ent[j][7] == 0u) continue;  // a vertex without a valid target: dropped
        const uint32_t dg = ent[j][0] >> 24;
        if (dg > thr || (dg == thr && done)) emit |= 1u << j;
        else if (dg == thr) keep |= 1u << j;
      }
    }
    int32_t tot;
    const int32_t rk =
        block_excl_scan<kSplitThreads>((int32_t)(__popc(emit) | (__popc(keep) << 16)), sm, &tot);
    const int32_t etot = tot & 0xffff, ktot = tot >> 16;
    if (tid == 0) {
      s_ebase = etot ? atomicAdd(&st->n_moves, etot) : 0;
      s_kbase = ktot ? atomicAdd(&st->rb_kept[b], ktot) : 0;
    }
    __syncthreads();
    int32_t pos = s_ebase + (rk & 0xffff), kp = s_kbase + (rk >> 16);
#pragma unroll
    for (int j = 0; j < kSelPer; ++j) {
      const bool e = (emit >> j) & 1u;
      int64_t d = 0;
      if (e) {
        d = voff[ent[j][5] + 1] - voff[ent[j][5]];
        put_move(ent[j], b, pos, moves, sel_target, mvto);
      }
      push_big_move(d > kLaneDegree, pos, st, bigmv);
      pos += e ? 1 : 0;
      deg += (unsigned long long)d;
      if ((keep >> j) & 1u) {
#pragma unroll
        for (int w = 0; w < kEntryWords; ++w) kept[(int64_t)kp * kEntryWords + w] = ent[j][w];
        ++kp;
      }
    }
    __syncthreads();  // s_ebase and s_kbase are rewritten by the next tile
  }
  deg = wave_sum(deg);
  if (lane_id() == 0 && deg) atomicAdd(&s_deg, deg);
  __syncthreads();
  if (tid == 0 && s_deg) atomicAdd((unsigned long long *)&st->mv_inc, s_deg);
}

// One block per overloaded block b: selects the minimal prefix of b's entries in key order whose
// weight reaches rb_need[b] (all entries if their total falls short).  Radix selection over the
// 20 key bytes, most significant first; each pass emits the entries above the threshold digit and
// keeps those on it.  Passes whose digit is shared by every remaining entry change nothing and
// only cost the histogram; when the remaining entries share words 1..3 those 12 passes are
// skipped outright.  Emitted moves take their slots with one reservation per tile of the list,
// and their incidence total is added to mv_inc once at the end.  With gw / gc (the first-byte
// histograms of the grid-wide first pass) the first pass has already run: the kernel rederives
// its threshold, clears the histogram, and continues from the second byte over the entries that
// pass kept in keep2 (nothing is left to do when it completed the selection).
__device__ __forceinline__ void select_segment(const int32_t sgm, uint32_t *__restrict__ entries, DevStatus *st,
                                               int4 *__restrict__ moves, int32_t *__restrict__ sel_target,
                                               uint8_t *__restrict__ mvto, const int64_t *__restrict__ voff,
                                               int32_t *__restrict__ bigmv, unsigned long long *__restrict__ gw,
                                               uint32_t *__restrict__ gc, uint32_t *__restrict__ keep2, int32_t k,
                                               const Union &u) {
  __shared__ unsigned long long hw[256];
  __shared__ int32_t hc[256];
  __shared__ int32_t s_thr, s_done, s_len, s_same, s_base;
  __shared__ int64_t s_need;
  __shared__ unsigned long long s_deg;
  __shared__ int32_t s_emitted;
  __shared__ int32_t scan_sm[2][kSelThreads / kWave];
  int parity = 0;
  const int32_t b = sgm % k;        // the block the selected vertices leave
  const int tid = threadIdx.x;
  int64_t need = st->rb_need[sgm];
  if (need <= 0) return;
  uint32_t *list = entries + st->rb_off[sgm] * kEntryWords;
  int32_t len = st->rb_count[sgm];
  int d0 = 0;
  if (gw) {  // the first pass ran over all CUs: continue from the second byte over the kept entries
    for (int i = tid; i < 256; i += kSelThreads) {
      hw[i] = gw[(int64_t)b * 256 + i];
      hc[i] = (int32_t)gc[(int64_t)b * 256 + i];
      gw[(int64_t)b * 256 + i] = 0ull;
      gc[(int64_t)b * 256 + i] = 0u;
    }
    __syncthreads();
    if (tid < kWave) pass_threshold(hw, hc, need, &s_thr, &s_need, &s_done);
    __syncthreads();
    if (s_done) return;  // the split pass emitted the whole selection
    need = s_need;
    list = keep2 + st->rb_off[sgm] * kEntryWords;
    len = st->rb_kept[sgm];
    d0 = 1;
    __syncthreads();  // every thread has read s_need and s_done before they are rewritten
  }
  if (len == 0) return;
  // One tile: kSelPer entries per thread (entry tb + j * kSelThreads + tid).  Emits those with
  // bit j of `emit` set and compacts those with bit j of `keep` to list[out..]; returns the number
  // kept.  Every thread of the block calls it, after loading its entries.
  auto emit_keep = [&](uint32_t emit, uint32_t keep, const uint32_t (*ent)[kEntryWords], int32_t out) -> int32_t {
    const int32_t ne = __popc(emit), nk = __popc(keep);
    // block-wide exclusive scan with one barrier: the wave totals go to the half of scan_sm this
    // tile owns (tiles alternate), so no barrier is needed before the next tile writes
    const int32_t x = ne | (nk << 16);
    const int32_t inc = wave_incl_scan(x);
    int32_t *ws = scan_sm[parity];
    parity ^= 1;
    if (lane_id() == kWave - 1) ws[tid / kWave] = inc;
    __syncthreads();
    int32_t off = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kSelThreads / kWave; ++i) {
      const int32_t v = ws[i];
      off += i < tid / kWave ? v : 0;
      tot += v;
    }
    const int32_t rk = inc - x + off;
    const int32_t etot = tot & 0xffff;
    if (etot) {  // block-uniform
      if (tid == 0) {
        s_base = atomicAdd(&st->n_moves, etot);
        s_emitted += etot;
      }
      __syncthreads();
      int32_t pos = s_base + (rk & 0xffff);
      int64_t dsum = 0;
#pragma unroll
      for (int j = 0; j < kSelPer; ++j) {
        int64_t d = 0;
        const bool e = (emit >> j) & 1u;
        if (e) {
          d = voff[ent[j][5] + 1] - voff[ent[j][5]];
          put_move(ent[j], b, pos, moves, sel_target, mvto);
        }
        push_big_move(d > kLaneDegree, pos, st, bigmv);
        pos += e ? 1 : 0;
        dsum += d;
      }
      const int64_t wd = wave_sum(dsum);
      if (lane_id() == 0 && wd) atomicAdd(&s_deg, (unsigned long long)wd);
    }
    int32_t kp = out + (rk >> 16);
#pragma unroll
    for (int j = 0; j < kSelPer; ++j) {
      if ((keep >> j) & 1u) {
#pragma unroll
        for (int w = 0; w < kEntryWords; ++w) list[(int64_t)kp * kEntryWords + w] = ent[j][w];
        ++kp;
      }
    }
    // s_base is read above, before this thread reaches the next tile's barrier; the next tile reads
    // list slots at or beyond this tile's end, which no thread of this tile writes
    return tot >> 16;
  };
  if (tid == 0) {
    s_deg = 0ull;
    s_emitted = 0;
    s_need = need;
    s_len = len;
  }
  for (int d = d0; d < 20; ++d) {
    __syncthreads();  // every thread has finished reading the previous pass's histogram
    len = s_len;
    if (d == 4) {  // do the remaining entries share the exact rational part of the key?
      if (tid == 0) s_same = 1;
      __syncthreads();
      const uint32_t r1 = list[1], r2 = list[2], r3 = list[3];
      for (int32_t i = tid; i < len; i += kSelThreads) {
        const uint32_t *ent = list + (int64_t)i * kEntryWords;
        if (ent[1] != r1 || ent[2] != r2 || ent[3] != r3) s_same = 0;
      }
      __syncthreads();
      if (s_same) d = 16;
    }
    for (int i = tid; i < 256; i += kSelThreads) {
      hw[i] = 0;
      hc[i] = 0;
    }
    __syncthreads();
    for (int32_t i = tid; i < len; i += kSelThreads) {
      const uint32_t *ent = list + (int64_t)i * kEntryWords;
      if (ent[7] == 0u) continue;  // a vertex without a valid target
      const uint32_t dg = digit_of(ent, d);
      atomicAdd(&hw[dg], (unsigned long long)ent[7]);
      atomicAdd(&hc[dg], 1);
    }
    __syncthreads();
    if (tid < kWave) pass_threshold(hw, hc, s_need, &s_thr, &s_need, &s_done);
    __syncthreads();
    const uint32_t thr = (uint32_t)s_thr;
    const bool done = s_done != 0;
    if (!done && hc[thr] == len) continue;  // every entry on the threshold digit: nothing changes
    // emit entries above the threshold digit, keep (or emit, when done) those on it
    int32_t out = 0;
    for (int32_t tb = 0; tb < len; tb += kSelThreads * kSelPer) {
      uint32_t ent[kSelPer][kEntryWords];
      uint32_t emit = 0, keep = 0;
#pragma unroll
      for (int j = 0; j < kSelPer; ++j) {
        const int32_t i = tb + j * kSelThreads + tid;
        if (i < len) {
#pragma unroll
          for (int w = 0; w < kEntryWords; ++w) ent[j][w] = list[(int64_t)i * kEntryWords + w];
          const uint32_t dg = digit_of(ent[j], d);
          if (ent[j][7] == 0u) continue;  // a vertex without a valid target: dropped
          if (dg > thr || (dg == thr && done)) emit |= 1u << j;
          if (!done && dg == thr) keep |= 1u << j;
        }
      }
      out += emit_keep(emit, keep, ent, out);
    }
    if (done) break;
    if (tid == 0) s_len = out;
  }
  __syncthreads();
  if (tid == 0 && s_deg) atomicAdd((unsigned long long *)&st->mv_inc, s_deg);
  if (tid == 0 && u.lcs && s_emitted) atomicAdd(&st->hmoves[sgm / k], s_emitted);  // union: per hypergraph
}

// One workgroup per overloaded block: the block's segment (one hypergraph).  A union's workgroups
// walk the segments of the hypergraphs in their rebalancing phase.
__global__ __launch_bounds__(kSelThreads) void k_rb_select(uint32_t *__restrict__ entries, DevStatus *st,
                                                           int4 *__restrict__ moves, int32_t *__restrict__ sel_target,
                                                           uint8_t *__restrict__ mvto,
                                                           const int64_t *__restrict__ voff,
                                                           int32_t *__restrict__ bigmv,
                                                           unsigned long long *__restrict__ gw,
                                                           uint32_t *__restrict__ gc, uint32_t *__restrict__ keep2,
                                                           const LoopCtl *lc, int32_t k, Union u) {
  JET_GATE(lc, kPhRb);
  if (!u.lcs) {
    select_segment(blockIdx.x, entries, st, moves, sel_target, mvto, voff, bigmv, gw, gc, keep2, k, u);
    return;
  }
  const int32_t nseg = st->rb_nseg;  // the overloaded segments, listed by the preparation
  for (int32_t x = blockIdx.x; x < nseg; x += gridDim.x) {  // block-uniform trip count
    select_segment(st->rb_seg[x], entries, st, moves, sel_target, mvto, voff, bigmv, gw, gc, keep2, k, u);
    __syncthreads();  // shared state is reused by the next segment
  }
}

inline unsigned grid_for(int64_t work, int block, int64_t cap) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

template <int G, bool UNIT>
hipError_t gain_launch(Ctx &c, const int32_t *part, int64_t dz, const LoopCtl *lc) {
  constexpr int BLOCK = (G == 16) ? 512 : 256;
  constexpr int VPB = BLOCK / G;
  const Union u = union_of(c);
  if (c.H > 1)
    hipLaunchKernelGGL(k_rb_list_union, dim3(grid_for(c.n, 8 * kUnionTile, c.grid_cap)), dim3(kUnionTile), 0, c.stream, part, c.vw, c.voff,
                       c.n, c.k, c.st, c.rb_list, c.rb_slot, lc, u);
  else
    hipLaunchKernelGGL(k_rb_list, dim3((unsigned)((c.n + kListBlock * kListPer - 1) / (kListBlock * kListPer))),
                       dim3(kListBlock), 0, c.stream, part, c.vw, c.voff, c.n, c.k, c.lmax, c.A, c.st, c.rb_list,
                       c.rb_slot, lc);
  // the list length is known on the device only: a persistent grid walks it; unit net weights and
  // k <= 64 take the bit-sliced kernel (one lane per vertex on light levels, eight otherwise) on
  // a context of one hypergraph
  if (c.H == 1 && UNIT && c.k <= 64 && c.p_low < (int64_t)c.lane_degree * c.n_low) {
    hipLaunchKernelGGL(k_rb_gain_bits<1>, dim3((unsigned)std::min<int64_t>(c.grid_cap, (c.n + 255) / 256)), dim3(256), 0,
                       c.stream, part, c.voff, c.inc, c.ns, c.sumw, c.vw, c.rb_list, c.rb_slot, c.k, c.lmax, dz, c.st,
                       c.rb_keys, lc, c.rb_xcd);
  } else if (c.H == 1 && UNIT && c.k <= 64) {
    hipLaunchKernelGGL(k_rb_gain_bits<8>, dim3((unsigned)std::min<int64_t>(c.grid_cap, (c.n + 31) / 32)), dim3(256), 0,
                       c.stream, part, c.voff, c.inc, c.ns, c.sumw, c.vw, c.rb_list, c.rb_slot, c.k, c.lmax, dz, c.st,
                       c.rb_keys, lc, c.rb_xcd);
  } else {
    const unsigned grid = (unsigned)std::min<int64_t>(c.grid_cap, (c.n + VPB - 1) / VPB);
    hipLaunchKernelGGL((k_rb_gain<G, UNIT>), dim3(grid), dim3(BLOCK), 0, c.stream, part, c.voff, c.inc, c.nw, c.ns,
                       c.sumw, c.vw, c.rb_list, c.rb_slot, c.k, c.lmax, dz, c.st, c.rb_keys, lc, u, c.rb_xcd);
  }
  if (c.nhubs > 0) {
    hipLaunchKernelGGL(k_rb_hub_list, dim3((unsigned)((c.nhubs + 255) / 256)), dim3(256), 0, c.stream, part, c.vw,
                       c.hubs, c.nhubs, c.lmax, c.A, c.st, c.rb_hlist, lc, c.k, u);
    hipLaunchKernelGGL((k_rb_hub_accum<G, UNIT>), dim3(2048), dim3(256), 0, c.stream, part, c.voff, c.inc, c.nw, c.ns,
                       c.rb_hlist, c.k, c.nhubs, c.st, c.rb_hacc, lc);
    hipLaunchKernelGGL(k_rb_hub_finish, dim3(grid_for(c.nhubs, 256, 2048)), dim3(256), 0, c.stream, part, c.voff,
                       c.sumw, c.vw, c.rb_hlist, c.k, c.nhubs, c.lmax, dz, c.st, c.rb_hacc, c.rb_keys, lc, u);
  }
  return hipGetLastError();
}

template <bool UNIT>
hipError_t gain_dispatch(Ctx &c, const int32_t *part, int64_t dz, const LoopCtl *lc) {
  if (c.k <= 8) return gain_launch<1, UNIT>(c, part, dz, lc);
  if (c.k <= 16) return gain_launch<2, UNIT>(c, part, dz, lc);
  if (c.k <= 32) return gain_launch<4, UNIT>(c, part, dz, lc);
  if (c.k <= 64) return gain_launch<8, UNIT>(c, part, dz, lc);
  return gain_launch<16, UNIT>(c, part, dz, lc);
}

}  // namespace

hipError_t launch_rebalance_round(Ctx &c, const int32_t *part, int64_t dz, int32_t *sel_target,
                                  const LoopCtl *lc) {
  const int32_t want = lc ? (int32_t)kPhRb : (int32_t)kPhAny;
  if (c.H > 1)
    hipLaunchKernelGGL(k_rb_prepare_union, dim3(1), dim3(kPrepThreads), 0, c.stream, c.k, c.H, c.st, lc,
                       union_of(c));
  else
    hipLaunchKernelGGL(k_rb_prepare, dim3(1), dim3(kMaxK), 0, c.stream, c.k, c.lmax, c.st, lc);
  hipError_t e = hipGetLastError();
  // k_rb_prepare cleared the move list and the gain-pass counters
  if (e != hipSuccess) return e;
  int tok = prof_begin(c, kProfRbGain, lc, want);
  e = c.unit_nw ? gain_dispatch<true>(c, part, dz, lc) : gain_dispatch<false>(c, part, dz, lc);
  // 12 B per vertex, plus on the device: examined vertices, written entries, scanned incidences
  prof_end(c, tok, lc, want, 12.0 * c.n, 8.0 + (c.k + 7) / 8 + (c.unit_nw ? 0.0 : 4.0));
  if (e != hipSuccess) return e;
  tok = prof_begin(c, kProfRbSelect, lc, want);
  const bool split = c.H == 1 && c.n >= c.sel_split_min;
  if (split) {
    // about 2,048 entries of an average block per workgroup (an overloaded block lists at most its
    // vertices), or the set count (1..64); any S works, a workgroup whose slice is empty exits
    const unsigned S = c.sel_slices > 0 ? (unsigned)c.sel_slices
                                        : (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, (c.n / c.k + 2047) / 2048));
    hipLaunchKernelGGL(k_rb_sel_hist, dim3(S, (unsigned)c.k), dim3(kSplitThreads), 0, c.stream, c.rb_keys, c.st,
                       c.rb_gw, c.rb_gc, lc);
    hipLaunchKernelGGL(k_rb_sel_split, dim3(S, (unsigned)c.k), dim3(kSplitThreads), 0, c.stream, c.rb_keys,
                       c.rb_keys2, c.st, c.rb_gw, c.rb_gc, c.moves, sel_target, c.mvto, c.voff, c.bigmv, lc);
  }
  hipLaunchKernelGGL(k_rb_select, dim3(c.H > 1 ? (unsigned)std::min<int64_t>(512, (int64_t)c.H * c.k) : (unsigned)c.k),
                     dim3(kSelThreads), 0, c.stream, c.rb_keys, c.st,
                     c.moves, sel_target, c.mvto, c.voff, c.bigmv, split ? c.rb_gw : nullptr,
                     split ? c.rb_gc : nullptr, c.rb_keys2, lc, c.k, union_of(c));
  prof_end(c, tok, lc, want, 0.0, 0.0);  // bytes from the entry and move counts (device)
  return hipGetLastError();
}

}  // namespace jet
