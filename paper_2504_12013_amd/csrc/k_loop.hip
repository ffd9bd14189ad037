// The Jet loop of Algorithm 1 kept on the device.  The decisions of the loop (rebalance or not,
// strict improvement of the key (overload, metric), snapshot, iteration limit, fixed point, end of a
// temperature round and rollback to its best partition) are taken by small control kernels on a
// loop record (LoopCtl); every kernel of the iteration returns at once unless the record is in the
// phase it belongs to.  One iteration's launches -- the Jet phase, rb_slots rebalancing rounds, the
// end of the iteration and the rollback -- form a "tick"; the host captures a tick in a HIP graph
// once per context and replays it several times between two looks at the record.  Ticks after the
// loop finished do nothing.  The sequence of states is exactly that of the host loop it replaces
// (one Jet phase, then rebalancing rounds while a block is overloaded, a round moved something
// and the cap allows, then the key), so results and per-iteration records do not depend on how
// many ticks run between polls.
#include <algorithm>

#include "dev_util.h"
#include "jet_internal.h"

namespace jet {

namespace {

// Per-hypergraph views of the status block: one hypergraph (H == 1) keeps its metric in st->km1
// plus spread slots and its move count in st->n_moves; a union keeps them per hypergraph.
struct HgStatus {
  DevStatus *st;
  int32_t H, k;

  __device__ int64_t overload(int32_t hg, int64_t lmax) const {
    int64_t worst = 0;
    const int64_t *bw = st->bw + (int64_t)hg * k;
    for (int b = 0; b < k; ++b) worst = max(worst, bw[b] - lmax);
    return worst;
  }
  // the metric after folding the changes accumulated since the last fold
  __device__ int64_t fold(LoopCtl &r, int32_t hg) const {
    if (H == 1) {
      int64_t s = st->km1;
      for (int i = 0; i < kKm1Slots; ++i) {
        s += st->km1_slot[i];
        st->km1_slot[i] = 0;
      }
      st->km1 = s;
      r.km1 = s;
    } else {
      r.km1 += st->hkm1[hg];
      st->hkm1[hg] = 0;
    }
    return r.km1;
  }
  __device__ int32_t moves(int32_t hg) const { return H == 1 ? st->n_moves : st->hmoves[hg]; }
  __device__ int32_t cand() const { return H == 1 ? st->n_cand : 0; }
};

constexpr int kCtlThreads = 256;

// Union: the lists of hypergraphs per phase (and of those whose iteration improved), with the
// prefix sums of their tiles and chunks, in hypergraph order (one workgroup, block scans).
__device__ __forceinline__ void build_lists(const LoopCtl *lcs, int32_t H, ActList *act, const int32_t *ht0,
                                            const int32_t *hch0) {
  __shared__ int32_t sm[kCtlThreads / kWave + 1];
  __shared__ int32_t cn[kActLists], ct[kActLists], cc[kActLists];
  const int tid = threadIdx.x;
  if (tid < kActLists) cn[tid] = ct[tid] = cc[tid] = 0;
  __syncthreads();
  for (int32_t base = 0; base < H; base += kCtlThreads) {  // block-uniform trip count
    const int32_t hg = base + tid;
    const bool valid = hg < H;
    int32_t ph = kPhDone, imp = 0, tcnt = 0, ccnt = 0;
    if (valid) {
      ph = lcs[hg].phase;
      imp = lcs[hg].improved;
      tcnt = ht0[hg + 1] - ht0[hg];
      ccnt = hch0[hg + 1] - hch0[hg];
    }
    for (int L = 0; L < kActLists; ++L) {
      const bool in = valid && (L == kActImproved ? imp != 0 : ph == (L == kActJet ? kPhJet : L == kActRb ? kPhRb : kPhRoll));
      int32_t tn, tt, tc;
      const int32_t rn = block_excl_scan<kCtlThreads>(in ? 1 : 0, sm, &tn);
      const int32_t rt = block_excl_scan<kCtlThreads>(in ? tcnt : 0, sm, &tt);
      const int32_t rc = block_excl_scan<kCtlThreads>(in ? ccnt : 0, sm, &tc);
      if (in) {
        act[L].hg[cn[L] + rn] = hg;
        act[L].tpref[cn[L] + rn] = ct[L] + rt;
        act[L].cpref[cn[L] + rn] = cc[L] + rc;
      }
      __syncthreads();
      if (tid == 0) {
        cn[L] += tn;
        ct[L] += tt;
        cc[L] += tc;
      }
      __syncthreads();
    }
  }
  if (tid < kActLists) {
    act[tid].cnt = cn[tid];
    act[tid].tpref[cn[tid]] = ct[tid];
    act[tid].cpref[cn[tid]] = cc[tid];
  }
}

// Runs f(record, hg) for every hypergraph (one workgroup striding over them), then sets the gate
// record's phase mask and snapshot flag from all records (a union's gate is a record of its own)
// and rebuilds the union's lists.
template <typename F>
__device__ __forceinline__ void for_each_hg(LoopCtl *lcs, int32_t H, LoopCtl *gate, Union u, F f) {
  __shared__ int32_t smask, simp;
  if (threadIdx.x == 0) {
    smask = 0;
    simp = 0;
  }
  __syncthreads();
  int32_t m = 0, imp = 0;
  for (int32_t hg = threadIdx.x; hg < H; hg += blockDim.x) {
    f(lcs[hg], hg);
    m |= lcs[hg].phase_mask;
    imp |= lcs[hg].improved;
  }
  if (m) atomicOr(&smask, m);
  if (imp) atomicOr(&simp, imp);
  __syncthreads();
  if (threadIdx.x == 0 && gate != lcs) {
    gate->phase_mask = smask;
    gate->improved = simp;
  }
  if (u.lcs) build_lists(lcs, H, const_cast<ActList *>(u.act), u.ht0, u.hch0);
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t count, uint32_t value, const LoopCtl *lc,
                           int32_t want) {
  JET_GATE(lc, want);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// Completes the records the host wrote (parameters, limits, stamp) from the state build_state left
// (metric, block weights): the first round's key and the first phase.
__global__ __launch_bounds__(kCtlThreads) void k_loop_init(LoopCtl *lcs, int32_t H, LoopCtl *gate, DevStatus *st,
                                                           int32_t k, Union u) {
  const HgStatus hs{st, H, k};
  for_each_hg(lcs, H, gate, u, [&](LoopCtl &r, int32_t hg) {
    if (H > 1) r.km1 = 0;
    const int64_t km1 = hs.fold(r, hg);
    const int64_t ovl = hs.overload(hg, r.lmax);
    r.km1_in = km1;
    r.best_ovl = ovl;
    r.best_km1 = km1;
    if (r.rb_only) set_phase(r, (ovl > 0 && r.max_rb > 0) ? kPhRb : kPhDone);  // jet_rebalance
    else set_phase(r, kPhJet);
  });
}

// Start of a piece: the snapshot flags of the previous piece are cleared.
__global__ __launch_bounds__(kCtlThreads) void k_tick_begin(LoopCtl *lcs, int32_t H, LoopCtl *gate, Union u) {
  for_each_hg(lcs, H, gate, u, [&](LoopCtl &r, int32_t) {
    r.improved = 0;
    if (r.phase != kPhDone) r.ticks += 1;
  });
}

// Start of a Jet phase (launched only where the phase follows): a new iteration stamp, so the
// vertices moved by the previous iteration's Jet phase (stamped stamp - 1) are the locked ones.
__global__ __launch_bounds__(kCtlThreads) void k_jet_begin(LoopCtl *lcs, int32_t H, LoopCtl *gate, Union u) {
  for_each_hg(lcs, H, gate, u, [&](LoopCtl &r, int32_t) {
    if (r.phase != kPhJet) return;
    r.stamp += 1;
    r.lock_was_any = r.lock_any;
  });
}

// After the Jet phase's moves are applied: its counts, the locks it leaves, and whether a
// rebalancing round follows (Algorithm 1: rebalance while a block is overloaded).
__global__ __launch_bounds__(kCtlThreads) void k_jet_post(LoopCtl *lcs, int32_t H, LoopCtl *gate, DevStatus *st,
                                                          int32_t k, Union u) {
  const HgStatus hs{st, H, k};
  for_each_hg(lcs, H, gate, u, [&](LoopCtl &r, int32_t hg) {
    if (r.phase != kPhJet) return;
    hs.fold(r, hg);
    const int32_t moved = hs.moves(hg);
    r.n_cand = hs.cand();
    r.n_moved = moved;
    r.lock_any = moved > 0 ? 1 : 0;
    r.moves_executed += moved;
    r.rb_rounds = 0;
    r.rb_moved = 0;
    set_phase(r, (hs.overload(hg, r.lmax) > 0 && r.max_rb > 0) ? kPhRb : kPhEnd);
  });
}

// After a rebalancing round's moves are applied: another round while a block is still overloaded,
// the round moved a vertex and the cap allows (Section 4.3).
__global__ __launch_bounds__(kCtlThreads) void k_rb_post(LoopCtl *lcs, int32_t H, LoopCtl *gate, DevStatus *st,
                                                         int32_t k, Union u) {
  const HgStatus hs{st, H, k};
  for_each_hg(lcs, H, gate, u, [&](LoopCtl &r, int32_t hg) {
    if (r.phase != kPhRb) return;
    hs.fold(r, hg);
    const int32_t moved = hs.moves(hg);
    r.rb_rounds += 1;
    r.rb_moved += moved;
    if (hs.overload(hg, r.lmax) == 0 || r.rb_rounds >= r.max_rb || moved == 0) {
      if (r.rb_only) {
        r.rebalance_rounds += r.rb_rounds;
        set_phase(r, kPhDone);
      } else {
        set_phase(r, kPhEnd);
      }
    }
  });
}

// End of an iteration: the key (overload, metric) against the round's best (strict, lexicographic),
// the iteration record, the limit of non-improving iterations, the round's cap and the fixed point.
__global__ __launch_bounds__(kCtlThreads) void k_iter_end(LoopCtl *lcs, int32_t H, LoopCtl *gate,
                                                          const DevStatus *st, int32_t k, jet_trace *trace, Union u) {
  const HgStatus hs{const_cast<DevStatus *>(st), H, k};
  for_each_hg(lcs, H, gate, u, [&](LoopCtl &r, int32_t hg) {
    if (r.phase != kPhEnd) return;
    const int64_t ovl = hs.overload(hg, r.lmax), km1 = r.km1;
    r.it += 1;
    r.round += 1;
    if (ovl < r.best_ovl || (ovl == r.best_ovl && km1 < r.best_km1)) {
      r.best_ovl = ovl;
      r.best_km1 = km1;
      r.improved = 1;
      r.round = 0;
    }
    r.iterations += 1;
    r.rebalance_rounds += r.rb_rounds;
    if (trace && H == 1 && r.ntrace < r.trace_cap) {
      jet_trace t;
      t.km1 = km1;
      t.overload = ovl;
      t.n_cand = r.n_cand;
      t.n_moved = r.n_moved;
      t.rb_rounds = r.rb_rounds;
      t.rb_moved = r.rb_moved;
      trace[r.ntrace] = t;
    }
    r.ntrace += 1;
    // nothing moved, nothing rebalanced and nothing was locked: the next iteration would repeat it
    const bool fixed = r.n_moved == 0 && r.rb_moved == 0 && r.lock_was_any == 0;
    set_phase(r, (r.round >= r.limit || r.it >= r.max_iters || fixed) ? kPhRoll : kPhJet);
  });
}

// The snapshot of an improving iteration (Algorithm 1's rollback point), per vertex of the
// hypergraphs whose iteration improved.
__global__ void k_snapshot(const int32_t *__restrict__ part, int32_t *__restrict__ best, int32_t n, const LoopCtl *lc,
                           Union u) {
  if (lc->improved == 0) return;
  if (u.lcs) {  // union: the tiles of the hypergraphs whose iteration improved
    const ActList &L = u.act[kActImproved];
    const int32_t nt = L.tpref[L.cnt];
    for (int32_t t = blockIdx.x; t < nt; t += gridDim.x) {
      const int64_t v = act_tile_base(L, u.ht0, t) + threadIdx.x;
      if (v < n) best[v] = part[v];
    }
    return;
  }
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    best[v] = part[v];
}

// After the rollback's moves are applied: the next temperature round starts from the round's
// best partition with no locks, or the loop is done.
__global__ __launch_bounds__(kCtlThreads) void k_roll_post(LoopCtl *lcs, int32_t H, LoopCtl *gate, DevStatus *st,
                                                           int32_t k, Union u) {
  const HgStatus hs{st, H, k};
  for_each_hg(lcs, H, gate, u, [&](LoopCtl &r, int32_t hg) {
    if (r.phase != kPhRoll) return;
    const int64_t km1 = hs.fold(r, hg);
    r.tau_r += 1;
    if (r.tau_r >= r.num_tau) {
      set_phase(r, kPhDone);
      return;
    }
    r.tau_q = r.tau_qs[r.tau_r];
    r.stamp += 2;  // the round's first iteration sees no lock
    r.round = 0;
    r.it = 0;
    r.lock_any = 0;
    r.best_ovl = hs.overload(hg, r.lmax);
    r.best_km1 = km1;
    set_phase(r, kPhJet);
  });
}

// Device timing marks of a kernel family: `end` == 0 stores the wall clock, `end` == 1 adds the
// elapsed ticks, one launch and the family's algorithmic bytes (static part plus the part the
// device counters give).  Gated like the family.
__global__ void k_prof_mark(DevProf *dp, const DevStatus *st, const LoopCtl *lc, int32_t want, int32_t fam,
                            int32_t end, double bytes, double per_inc) {
  JET_GATE(lc, want);
  if (threadIdx.x != 0) return;
  const unsigned long long now = wall_clock64();
  if (!end) {
    dp->t0[fam] = now;
    return;
  }
  double b = bytes;
  switch (fam) {
  case kProfCandidates: b += per_inc * (double)st->inc_low; break;
  case kProfCandidatesHub: b += per_inc * (double)st->inc_hub; break;
  case kProfAfterburner:  // per_inc is nonzero for the graph afterburner only
    if (per_inc > 0.0) b += per_inc * (double)st->ab_inc + 24.0 * (double)st->n_cand;
    break;
  case kProfApply: b += 5.0 * st->n_moves + 20.0 * (double)st->mv_inc; break;
  case kProfRbGain:
    b += 4.0 * (double)st->rb_elig + 32.0 * (double)st->rb_ent + per_inc * (double)st->rb_inc;
    break;
  case kProfRbSelect: b += 32.0 * (double)st->rb_ent + 8.0 * st->n_moves; break;
  default: break;
  }
  dp->ticks[fam] += now - dp->t0[fam];
  dp->launches[fam] += 1;
  dp->bytes[fam] += b;
}

inline unsigned grid_for(int64_t work, int block, int64_t cap) {
  int64_t g = (work + block - 1) / block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

}  // namespace

int prof_begin(Ctx &c, int fam, const LoopCtl *lc, int32_t want) {
  if (!c.prof || !((c.prof_mask >> fam) & 1u) || !c.dprof) return -1;
  hipLaunchKernelGGL(k_prof_mark, dim3(1), dim3(64), 0, c.stream, c.dprof, c.st, lc, want, fam, 0, 0.0, 0.0);
  return fam;
}

void prof_end(Ctx &c, int token, const LoopCtl *lc, int32_t want, double bytes, double per_inc) {
  if (token < 0) return;
  hipLaunchKernelGGL(k_prof_mark, dim3(1), dim3(64), 0, c.stream, c.dprof, c.st, lc, want, token, 1, bytes, per_inc);
}

hipError_t launch_fill_u32(Ctx &c, uint32_t *p, int64_t count, uint32_t value, const LoopCtl *lc, int32_t want) {
  hipLaunchKernelGGL(k_fill_u32, dim3(grid_for(count, 256, 1024)), dim3(256), 0, c.stream, p, count, value, lc, want);
  return hipGetLastError();
}

hipError_t launch_loop_init(Ctx &c) {
  hipLaunchKernelGGL(k_loop_init, dim3(1), dim3(kCtlThreads), 0, c.stream, c.lcs, c.H, c.lc, c.st, c.k, union_of(c));
  return hipGetLastError();
}

hipError_t launch_tick(Ctx &c, int kind) {
  const LoopCtl *lc = c.lc;
  const bool jet = kind == kTickJet || kind == kTickJetRb || kind == kTickAll;
  const bool rb = kind == kTickJetRb || kind == kTickRb || kind == kTickAll;
  const bool roll = kind == kTickRoll || kind == kTickAll;
  const dim3 one(1), ctl(kCtlThreads);
  hipError_t e = hipSuccess;
  const Union u = union_of(c);
  hipLaunchKernelGGL(k_tick_begin, one, ctl, 0, c.stream, c.lcs, c.H, c.lc, u);
  if (jet) {
    // Jet phase: candidates, afterburner, kept moves (locks), their application
    hipLaunchKernelGGL(k_jet_begin, one, ctl, 0, c.stream, c.lcs, c.H, c.lc, u);
    e = launch_candidates(c, c.cpart, 0, nullptr, 0, lc);
    if (e == hipSuccess) e = launch_afterburner(c, c.cpart, lc);
    if (e == hipSuccess) e = launch_select_moves(c, c.cpart, 0, lc);
    if (e == hipSuccess) e = launch_apply_moves(c, c.cpart, false, lc, kPhJet);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_jet_post, one, ctl, 0, c.stream, c.lcs, c.H, c.lc, c.st, c.k, u);
  }
  if (rb) {
    for (int r = 0; r < c.rb_slots; ++r) {
      e = launch_rebalance_round(c, c.cpart, 0, nullptr, lc);
      if (e == hipSuccess) e = launch_apply_moves(c, c.cpart, false, lc, kPhRb);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_rb_post, one, ctl, 0, c.stream, c.lcs, c.H, c.lc, c.st, c.k, u);
    }
  }
  if (jet || rb) {
    // end of the iteration, snapshot
    hipLaunchKernelGGL(k_iter_end, one, ctl, 0, c.stream, c.lcs, c.H, c.lc, c.st, c.k, c.dtrace, u);
    hipLaunchKernelGGL(k_snapshot, dim3(grid_for(c.n, 256, 2048)), dim3(kUnionTile), 0, c.stream, c.cpart, c.best, c.n,
                       lc, u);
  }
  if (roll) {
    // end of a temperature round: back to its best partition
    e = launch_diff_moves(c, c.cpart, c.best, lc);
    if (e == hipSuccess) e = launch_apply_moves(c, c.cpart, false, lc, kPhRoll);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_roll_post, one, ctl, 0, c.stream, c.lcs, c.H, c.lc, c.st, c.k, u);
  }
  return hipGetLastError();
}

}  // namespace jet
