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

__device__ __forceinline__ int64_t dev_overload(const DevStatus *st, int32_t k, int64_t lmax) {
  int64_t worst = 0;
  for (int b = 0; b < k; ++b) worst = max(worst, st->bw[b] - lmax);
  return worst;
}

// the metric's spread slots folded into st->km1 (one thread)
__device__ __forceinline__ int64_t fold_km1(DevStatus *st) {
  int64_t s = st->km1;
  for (int i = 0; i < kKm1Slots; ++i) {
    s += st->km1_slot[i];
    st->km1_slot[i] = 0;
  }
  st->km1 = s;
  return s;
}

__global__ void k_fill_u32(uint32_t *__restrict__ p, int64_t count, uint32_t value, const LoopCtl *lc,
                           int32_t want) {
  JET_GATE(lc, want);
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

struct LoopParams {
  int32_t limit, max_iters, num_tau, max_rb, rb_only, trace_cap;
  int32_t tau_qs[8];
  int64_t lmax, dz;
};

// A call's loop record, from the state build_state left (metric in st->km1 plus slots, block weights).
__global__ void k_loop_init(LoopCtl *lc, DevStatus *st, int32_t k, LoopParams prm) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const int64_t km1 = fold_km1(st);
  const int64_t ovl = dev_overload(st, k, prm.lmax);
  const int32_t stamp = lc->stamp;  // kept across calls: lock stamps of earlier calls never match
  LoopCtl r;
  r.stamp = stamp + 2;  // nothing was moved in the iteration before the first one: no locks
  r.tau_r = 0;
  r.tau_q = prm.tau_qs[0];
  r.round = 0;
  r.it = 0;
  r.lock_any = 0;
  r.lock_was_any = 0;
  r.n_cand = r.n_moved = 0;
  r.rb_rounds = r.rb_moved = 0;
  r.improved = 0;
  r.ntrace = 0;
  r.iterations = r.rebalance_rounds = r.moves_executed = 0;
  r.ticks = 0;
  r.km1 = km1;
  r.km1_in = km1;
  r.best_ovl = ovl;
  r.best_km1 = km1;
  r.limit = prm.limit;
  r.max_iters = prm.max_iters;
  r.num_tau = prm.num_tau;
  r.max_rb = prm.max_rb;
  for (int i = 0; i < 8; ++i) r.tau_qs[i] = prm.tau_qs[i];
  r.rb_only = prm.rb_only;
  r.trace_cap = prm.trace_cap;
  r.lmax = prm.lmax;
  r.dz = prm.dz;
  if (prm.rb_only) {
    // jet_rebalance: rounds while a block is overloaded (none when the cap is 0)
    r.phase = (ovl > 0 && prm.max_rb > 0) ? kPhRb : kPhDone;
  } else {
    r.phase = kPhJet;
  }
  *lc = r;
}

// Start of a piece: the snapshot flag of the previous piece is cleared.
__global__ void k_tick_begin(LoopCtl *lc) {
  if (threadIdx.x != 0) return;
  lc->improved = 0;
  if (lc->phase != kPhDone) lc->ticks += 1;
}

// Start of a Jet phase (launched only where the phase follows): a new iteration stamp, so the
// vertices moved by the previous iteration's Jet phase (stamped stamp - 1) are the locked ones.
__global__ void k_jet_begin(LoopCtl *lc) {
  if (threadIdx.x != 0 || lc->phase != kPhJet) return;
  lc->stamp += 1;
  lc->lock_was_any = lc->lock_any;
}

// After the Jet phase's moves are applied: its counts, the locks it leaves, and whether a
// rebalancing round follows (Algorithm 1: rebalance while a block is overloaded).
__global__ void k_jet_post(LoopCtl *lc, DevStatus *st, int32_t k) {
  if (threadIdx.x != 0 || lc->phase != kPhJet) return;
  lc->km1 = fold_km1(st);
  const int32_t moved = st->n_moves;
  lc->n_cand = st->n_cand;
  lc->n_moved = moved;
  lc->lock_any = moved > 0 ? 1 : 0;
  lc->moves_executed += moved;
  lc->rb_rounds = 0;
  lc->rb_moved = 0;
  lc->phase = (dev_overload(st, k, lc->lmax) > 0 && lc->max_rb > 0) ? kPhRb : kPhEnd;
}

// After a rebalancing round's moves are applied: another round while a block is still overloaded,
// the round moved a vertex and the cap allows (Section 4.3).
__global__ void k_rb_post(LoopCtl *lc, DevStatus *st, int32_t k) {
  if (threadIdx.x != 0 || lc->phase != kPhRb) return;
  lc->km1 = fold_km1(st);
  const int32_t moved = st->n_moves;
  lc->rb_rounds += 1;
  lc->rb_moved += moved;
  if (dev_overload(st, k, lc->lmax) == 0 || lc->rb_rounds >= lc->max_rb || moved == 0) {
    if (lc->rb_only) {
      lc->rebalance_rounds += lc->rb_rounds;
      lc->phase = kPhDone;
    } else {
      lc->phase = kPhEnd;
    }
  }
}

// End of an iteration: the key (overload, metric) against the round's best (strict, lexicographic),
// the iteration record, the limit of non-improving iterations, the round's cap and the fixed point.
__global__ void k_iter_end(LoopCtl *lc, const DevStatus *st, int32_t k, jet_trace *trace) {
  if (threadIdx.x != 0 || lc->phase != kPhEnd) return;
  const int64_t ovl = dev_overload(st, k, lc->lmax), km1 = lc->km1;
  lc->it += 1;
  lc->round += 1;
  if (ovl < lc->best_ovl || (ovl == lc->best_ovl && km1 < lc->best_km1)) {
    lc->best_ovl = ovl;
    lc->best_km1 = km1;
    lc->improved = 1;
    lc->round = 0;
  }
  lc->iterations += 1;
  lc->rebalance_rounds += lc->rb_rounds;
  if (trace && lc->ntrace < lc->trace_cap) {
    jet_trace t;
    t.km1 = km1;
    t.overload = ovl;
    t.n_cand = lc->n_cand;
    t.n_moved = lc->n_moved;
    t.rb_rounds = lc->rb_rounds;
    t.rb_moved = lc->rb_moved;
    trace[lc->ntrace] = t;
  }
  lc->ntrace += 1;
  // nothing moved, nothing rebalanced and nothing was locked: the next iteration would repeat this one
  const bool fixed = lc->n_moved == 0 && lc->rb_moved == 0 && lc->lock_was_any == 0;
  lc->phase = (lc->round >= lc->limit || lc->it >= lc->max_iters || fixed) ? kPhRoll : kPhJet;
}

// The snapshot of an improving iteration (Algorithm 1's rollback point).
__global__ void k_snapshot(const int32_t *__restrict__ part, int32_t *__restrict__ best, int32_t n,
                           const LoopCtl *lc) {
  if (lc->improved == 0) return;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += (int64_t)gridDim.x * blockDim.x)
    best[v] = part[v];
}

// After the rollback's moves are applied: the next temperature round starts from the round's
// best partition with no locks, or the loop is done.
__global__ void k_roll_post(LoopCtl *lc, DevStatus *st, int32_t k) {
  if (threadIdx.x != 0 || lc->phase != kPhRoll) return;
  const int64_t km1 = fold_km1(st);
  lc->km1 = km1;
  lc->tau_r += 1;
  if (lc->tau_r >= lc->num_tau) {
    lc->phase = kPhDone;
    return;
  }
  lc->tau_q = lc->tau_qs[lc->tau_r];
  lc->stamp += 2;  // the round's first iteration sees no lock
  lc->round = 0;
  lc->it = 0;
  lc->lock_any = 0;
  lc->best_ovl = dev_overload(st, k, lc->lmax);
  lc->best_km1 = km1;
  lc->phase = kPhJet;
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

hipError_t launch_loop_init(Ctx &c, const jet_params &prm, int32_t rb_only, int64_t dz, int32_t trace_cap) {
  LoopParams lp;
  lp.limit = prm.limit;
  lp.max_iters = prm.max_iters;
  lp.num_tau = prm.num_tau;
  lp.max_rb = prm.max_rebalance_rounds;
  lp.rb_only = rb_only;
  lp.trace_cap = trace_cap;
  for (int i = 0; i < 8; ++i)
    lp.tau_qs[i] = i < prm.num_tau ? (int32_t)std::floor((double)prm.tau[i] * 65536.0 + 0.5) : 0;
  lp.lmax = c.lmax;
  lp.dz = dz;
  hipLaunchKernelGGL(k_loop_init, dim3(1), dim3(64), 0, c.stream, c.lc, c.st, c.k, lp);
  return hipGetLastError();
}

hipError_t launch_tick(Ctx &c, int kind) {
  const LoopCtl *lc = c.lc;
  const bool jet = kind == kTickJet || kind == kTickJetRb || kind == kTickAll;
  const bool rb = kind == kTickJetRb || kind == kTickRb || kind == kTickAll;
  const bool roll = kind == kTickRoll || kind == kTickAll;
  hipError_t e = hipSuccess;
  hipLaunchKernelGGL(k_tick_begin, dim3(1), dim3(64), 0, c.stream, c.lc);
  if (jet) {
    // Jet phase: candidates, afterburner, kept moves (locks), their application
    hipLaunchKernelGGL(k_jet_begin, dim3(1), dim3(64), 0, c.stream, c.lc);
    e = launch_candidates(c, c.cpart, 0, nullptr, 0, lc);
    if (e == hipSuccess) e = launch_afterburner(c, c.cpart, lc);
    if (e == hipSuccess) e = launch_select_moves(c, c.cpart, 0, lc);
    if (e == hipSuccess) e = launch_apply_moves(c, c.cpart, false, lc, kPhJet);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_jet_post, dim3(1), dim3(64), 0, c.stream, c.lc, c.st, c.k);
  }
  if (rb) {
    for (int r = 0; r < c.rb_slots; ++r) {
      e = launch_rebalance_round(c, c.cpart, 0, nullptr, lc);
      if (e == hipSuccess) e = launch_apply_moves(c, c.cpart, false, lc, kPhRb);
      if (e != hipSuccess) return e;
      hipLaunchKernelGGL(k_rb_post, dim3(1), dim3(64), 0, c.stream, c.lc, c.st, c.k);
    }
  }
  if (jet || rb) {
    // end of the iteration, snapshot
    hipLaunchKernelGGL(k_iter_end, dim3(1), dim3(64), 0, c.stream, c.lc, c.st, c.k, c.dtrace);
    hipLaunchKernelGGL(k_snapshot, dim3(grid_for(c.n, 256, 2048)), dim3(256), 0, c.stream, c.cpart, c.best, c.n, lc);
  }
  if (roll) {
    // end of a temperature round: back to its best partition
    e = launch_diff_moves(c, c.cpart, c.best, lc);
    if (e == hipSuccess) e = launch_apply_moves(c, c.cpart, false, lc, kPhRoll);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_roll_post, dim3(1), dim3(64), 0, c.stream, c.lc, c.st, c.k);
  }
  return hipGetLastError();
}

}  // namespace jet
