// Internal definitions of the gfx950 Jet library: device context layout and the host-side launch
// wrappers of every kernel.  Not part of the public ABI (see include/jet.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/jet.h"

namespace jet {

constexpr int kMaxK = 128;
constexpr int kSmallNet = 64;      // nets up to this size are processed by one wave, several per wave
constexpr int kMediumNet = 1024;   // nets up to this size: one 64-thread workgroup, candidates in LDS
constexpr int kMediumSmall = 256;  // medium nets up to this size use a smaller LDS list (more per CU)
constexpr int kLaneDegree = 32;    // moves with more incident nets are applied by many threads
constexpr int kBigCap = 4096;      // larger nets: one 256-thread workgroup, up to kBigCap candidates in LDS
constexpr int kMaxSortedDegree = 8192;  // longer incidence lists are radix-sorted in global scratch
constexpr int kHubDegree = 256;        // vertices with more incident nets get a whole workgroup

// Device status block, read back by the host after each phase that needs a decision.
constexpr int kKm1Slots = 64;
// A union context refines many hypergraphs with the same k at once (the batch): vertices and nets
// are concatenated, and every per-block quantity is kept per segment hg * k + b.
constexpr int kMaxH = 4096;    // hypergraphs in one union context
constexpr int kMaxSeg = 16384; // segments (hypergraph, block) of one context

struct DevStatus {
  int64_t km1;            // current metric, maintained incrementally: km1 + sum of km1_slot
  int64_t km1_slot[kKm1Slots];  // metric changes spread over slots (no single hot address)
  int32_t n_cand;         // |M| of the last candidate pass
  int32_t n_moves;        // entries in the move list
  int32_t n_ovf;          // large nets handed to the global-scratch afterburner this iteration
  int32_t n_bigmv;        // listed moves with more than kLaneDegree incident nets
  int64_t inc_low;        // incidences scanned by the last candidate pass (non-hub / hub vertices)
  int64_t inc_hub;
  int64_t ab_inc;         // incidences of candidates scanned by the graph afterburner
  int64_t mv_inc;         // incident nets of the listed moves (sum of their degrees)
  int64_t rb_inc;         // incidences scanned by the last rebalancing gain pass
  int64_t rb_elig;        // vertices it examined in full
  int64_t rb_ent;         // order-key entries it wrote
  int32_t rb_nlist;       // vertices on the rebalancing candidate list of the round
  int32_t rb_nhub;        // hub vertices on the hub candidate list of the round
  int32_t rb_nseg;        // union: overloaded segments of the round (listed in rb_seg)
  int32_t err;            // nonzero: a kernel met an input it cannot handle (see kErr*)
  int32_t err_arg;        // detail for err
  int64_t bw[kMaxSeg];    // block weights per segment (the host reads the first H * k)
  // not read back by the host:
  int32_t bcnt[kMaxSeg];     // vertices per segment
  int32_t rb_count[kMaxSeg];   // rebalancing: eligible entries per segment
  int64_t rb_off[kMaxSeg + 1]; // rebalancing: list offsets per segment
  int64_t rb_need[kMaxSeg];    // rebalancing: weight that must leave the segment's block
  int32_t rb_kept[kMaxSeg];    // rebalancing: entries the grid-wide first selection pass kept per block
  int64_t hkm1[kMaxH];    // union: metric change per hypergraph since the last fold
  int32_t hmoves[kMaxH];  // union: moves listed per hypergraph in the current phase
  int32_t rb_seg[kMaxSeg];   // union: the overloaded segments of the round
};

// Device-resident Jet loop (Algorithm 1).  One record per context holds the state the loop's
// decisions need; small control kernels advance it between the phases of an iteration, and every
// kernel of a phase returns at once unless the record is in that phase, so one captured iteration
// can be replayed without the host looking at the device in between.
enum LoopPhase : int32_t {
  kPhJet = 0,    // candidates, afterburner, selection and application of the kept moves
  kPhRb = 1,     // rebalancing rounds (Section 4.3)
  kPhEnd = 2,    // quality key, snapshot, iteration limit
  kPhRoll = 3,   // rollback to the best partition of the temperature round
  kPhDone = 4,
  kPhAny = -1,   // a launch outside the loop (inspection calls): never gated
};

struct LoopCtl {
  int32_t phase;
  int32_t phase_mask;     // bit p set iff a hypergraph of the record is in phase p (1 << phase for one)
  int32_t stamp;          // iteration stamp: v is locked iff lockstamp[v] == stamp - 1
  int32_t tau_q;          // quantised temperature of the current round
  int32_t tau_r;          // index of the current temperature round
  int32_t round;          // consecutive iterations without strict improvement
  int32_t it;             // iterations of the current round
  int32_t lock_any;       // the last Jet phase moved a vertex (some vertex is locked)
  int32_t lock_was_any;   // lock_any as it was when the current iteration began
  int32_t n_cand, n_moved;          // the current iteration's Jet phase
  int32_t rb_rounds, rb_moved;      // the current iteration's rebalancing rounds
  int32_t improved;       // the iteration just ended improved the key: snapshot wanted
  int32_t ntrace;         // iteration records written (counted beyond the capacity too)
  int32_t iterations, rebalance_rounds, moves_executed;  // totals of the call
  int32_t ticks;          // replays that found work
  int64_t km1;            // exact metric of the current partition
  int64_t best_ovl, best_km1;
  int64_t km1_in;
  // parameters of the call
  int32_t limit, max_iters, num_tau, max_rb;
  int32_t tau_qs[8];
  int32_t rb_only;        // rebalancing rounds only (jet_rebalance)
  int32_t rb_unw;         // rebalancing order, jet_params.rb_unweighted: 0, 1 or 2
  int32_t trace_cap;
  int64_t lmax, dz, A;    // balance limit, deadzone threshold, ceil(W/k) of the hypergraph
};

// A launch of a phase returns at once unless some hypergraph of the gate record is in it.
#define JET_GATE(lc, want)                                                      \
  do {                                                                          \
    if ((lc) != nullptr && (want) >= 0 && !(((lc)->phase_mask >> (want)) & 1)) \
      return;                                                                   \
  } while (0)

__device__ __forceinline__ void set_phase(LoopCtl &r, int32_t p) {
  r.phase = p;
  r.phase_mask = 1 << p;
}

// The hypergraphs of one phase in a union context, in index order, with prefix sums of their
// vertex tiles (kUnionTile vertices; every hypergraph's vertices start on a tile) and of their
// chunks of small nets (no chunk holds nets of two hypergraphs).  The control kernels rebuild the
// lists after every change of phase; kernels of a phase walk only the listed hypergraphs' tiles.
constexpr int kUnionTile = 256;
struct ActList {
  int32_t cnt;
  int32_t hg[kMaxH + 1];
  int32_t tpref[kMaxH + 2];
  int32_t cpref[kMaxH + 2];
};
enum : int { kActJet = 0, kActRb = 1, kActRoll = 2, kActImproved = 3, kActLists = 4 };

// The hypergraphs of a union context as the kernels see them; lcs == nullptr for a context of one
// hypergraph (its record is the gate record, segments are blocks).
struct Union {
  const LoopCtl *lcs;    // per-hypergraph loop records
  const uint16_t *vhg;   // hypergraph of every vertex (padding vertices: the pseudo-hypergraph H)
  const uint16_t *nhg;   // hypergraph of every net
  const ActList *act;    // [kActLists]
  const int32_t *ht0;    // [H + 1] first tile of every hypergraph
  const int32_t *hch0;   // [H + 1] first chunk of every hypergraph
};

// Last list position i with pref[i] <= x (pref[0] = 0 <= x < pref[cnt]), found by the 64 lanes of
// a wave together: each round every lane tests one sample position and a ballot keeps the last
// one that passed, so at most two rounds (dependent loads) for the 4,096 list entries a union
// holds.  Every lane of the wave must call it with the same x.
__device__ __forceinline__ int32_t act_find(const int32_t *pref, int32_t cnt, int32_t x) {
  const int lane = __lane_id();
  int32_t lo = 0, span = cnt;  // the answer lies in [lo, lo + span)
  while (span > 1) {
    const int32_t stride = (span + 63) >> 6;
    const int32_t pos = lo + lane * stride;
    const bool ok = lane * stride < span && pref[pos] <= x;
    const unsigned long long m = __ballot(ok);
    const int32_t top = 63 - __clzll(m);  // lane 0 always passes (pref[lo] <= x)
    lo += top * stride;
    span = stride < span - top * stride ? stride : span - top * stride;
  }
  return lo;
}

// Virtual tile t of a list -> its first vertex and its hypergraph (wave-uniform t).
__device__ __forceinline__ int64_t act_tile_base(const ActList &L, const int32_t *ht0, int32_t t,
                                                 int32_t *hg_out = nullptr) {
  const int32_t i = act_find(L.tpref, L.cnt, t);
  const int32_t hg = L.hg[i];
  if (hg_out) *hg_out = hg;
  return ((int64_t)ht0[hg] + (t - L.tpref[i])) * kUnionTile;
}
// Virtual chunk c of a list -> the chunk index (wave-uniform c).
__device__ __forceinline__ int32_t act_chunk(const ActList &L, const int32_t *hch0, int32_t c) {
  const int32_t i = act_find(L.cpref, L.cnt, c);
  return hch0[L.hg[i]] + (c - L.cpref[i]);
}

// Per-family timing and algorithmic bytes accumulated on the device: a mark kernel before the
// family's launches records the wall clock, one after it adds the elapsed ticks and the bytes.
struct DevProf {
  unsigned long long t0[8];
  unsigned long long ticks[8];
  unsigned long long launches[8];
  double bytes[8];
};

// Destination of the afterburner's recomputed-gain contributions.  On small levels (few
// vertices, many incident nets each) the contributions would pile onto a few cache lines, so they
// go to `copies` private copies of the array (chosen by the contributing wave or block), summed
// into rg afterwards; otherwise copies == 1 and base is rg itself.
struct RgSink {
  int32_t *base;
  int32_t n;
  int32_t copies;
};
__device__ __forceinline__ void rg_add(const RgSink &s, uint32_t slot, int32_t v, int32_t d) {
  atomicAdd(&s.base[(size_t)(slot % (uint32_t)s.copies) * (size_t)s.n + (size_t)v], d);
}

// adds a metric change to one of the slots (chosen by the caller, e.g. from the block index)
__device__ __forceinline__ void add_km1(DevStatus *st, uint32_t slot, int64_t d) {
  if (d != 0) atomicAdd((unsigned long long *)&st->km1_slot[slot % kKm1Slots], (unsigned long long)d);
}
// union: the metric change of hypergraph hg
__device__ __forceinline__ void add_km1_hg(DevStatus *st, int32_t hg, int64_t d) {
  if (d != 0) atomicAdd((unsigned long long *)&st->hkm1[hg], (unsigned long long)d);
}

enum : int32_t {
  kErrNone = 0,
  kErrPartRange = 1,      // part[v] outside [0,k)
  kErrPinRange = 2,       // pin outside [0,n)
  kErrDupPin = 3,         // a vertex twice in one net
  kErrDegree = 4,         // vertex degree above kMaxSortedDegree
  kErrMixedOverflow = 5,  // afterburner: too many ordered events in one huge net
  kErrWeight = 6,         // weight < 1
  kErrOverflow = 7,       // a vertex's incident weight sum >= 2^31
  kErrTarget = 8,         // inspection input: candidate target outside [0,k) or equal to its block
};

// kernel families timed by the optional instrumentation
enum ProfFamily : int {
  kProfCandidates = 0,   // k_candidates (vertices with at most kHubDegree incident nets)
  kProfCandidatesHub,    // k_candidates_hub
  kProfAfterburner,      // k_ab_chunks + k_ab_nets + k_ab_overflow
  kProfSelect,           // k_select_moves
  kProfApply,            // k_apply
  kProfRbGain,           // k_rb_gain + k_rb_gain_hub
  kProfRbSelect,         // k_rb_prepare + k_rb_select
  kProfFamilies
};

// Synchronous clustering of the coarsening phase (Section 6, Algorithm 4): one rating-table slot
struct CoSlot {
  int32_t key;               // cluster label, -1 empty
  int32_t mark;              // last net that added to val
  unsigned long long val;    // heavy-edge rating, 32.32 fixed point
};

// Clustering state, allocated at the first clustering call of a context.  Between sub-rounds the
// per-vertex arrays hold -1 (tp, tt, gslot, newlab) or 0 (jw, gcnt).
struct CoState {
  bool ready = false;
  uint64_t *qnet = nullptr;          // [m] floor(w(e) 2^32 / (|e| - 1)), 0 for single-pin nets
  int64_t *deg = nullptr;            // [n] sum over incident nets of (|e| - 1)
  std::vector<int64_t> hdeg;         // host copy
  int64_t *cw = nullptr;             // [n] cluster weights of jet_coarsen's own clustering
  int32_t *tp = nullptr, *tt = nullptr;  // [n] proposals, targets after swap prevention
  int32_t *gcnt = nullptr, *gslot = nullptr, *newlab = nullptr, *flag = nullptr;  // [n]
  unsigned long long *jw = nullptr;  // [n] proposal weight per target
  int64_t cap = 0;                   // entries of the per-sub-round arrays below
  int32_t *gpos = nullptr, *gtarget = nullptr, *members = nullptr;  // [cap]
  int64_t *goff = nullptr, *gmoved = nullptr;                       // [cap + 1], [cap]
  int64_t ptab_len = 0;
  int64_t *ptab = nullptr;           // [ptab_len] rating-table offsets over list positions
  int64_t tab_slots = 0;
  CoSlot *tab = nullptr;             // [tab_slots] rating tables of one launch
  int32_t *ctr = nullptr;            // [4] device counters: groups, bad entries, clusters
  int32_t *ngroups = nullptr;        // == ctr
};

// Flow-based refinement of one block pair (Section 5), allocated at the first flow call of a
// context; the network arrays grow to the largest pair seen.  The Lawler network of the pair's
// induced subhypergraph: node 0 the contracted source terminals, node 1 the contracted sink
// terminals, nodes 2 .. NV-1 the region vertices in increasing ID, then per relevant net (two or
// more distinct endpoints) e_in = NV + 2 r and e_out = e_in + 1.  Net r owns the arc block
// [rbase[r], rbase[r] + 2 + 4 ends): e_in -> e_out and its reverse, then per endpoint j the arcs
// x -> e_in, e_in -> x, e_out -> x, x -> e_out; arc a's reverse is a ^ 1.
struct FlowState {
  // per net / per vertex, sized at first use
  int32_t *cnt_a = nullptr, *cnt_b = nullptr;  // [m] pins in block a / b
  int32_t *nexp = nullptr;      // [m] net expanded by the region search
  int32_t *ends = nullptr;      // [m] distinct endpoints
  int32_t *asize = nullptr;     // [m] arc block size (0 if not relevant)
  int32_t *rel = nullptr;       // [m] relevant
  int64_t *nbase = nullptr;     // [m + 1] arc block offsets
  int64_t *nrid = nullptr;      // [m + 1] relevant index
  int32_t *lvl = nullptr;       // [n] region search level (-1 unseen)
  int8_t *rmark = nullptr;      // [n] 1: region of a, 2: region of b
  int32_t *wtmp = nullptr;      // [n] scan input
  int64_t *wscan = nullptr;     // [n + 1] scan output
  int32_t *vnode = nullptr;     // [n] network node of a vertex of the pair, -1 otherwise
  int32_t *nvert = nullptr;     // [n] vertex of region node 2 + i
  int32_t *vcnt = nullptr;      // [n + 2] arcs per vertex node, then fill cursors
  int64_t *voffn = nullptr;     // [n + 3] vertex node adjacency offsets
  int64_t *sc = nullptr;        // [16] scalars
  int64_t *hsc = nullptr;       // [16] pinned host mirror
  // per relevant net
  int32_t *rnet = nullptr, *rends = nullptr;  // [m]
  int64_t *rbase = nullptr;                   // [m]
  // network, grown on demand
  int64_t node_cap = 0, arc_cap = 0, vadj_cap = 0;
  int32_t *head = nullptr, *tail = nullptr;   // [arcs]
  int64_t *res = nullptr;                     // [arcs] residual capacity
  int64_t *vadj = nullptr;                    // [vertex-node arc entries] first arc of each endpoint
  int32_t *h = nullptr;                       // [nodes] height
  int64_t *ex = nullptr;                      // [nodes] excess (net inflow)
  uint8_t *term = nullptr;                    // [nodes] 0 free, 1 source, 2 sink
  uint8_t *rs = nullptr, *rt = nullptr;       // [nodes] reaches from the sources / reaches the sinks
  int32_t *front[3] = {nullptr, nullptr, nullptr};  // [nodes] breadth-first frontiers (rotating)
  int32_t *fcnt = nullptr;                    // [3] their sizes
};

struct Ctx {
  hipStream_t stream = nullptr;
  int32_t n = 0, m = 0, k = 0, nw_words = 1;  // nw_words = ceil(k/64) words per mask
  int64_t p = 0;
  double eps = 0.0;
  int64_t W = 0, A = 0, lmax = 0;
  bool unit_nw = true, unit_vw = true;
  int32_t stamp = 0;  // iteration stamp for locks
  // move application: net-centric when (incident nets of the moves) * apply_divisor >= p,
  // vertex-centric otherwise (0 = always vertex-centric); environment JET_APPLY_DIVISOR overrides
  int32_t apply_divisor = 16;
  // the path the device took at the last application of each kind (Jet moves, rebalancing moves),
  // used to size the next launch of that kind
  bool wide_hint[2] = {false, false};
  bool wide_enabled = false;  // JET_OPT_APPLY_WIDE
  int32_t lane_degree = 24;   // JET_OPT_CAND_LANE_DEGREE
  int32_t cand_xcd = 1;       // JET_OPT_CAND_XCD: contiguous vertex ranges per XCD in the candidate kernels
  int32_t rb_xcd = 1;         // JET_OPT_RB_XCD: contiguous list ranges per XCD in the rebalancing gain pass
  int32_t apply_xcd = 0;      // JET_OPT_APPLY_XCD: contiguous move and chunk ranges per XCD in the application
  int32_t graph_kernels = 1;  // JET_OPT_GRAPH_KERNELS: graph-specialised afterburner when every net has two pins
  int32_t flow_workers = 4;   // JET_OPT_FLOW_WORKERS: block pairs of a matching refined at once
  int32_t sel_split_min = 1 << 18;  // JET_OPT_SEL_SPLIT_MIN
  int32_t sel_slices = 0;     // workgroups per block in the split pass; 0 = about 2,048 entries each
  int64_t grid_cap = 2048;    // JET_OPT_GRID: workgroups of the persistent (grid-stride) kernels

  // hypergraph
  int64_t *off = nullptr;    // [m+1]
  int32_t *pins = nullptr;   // [p]
  int32_t *nw = nullptr;     // [m] or null
  int32_t *vw = nullptr;     // [n] or null
  int64_t *voff = nullptr;   // [n+1] incidence offsets
  int32_t *inc = nullptr;    // [p] incident nets, ascending per vertex
  int32_t *sumw = nullptr;   // [n] omega(I(v))
  int32_t *adj = nullptr;    // [p] graphs only (every net of two pins): the other pin of net inc[q]

  // net scheduling (built once at init)
  int4 *chunks = nullptr;    // [nchunks] (first net, nets, pins, first pin) of runs of consecutive small nets
  uint8_t *pnet = nullptr;   // [p] index of the pin's net inside its chunk (chunked nets only)
  int32_t nchunks = 0;
  int32_t *mid_nets = nullptr;  // nets with kSmallNet < |e| <= kMediumNet, largest first
  int32_t nmid = 0;
  int32_t nmid_large = 0;       // leading entries of mid_nets with |e| > kMediumSmall
  int32_t *big_nets = nullptr;  // nets with |e| > kMediumNet, largest first
  int32_t nbig = 0;
  int32_t nbig_over = 0;
  int32_t *hubs = nullptr;      // vertices with more than kHubDegree incident nets
  int32_t nhubs = 0;        // leading entries of big_nets with |e| > kBigCap
  int2 *ovf_list = nullptr;     // [nbig_over] (index into big_nets, net) needing the scratch path
  int64_t *ovf_off = nullptr;   // [nbig_over + 1] scratch offsets: 2 |e| event slots per net
  unsigned long long *ovf_ka = nullptr, *ovf_kb = nullptr;  // event keys (ping-pong)
  uint32_t *ovf_ma = nullptr, *ovf_mb = nullptr;            // event block | kind<<8

  // partition state
  int32_t *phi = nullptr;     // [m*k] pin counts (when some net has more than 65,535 pins)
  uint16_t *phi16 = nullptr;  // [m*k] pin counts, 16-bit (otherwise); exactly one is allocated
  uint64_t *ns = nullptr;     // [m * 2 * nw_words]: connectivity mask words, then "exactly one pin" words
  uint64_t *rec = nullptr;    // [n] candidate record: gain (low 32), target (bits 32-39), source (40-47)
  uint32_t *inm = nullptr;    // candidate bitmask, padded to a multiple of 256 vertices
  int32_t *rg = nullptr;      // [n] recomputed gains
  int32_t rg_copies = 1;      // private copies of rg the afterburner accumulates into (small levels)
  int32_t *rgx = nullptr;     // [rg_copies * n] those copies, zero between calls
  int32_t *lockstamp = nullptr;  // [n] stamp of the iteration that last moved v
  int32_t *best = nullptr;    // [n] rollback snapshot
  int4 *moves = nullptr;      // [n] move list (v, from, to, weight)
  uint8_t *mvto = nullptr;    // [n] target of a listed move, 0xff otherwise (kept 0xff between calls)
  int32_t *bigmv = nullptr;   // [n] positions in the move list of the moves counted by n_bigmv
  int32_t *rb_list = nullptr; // [n] non-hub vertices that may move in the current rebalancing round
  int32_t *rb_slot = nullptr; // [n] the entry slot of each listed vertex (its block's region)
  int32_t *rb_hlist = nullptr; // [nhubs] hub vertices that may move in the current rebalancing round
  int32_t *rb_hacc = nullptr;  // [(k + 1) * nhubs] their connectivity and benefit sums, block-major (zero between rounds)
  int64_t *lstat = nullptr;   // [5] level statistics scratch
  float *tau_io = nullptr;    // [17] learned temperature: features in, temperature out

  // rebalancing
  uint32_t *rb_keys = nullptr;   // [n * 8] entries: 5 key words, v, target, weight
  uint32_t *rb_keys2 = nullptr;  // [n * 8] entries kept by the grid-wide first selection pass
  unsigned long long *rb_gw = nullptr;  // [kMaxK * 256] first-byte histogram per block: weights (zero between rounds)
  uint32_t *rb_gc = nullptr;            // [kMaxK * 256] and entry counts
  int32_t *rb_target = nullptr;  // [n] selected target for inspection (-1)

  // union context (batch): H hypergraphs with the same k; H == 1 otherwise
  int32_t H = 1;
  uint16_t *vhg = nullptr;       // [n] hypergraph of each vertex (union only)
  uint16_t *nhg = nullptr;       // [m] hypergraph of each net (union only)
  LoopCtl *lcs = nullptr;        // [H] per-hypergraph loop records (== lc when H == 1)
  LoopCtl *hlcs = nullptr;       // [H] pinned host mirror (== hlc when H == 1)
  std::vector<int32_t> hg_v0;    // [H+1] first vertex of each hypergraph (multiples of kUnionTile)
  std::vector<int32_t> hg_n;     // [H] its vertex count (the rest up to the next start is padding)
  std::vector<int32_t> hg_e0;    // [H+1] first net of each hypergraph
  ActList *act = nullptr;        // [kActLists] device lists of the hypergraphs per phase
  int32_t *ht0 = nullptr;        // [H+1] device: first tile of each hypergraph
  int32_t *hch0 = nullptr;       // [H+1] device: first chunk of each hypergraph
  std::vector<int64_t> hg_lmax, hg_A;  // [H] balance limit and ceil(W/k) per hypergraph
  std::vector<double> hg_eps;    // [H]
  std::vector<int64_t> hg_W;     // [H]
  // device-resident loop
  LoopCtl *lc = nullptr;         // device loop record (the gate record of a union)
  LoopCtl *hlc = nullptr;        // pinned host mirror
  int32_t *cpart = nullptr;      // [n] the partition the loop works on (copied in and out per call)
  jet_trace *dtrace = nullptr;   // device iteration records
  int32_t dtrace_cap = 0;
  hipStream_t gstream = nullptr; // stream the iteration graph is captured on
  // captured pieces of an iteration (TickKind): Jet phase + end, Jet phase + rebalancing slots +
  // end, rebalancing slots + end, rollback
  hipGraph_t graph[4] = {nullptr, nullptr, nullptr, nullptr};
  hipGraphExec_t gexec[4] = {nullptr, nullptr, nullptr, nullptr};
  bool use_graph = true;         // JET_OPT_GRAPH
  int32_t rb_slots = 4;          // JET_OPT_RB_SLOTS: rebalancing rounds per replay
  int32_t replays = 8;           // JET_OPT_REPLAYS: most replays per host poll
  int64_t polls = 0;             // host polls of the last call (diagnostic)
  int64_t replays_done = 0;      // graph replays or eager ticks of the last call
  DevProf *dprof = nullptr;      // device timing accumulators
  CoState *co = nullptr;         // clustering of the coarsening phase (allocated on first use)
  FlowState *fl = nullptr;       // flow-based refinement (allocated on first use)
  int64_t co_slots = (int64_t)1 << 28;  // JET_OPT_CO_TABLE_SLOTS: rating-table slots of one launch
  DevStatus *st = nullptr;       // device status
  DevStatus *hst = nullptr;      // pinned host mirror
  int64_t *scan_tmp = nullptr;   // scan scratch
  int64_t scan_tmp_len = 0;

  // instrumentation
  bool prof = false;
  int64_t n_low = 0, p_low = 0;  // vertices / incidences handled by the non-hub candidate kernel
  uint32_t prof_mask = 0xffffffffu;       // families marked while profiling is on
  double wall_khz = 100000.0;             // device wall clock rate

  std::string last_error;
};

// the union view of a context for the kernels
inline Union union_of(const Ctx &c) {
  return c.H > 1 ? Union{c.lcs, c.vhg, c.nhg, c.act, c.ht0, c.hch0}
                 : Union{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
}

// Mark a family's launches for the device timing when instrumentation is on (no-ops otherwise);
// the marks are gated like the family (want = its loop phase, or kPhAny outside the loop).
// bytes: static algorithmic bytes; per_inc: bytes per scanned incidence (families whose byte count
// depends on device counters add those on the device).
int prof_begin(Ctx &c, int fam, const LoopCtl *lc, int32_t want);
void prof_end(Ctx &c, int token, const LoopCtl *lc, int32_t want, double bytes, double per_inc);

// ------------------------------------------------------------------ launch wrappers
// All launch on c.stream; they return hipSuccess or the launch error.

// setup (k_setup.hip)
hipError_t launch_check_pins(Ctx &c);
hipError_t launch_degrees(Ctx &c, int32_t *deg);
hipError_t launch_exclusive_scan_i32_to_i64(Ctx &c, const int32_t *in, int64_t *out, int64_t len);
hipError_t launch_fill_incidence(Ctx &c, int64_t *cursor);
hipError_t launch_sort_incidence(Ctx &c);
hipError_t launch_check_weights(Ctx &c);

// state (k_state.hip)
hipError_t launch_check_part(Ctx &c, const int32_t *part);
hipError_t launch_build_phi(Ctx &c, const int32_t *part, int32_t *phi);
hipError_t launch_build_phi(Ctx &c, const int32_t *part, uint16_t *phi);
hipError_t launch_build_ns(Ctx &c);
hipError_t launch_block_weights(Ctx &c, const int32_t *part);
hipError_t launch_km1_from_ns(Ctx &c);
// one network evaluation on the network's stream: raw features x (device [16]) -> *tau (host);
// y is device scratch for the output
int mlp_infer_one(jet_mlp *net, const float *x, float *y, float *tau);

// cut nets, their weight, net weight total, largest net, boundary vertices (device int64[5])
hipError_t launch_level_stats(Ctx &c, int64_t *out5);

// iteration (k_iter.hip)
// Launches of the iteration's phases.  lc == nullptr: a launch outside the loop (never gated, the
// scalar arguments are used); otherwise every kernel returns at once unless lc->phase is the phase
// the launch belongs to, and the stamp, temperature and deadzone are read from lc.
hipError_t launch_candidates(Ctx &c, const int32_t *part, int32_t locked_stamp, const uint8_t *lock_bytes,
                             int32_t tau_q, const LoopCtl *lc = nullptr);
hipError_t launch_export_candidates(Ctx &c, int32_t *t, int32_t *g, uint8_t *in_m);
hipError_t launch_import_candidates(Ctx &c, const int32_t *part, const int32_t *t, const int32_t *g,
                                    const uint8_t *in_m);
// expects n_ovf == 0 (cleared by launch_candidates or launch_reset_counters)
hipError_t launch_afterburner(Ctx &c, const int32_t *part, const LoopCtl *lc = nullptr);
enum : int32_t { kResetCandidates = 1, kResetMoves = 2 };
hipError_t launch_reset_counters(Ctx &c, int32_t what, const LoopCtl *lc = nullptr, int32_t want = kPhAny);
hipError_t launch_afterburner_overflow(Ctx &c, RgSink sink, const LoopCtl *lc);  // k_ab_large.hip
hipError_t launch_select_moves(Ctx &c, const int32_t *part, int32_t stamp, const LoopCtl *lc = nullptr);
// wide: size the net-centric grids for that path (a performance hint; the device decides the path)
hipError_t launch_apply_moves(Ctx &c, int32_t *part, bool wide, const LoopCtl *lc = nullptr, int32_t want = kPhAny);
hipError_t launch_diff_moves(Ctx &c, const int32_t *part, const int32_t *target, const LoopCtl *lc = nullptr);

// rebalancing (k_rebal.hip)
hipError_t launch_rebalance_round(Ctx &c, const int32_t *part, int64_t dz, int32_t *sel_target,
                                  const LoopCtl *lc = nullptr);

// the device-resident loop (k_loop.hip)
// the launches of one piece of an iteration (kTickAll: every phase, rb_slots rebalancing rounds),
// gated by c.lc
enum TickKind : int { kTickJet = 0, kTickJetRb = 1, kTickRb = 2, kTickRoll = 3, kTickAll = 4 };
hipError_t launch_tick(Ctx &c, int kind);
// loop records for a call: the host wrote each hypergraph's parameters into c.lcs; this completes
// them from the status block (metric, overload, first phase) and sets the gate record
hipError_t launch_loop_init(Ctx &c);
hipError_t launch_fill_u32(Ctx &c, uint32_t *p, int64_t count, uint32_t value, const LoopCtl *lc, int32_t want);

// k_graph.hip: graph-specialised afterburner (every net of two pins)
hipError_t launch_build_adj(Ctx &c);
bool graph_afterburner(const Ctx &c);
hipError_t launch_ab_graph(Ctx &c, const int32_t *part, const LoopCtl *lc, int32_t want);

// k_coarsen.hip: synchronous clustering (Section 6, Algorithm 4)
hipError_t launch_co_prepare(Ctx &c);
hipError_t launch_co_init(Ctx &c, int32_t *label, int64_t *cw);
hipError_t launch_co_check(Ctx &c, const int32_t *list, int64_t len, int32_t *bad);
hipError_t launch_co_rate(Ctx &c, const int32_t *verts, int64_t a, int64_t b, int64_t base, const int32_t *label,
                          const int64_t *cw, int64_t wmax);
hipError_t launch_co_settle(Ctx &c, const int32_t *verts, int64_t len, int32_t *label, int64_t *cw, int64_t wmax,
                            int32_t *t_out);
hipError_t launch_co_count(Ctx &c, const int32_t *label, int32_t *count);

// flow-based refinement (k_flow.hip); each returns a JET_* code and sets c.last_error on failure
struct FlowPairResult {
  int64_t old_cut = 0, new_cut = 0;
  int64_t arcs = 0;  // sum over the maximum-flow iterations of the network's arcs
  int32_t iterations = 0, region_a = 0, region_b = 0, moved = 0, replaced = 0;
};
int flow_region(Ctx &c, const int32_t *part, int32_t a, int32_t b, int32_t alpha, int8_t *region);
int flow_mincut(Ctx &c, const int32_t *part, int32_t a, int32_t b, const int8_t *term, int64_t *flow,
                uint8_t *in_sr, uint8_t *in_tr);
int flow_pair(Ctx &c, int32_t *part, int32_t a, int32_t b, int32_t alpha, FlowPairResult *r);
struct FlowRefineResult {
  int64_t km1_in = 0, km1_out = 0;
  int64_t arcs = 0;
  int32_t rounds = 0, matchings = 0, pairs = 0, accepted = 0, flow_calls = 0, moved = 0;
};
int flow_refine(Ctx &c, int32_t *part, int32_t alpha, int32_t max_rounds, FlowRefineResult *r);
void flow_free(Ctx &c);

}  // namespace jet
